// Device helpers shared by the HIP kernels of libgsim (templated on the scalar
// type): 3-vectors, scalar math overloads, global loads and stores through
// address space 1, and the ground contact model with its adjoint.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace gsim {
namespace {

// ------------------------------------------------------------------ math ---
template <typename T>
struct V3 {
    T x, y, z;
};

template <typename T> __device__ __forceinline__ V3<T> mk3(T x, T y, T z) { return V3<T>{x, y, z}; }
template <typename T> __device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
template <typename T> __device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
template <typename T> __device__ __forceinline__ V3<T> operator-(V3<T> a) { return mk3(-a.x, -a.y, -a.z); }
template <typename T> __device__ __forceinline__ V3<T> operator*(V3<T> a, T s) { return mk3(a.x * s, a.y * s, a.z * s); }
template <typename T> __device__ __forceinline__ V3<T>& operator+=(V3<T>& a, V3<T> b) { a = a + b; return a; }
template <typename T> __device__ __forceinline__ V3<T>& operator-=(V3<T>& a, V3<T> b) { a = a - b; return a; }
template <typename T> __device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T> __device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
    return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <typename T> __device__ __forceinline__ V3<T> zero3() { return mk3(T(0), T(0), T(0)); }

__device__ __forceinline__ float gsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double gsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float gsin(float a) { return sinf(a); }
__device__ __forceinline__ double gsin(double a) { return sin(a); }
__device__ __forceinline__ float gcos(float a) { return cosf(a); }
__device__ __forceinline__ double gcos(double a) { return cos(a); }
__device__ __forceinline__ float gabs(float a) { return fabsf(a); }
__device__ __forceinline__ double gabs(double a) { return fabs(a); }
__device__ __forceinline__ float gatan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double gatan2(double y, double x) { return atan2(y, x); }

// Device-memory accesses through address space 1: pointers read out of the
// launch tables are generic, and generic (flat) loads both count against the
// LDS wait counter and may alias LDS, which would order every record load
// before the next LDS barrier.  Global loads do neither.
template <typename T> __device__ __forceinline__ T gld(const T* p, int64_t i) {
    return ((const __attribute__((address_space(1))) T*)p)[i];
}
template <typename T> __device__ __forceinline__ void gst(T* p, int64_t i, T v) {
    ((__attribute__((address_space(1))) T*)p)[i] = v;
}
template <typename T> __device__ __forceinline__ V3<T> ld3(const T* __restrict__ p, int64_t n, int64_t i) {
    return mk3(gld(p, i), gld(p, n + i), gld(p, 2 * n + i));
}
template <typename T> __device__ __forceinline__ void st3(T* __restrict__ p, int64_t n, int64_t i, V3<T> a) {
    gst(p, i, a.x);
    gst(p, n + i, a.y);
    gst(p, 2 * n + i, a.z);
}

// ------------------------------------------------------------- contact ---
// gap = n.x - d; C = -gap when gap < 0; lambda_n = k_e C + k_d Cdot, Cdot = -n.v;
// f_n = lambda_n n; u_t = v - (n.v) n; stick if k_f |u_t| <= mu_f |lambda_n|:
// f_f = -k_f u_t; otherwise f_f = -mu_f |lambda_n| u_t / |u_t|.
// The deformable kernels pass the gap itself (the rest gap of the particle plus
// n.u for its displacement u, so that no absolute coordinate is rounded); the
// rigid kernels pass a world point through the overloads below.
template <typename T>
__device__ __forceinline__ V3<T> contact_force_gap(T gap, V3<T> v, const T pl[4], const T c[4]) {
    const V3<T> n = mk3(pl[0], pl[1], pl[2]);
    if (!(gap < T(0))) return zero3<T>();
    const T C = -gap;
    const T vn = dot(n, v);
    const T lam = c[0] * C - c[1] * vn;
    const V3<T> ut = v - n * vn;
    const T s = gsqrt(dot(ut, ut));
    const T lim = c[3] * (lam < T(0) ? -lam : lam);
    V3<T> ff;
    if (c[2] * s <= lim) ff = ut * (-c[2]);
    else ff = ut * (-lim / s);
    return n * lam + ff;
}

// Adjoint of contact_force_gap for the force adjoint fb: adds to xb (through
// d gap / dx = n), vb and the contact-parameter gradients gc (k_e, k_d, k_f,
// mu_f); returns the force.
template <typename T>
__device__ __forceinline__ V3<T> contact_adjoint_gap(T gap, V3<T> v, const T pl[4], const T c[4], V3<T> fb, V3<T>& xb,
                                                     V3<T>& vb, T gc[4]) {
    const V3<T> n = mk3(pl[0], pl[1], pl[2]);
    if (!(gap < T(0))) return zero3<T>();
    const T C = -gap;
    const T vn = dot(n, v);
    const T lam = c[0] * C - c[1] * vn;
    const V3<T> ut = v - n * vn;
    const T s = gsqrt(dot(ut, ut));
    const T sg = lam < T(0) ? T(-1) : T(1);
    const T lim = c[3] * lam * sg;
    T lamb = dot(fb, n);
    V3<T> utb;
    V3<T> ff;
    if (c[2] * s <= lim) {
        ff = ut * (-c[2]);
        utb = fb * (-c[2]);
        gc[2] -= dot(ut, fb);
    } else {
        const T is = T(1) / s;
        const V3<T> th = ut * is;
        ff = th * (-lim);
        const T limb = -dot(th, fb);
        const V3<T> thb = fb * (-lim);
        utb = (thb - th * dot(th, thb)) * is;
        gc[3] += lam * sg * limb;
        lamb += c[3] * sg * limb;
    }
    vb += utb - n * dot(n, utb);
    gc[0] += C * lamb;
    gc[1] -= vn * lamb;
    xb -= n * (c[0] * lamb);
    vb -= n * (c[1] * lamb);
    return n * lam + ff;
}

template <typename T>
__device__ __forceinline__ V3<T> contact_force(V3<T> x, V3<T> v, const T pl[4], const T c[4]) {
    return contact_force_gap(dot(mk3(pl[0], pl[1], pl[2]), x) - pl[3], v, pl, c);
}
template <typename T>
__device__ __forceinline__ V3<T> contact_adjoint(V3<T> x, V3<T> v, const T pl[4], const T c[4], V3<T> fb, V3<T>& xb,
                                                 V3<T>& vb, T gc[4]) {
    return contact_adjoint_gap(dot(mk3(pl[0], pl[1], pl[2]), x) - pl[3], v, pl, c, fb, xb, vb, gc);
}

}  // namespace
}  // namespace gsim
