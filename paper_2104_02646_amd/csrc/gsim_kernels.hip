// HIP kernels of the differentiable simulation step for CDNA4 (gfx950).
//
// One step is two passes (Sec. 2.1 step relation; App. A.2 semi-implicit Euler):
//   element pass   one thread per element: gathers its corner positions, evaluates
//                  the element force (tet / membrane / bending, App. A.1) and
//                  writes each corner's 4-vector into that corner's gather slot;
//   particle pass  one thread per particle: sums its slots in a fixed order (no
//                  atomics, bitwise deterministic; slots are interleaved per
//                  64-particle slice so each gather load is coalesced), adds
//                  ground contact and
//                  friction (App. A.1 "Contact", App. B.2) and integrates.
// The adjoint step (App. A, App. A.2 Jacobians) has the same two passes in the
// same layout: the element pass applies the hand-written reverse mode of each
// element force to the corner adjoint forces fbar = dt w (vbar+ + dt xbar+),
// the particle pass gathers those contributions, applies the contact adjoint and
// closes the integrator's adjoint.  Element-owned parameter gradients (mu,
// lambda, k) are accumulated by their element's thread; per-body contact
// gradients go through a per-tile partial buffer reduced in fixed order.
//
// All state arrays are SoA [3][n]; element records SoA over elements; partial slots
// AoS: forward [nslot][3] (12 bytes), adjoint [nslot][4] (one 16-byte FP32 access).  The kernels are
// templated on the scalar type: float for production, double for checking the
// algorithm against the FP64 oracle independently of FP32 rounding.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "gsim_device.h"
#include "gsim_internal.h"

namespace gsim {
namespace {

// Slots are 4-vectors accessed as one 16-byte (FP32) or two 16-byte (FP64)
// global accesses (clang vector types: they can live in address space 1).
typedef float gf4 __attribute__((ext_vector_type(4)));
typedef double gd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_slot(float* s, int64_t k, float a, float b, float c, float d) {
    gf4 v = {a, b, c, d};
    ((__attribute__((address_space(1))) gf4*)(s + 4 * k))[0] = v;
}
__device__ __forceinline__ void st_slot(double* s, int64_t k, double a, double b, double c, double d) {
    __attribute__((address_space(1))) gd2* p = (__attribute__((address_space(1))) gd2*)(s + 4 * k);
    gd2 v0 = {a, b}, v1 = {c, d};
    p[0] = v0;
    p[1] = v1;
}
__device__ __forceinline__ void ld_slot(const float* s, int64_t k, float& a, float& b, float& c, float& d) {
    const gf4 q = ((const __attribute__((address_space(1))) gf4*)(s + 4 * k))[0];
    a = q.x; b = q.y; c = q.z; d = q.w;
}
__device__ __forceinline__ void ld_slot(const double* s, int64_t k, double& a, double& b, double& c, double& d) {
    const __attribute__((address_space(1))) gd2* p = (const __attribute__((address_space(1))) gd2*)(s + 4 * k);
    const gd2 q0 = p[0], q1 = p[1];
    a = q0.x; b = q0.y; c = q1.x; d = q1.y;
}

// Forward partials are 3-vectors, 12 (FP32) or 24 (FP64) bytes a slot (the adjoint's
// carry a fourth value and keep 4-vector slots of their own).
__device__ __forceinline__ void st_fslot(float* s, int64_t k, float a, float b, float c) {
    __attribute__((address_space(1))) float* p = (__attribute__((address_space(1))) float*)(s + 3 * k);
    p[0] = a;
    p[1] = b;
    p[2] = c;
}
__device__ __forceinline__ void st_fslot(double* s, int64_t k, double a, double b, double c) {
    __attribute__((address_space(1))) double* p = (__attribute__((address_space(1))) double*)(s + 3 * k);
    p[0] = a;
    p[1] = b;
    p[2] = c;
}
template <typename T>
__device__ __forceinline__ V3<T> ld_fslot(const T* s, int64_t k) {
    const __attribute__((address_space(1))) T* p = (const __attribute__((address_space(1))) T*)(s + 3 * k);
    return mk3(p[0], p[1], p[2]);
}

// w = 1/m, 0 for pinned particles.  The mass is loaded whether or not the particle
// is pinned (the mass array covers every particle), so its load does not wait for
// the pin flag.
template <typename T> __device__ __forceinline__ T inv_mass(const ModelDev<T>& M, const StepDev<T>& S, int64_t i) {
    const bool pin = gld(M.pinned, i) != 0;
    const T m = gld(S.mass, i);
    return pin ? T(0) : T(1) / m;
}

// State positions are displacements u from the rest positions, except where a
// launch record marks its input (x_abs) or output (xo_abs) as absolute positions
// (the caller's states at the ends of a call).  Tets use u itself; triangles,
// hinges and lift/drag take the absolute position X + u.
template <typename T>
__device__ __forceinline__ V3<T> load_disp(const ModelDev<T>& M, const T* x, int32_t abs, int64_t i) {
    const V3<T> a = ld3(x, M.np, i);
    return abs ? a - ld3(M.rest, M.np, i) : a;
}
template <typename T>
__device__ __forceinline__ V3<T> load_pos(const ModelDev<T>& M, const T* x, int32_t abs, int64_t i) {
    const V3<T> a = ld3(x, M.np, i);
    return abs ? a : ld3(M.rest, M.np, i) + a;
}
// Ground gap of particle i at displacement u: its rest gap n.X - d plus n.u.
template <typename T>
__device__ __forceinline__ T gap_of(T rgap, const T pl[4], V3<T> u) {
    return rgap + dot(mk3(pl[0], pl[1], pl[2]), u);
}

// Body status words (ModelDev::bflag): a plain store of 1, so any number of threads
// may raise the same flag in any order.
__device__ __forceinline__ bool finite3(float a, float b, float c) { return isfinite(a + b + c); }
__device__ __forceinline__ bool finite3(double a, double b, double c) { return isfinite(a + b + c); }
template <typename T>
__device__ __forceinline__ bool finite_pair(V3<T> a, V3<T> b) {
    return finite3(a.x, a.y, a.z) && finite3(b.x, b.y, b.z);
}
template <typename T>
__device__ __forceinline__ void raise_flag(const ModelDev<T>& M, int body, int which) {
    gst(M.bflag, 2 * (int64_t)body + which, int32_t(1));
}

// Sum, in slot order, of a particle's deg partial slots at base, base + 64, ...
// (xyz into f, w into d).  The first SLOT_BATCH slots are fetched before any is
// used, so their loads overlap instead of waiting one after another; the sum order
// is the same as a plain loop's.
constexpr int SLOT_BATCH = 4;
template <typename T>
__device__ __forceinline__ void sum_slots(const T* slots, int64_t base, int32_t deg, V3<T>& f, T& d) {
    T q[SLOT_BATCH][4];
#pragma unroll
    for (int k = 0; k < SLOT_BATCH; ++k)
        if (k < deg) ld_slot(slots, base + 64 * k, q[k][0], q[k][1], q[k][2], q[k][3]);
#pragma unroll
    for (int k = 0; k < SLOT_BATCH; ++k)
        if (k < deg) {
            f += mk3(q[k][0], q[k][1], q[k][2]);
            d += q[k][3];
        }
    for (int32_t k = SLOT_BATCH; k < deg; ++k) {
        T a, b, c, e;
        ld_slot(slots, base + 64 * k, a, b, c, e);
        f += mk3(a, b, c);
        d += e;
    }
}

// Sum, in slot order, of a particle's deg forward partials at base, base + 64, ...
// (the first SLOT_BATCH fetched before any is used, as in sum_slots).
template <typename T>
__device__ __forceinline__ void sum_fslots(const T* slots, int64_t base, int32_t deg, V3<T>& f) {
    V3<T> q[SLOT_BATCH];
#pragma unroll
    for (int k = 0; k < SLOT_BATCH; ++k)
        if (k < deg) q[k] = ld_fslot(slots, base + 64 * k);
#pragma unroll
    for (int k = 0; k < SLOT_BATCH; ++k)
        if (k < deg) f += q[k];
    for (int32_t k = SLOT_BATCH; k < deg; ++k) f += ld_fslot(slots, base + 64 * k);
}

// ---------------------------------------------------------- tet (NH) ---
// The state holds each particle's displacement u from its rest position, so the
// displacement gradient H = F - I = [u1-u0, u2-u0, u3-u0] Dm^-1 comes straight from
// differences of small numbers, and every term that vanishes at rest is formed
// from H without subtracting O(1) quantities:
//   s      = Ic - 3 = 2 tr H + |H|^2,              1 - 1/(Ic+1) = 3/4 + s / (4 (4 + s)),
//   J - 1  = tr H + tr(cof H) + det H               (characteristic polynomial of H),
//   cof F  = (1 + tr H) I - H^T + cof H,
//   Pmu    = (1 - 1/(Ic+1)) F - 3/4 cof F = 3/4 (H + H^T - tr H I - cof H) + s/(4(4+s)) F.
// With alpha = 1 + 3 mu/(4 lambda) + a the stress is
//   P = mu (1 - 1/(Ic+1)) F + lambda (J - alpha) cof F = mu Pmu + lambda (J - 1 - a) cof F,
// whose parameter partials are dP/dmu = Pmu, dP/dlambda = (J - 1 - a) cof F and
// dP/da = -lambda cof F.  Corner forces [f1 f2 f3] = -V P Dm^-T, f0 = -(f1 + f2 + f3).
template <typename T>
struct TetKin {
    V3<T> F[3];    // columns of F = I + H
    V3<T> C[3];    // columns of cof F
    V3<T> Pmu[3];  // columns of dP/dmu
    T s, J1;       // Ic - 3, J - 1
};

template <typename T>
__device__ __forceinline__ void tet_kin(const V3<T> u[4], const T D[9], TetKin<T>& k) {
    const V3<T> d0 = u[1] - u[0], d1 = u[2] - u[0], d2 = u[3] - u[0];
    V3<T> H[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) H[j] = d0 * D[j] + d1 * D[3 + j] + d2 * D[6 + j];
    // row j of H, as a vector (column j of H^T)
    const V3<T> R[3] = {mk3(H[0].x, H[1].x, H[2].x), mk3(H[0].y, H[1].y, H[2].y), mk3(H[0].z, H[1].z, H[2].z)};
    const T tr = H[0].x + H[1].y + H[2].z;
    const V3<T> cH[3] = {cross(H[1], H[2]), cross(H[2], H[0]), cross(H[0], H[1])};
    const T detH = dot(H[0], cH[0]);
    const T tcH = cH[0].x + cH[1].y + cH[2].z;
    k.s = T(2) * tr + (dot(H[0], H[0]) + dot(H[1], H[1]) + dot(H[2], H[2]));
    k.J1 = tr + tcH + detH;
    const T q = k.s / (T(4) * (T(4) + k.s));
    const V3<T> E[3] = {mk3(T(1), T(0), T(0)), mk3(T(0), T(1), T(0)), mk3(T(0), T(0), T(1))};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        k.F[j] = H[j] + E[j];
        k.C[j] = E[j] * (T(1) + tr) - R[j] + cH[j];
        k.Pmu[j] = (H[j] + R[j] - E[j] * tr - cH[j]) * T(0.75) + k.F[j] * q;
    }
}

template <typename T>
__device__ __forceinline__ void tet_force(const V3<T> u[4], const T D[9], T V, T mu, T lam, T act, V3<T> f[4],
                                          T& J1) {
    TetKin<T> k;
    tet_kin(u, D, k);
    J1 = k.J1;
    const T B = lam * (k.J1 - act);
    V3<T> P[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) P[j] = k.Pmu[j] * mu + k.C[j] * B;
    f[0] = zero3<T>();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        f[i + 1] = (P[0] * D[3 * i] + P[1] * D[3 * i + 1] + P[2] * D[3 * i + 2]) * (-V);
        f[0] -= f[i + 1];
    }
}

// Reverse mode of tet_force for corner adjoints fb: displacement (= position)
// adjoints xb (the transpose of df/dx applied to fb), d/dmu, d/dlambda and d/da
// of <fb, f>; also returns the forces themselves (for the mass gradient).  The
// position adjoint differentiates P = A F + B cof F with A = mu (1 - 1/(Ic+1)) and
// B = lambda (J - alpha) (both O(mu) at rest, so no cancellation reaches it).
template <typename T>
__device__ __forceinline__ void tet_adjoint(const V3<T> u[4], const T D[9], T V, T mu, T lam, T act, const V3<T> fb[4],
                                            V3<T> f[4], V3<T> xb[4], T& gmu, T& glam, T& gact) {
    TetKin<T> k;
    tet_kin(u, D, k);
    const V3<T>* F = k.F;
    const V3<T>* C = k.C;
    const T Ja = k.J1 - act;
    V3<T> P[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) P[j] = k.Pmu[j] * mu + C[j] * (lam * Ja);
    f[0] = zero3<T>();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        f[i + 1] = (P[0] * D[3 * i] + P[1] * D[3 * i + 1] + P[2] * D[3 * i + 2]) * (-V);
        f[0] -= f[i + 1];
    }
    // f_{i+1} = G_i, f_0 = -sum G_i  =>  Gbar_i = fb_{i+1} - fb_0
    const V3<T> Hb[3] = {fb[1] - fb[0], fb[2] - fb[0], fb[3] - fb[0]};
    V3<T> Pb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) Pb[j] = (Hb[0] * D[j] + Hb[1] * D[3 + j] + Hb[2] * D[6 + j]) * (-V);
    const T Ab = dot(Pb[0], F[0]) + dot(Pb[1], F[1]) + dot(Pb[2], F[2]);
    const T Bb = dot(Pb[0], C[0]) + dot(Pb[1], C[1]) + dot(Pb[2], C[2]);
    gmu = dot(Pb[0], k.Pmu[0]) + dot(Pb[1], k.Pmu[1]) + dot(Pb[2], k.Pmu[2]);
    glam = Ja * Bb;
    gact = -lam * Bb;
    const T ip = T(1) / (T(4) + k.s);             // 1/(Ic+1)
    const T A = mu * (T(0.75) + k.s * T(0.25) * ip);  // mu (1 - 1/(Ic+1))
    const T B = lam * Ja - T(0.75) * mu;          // lambda (J - alpha)
    const T Icb = Ab * mu * ip * ip;
    const T Jb = Bb * lam;
    V3<T> Fb[3], Cb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Fb[j] = Pb[j] * A + C[j] * Jb + F[j] * (T(2) * Icb);
        Cb[j] = Pb[j] * B;
    }
    // C0 = F1 x F2, C1 = F2 x F0, C2 = F0 x F1;  (a x b) adjoint: abar = b x cbar, bbar = cbar x a
    Fb[1] += cross(F[2], Cb[0]);
    Fb[2] += cross(Cb[0], F[1]);
    Fb[2] += cross(F[0], Cb[1]);
    Fb[0] += cross(Cb[1], F[2]);
    Fb[0] += cross(F[1], Cb[2]);
    Fb[1] += cross(Cb[2], F[0]);
#pragma unroll
    for (int c = 0; c < 3; ++c) xb[c + 1] = Fb[0] * D[3 * c] + Fb[1] * D[3 * c + 1] + Fb[2] * D[3 * c + 2];
    xb[0] = -(xb[1] + xb[2] + xb[3]);
}

// --------------------------------------------------- membrane triangle ---
// F (3x2) = [x1-x0, x2-x0] Dm^-1; Ic = |F0|^2+|F1|^2; J = |F0 x F1|; n = (F0 x F1)/J;
// dJ/dF = [F1 x n, n x F0]; mu = lambda = k, alpha2 = 5/3;
// P = k (1 - 1/(Ic+1)) F + k (J - 5/3) dJ/dF; [f1 f2] = -A P Dm^-T; f0 = -(f1+f2).
template <typename T>
__device__ __forceinline__ void tri_force(const V3<T> x[3], const T D[4], T area, T k, V3<T> f[3]) {
    const V3<T> d0 = x[1] - x[0], d1 = x[2] - x[0];
    const V3<T> F0 = d0 * D[0] + d1 * D[2];
    const V3<T> F1 = d0 * D[1] + d1 * D[3];
    const T Ic = dot(F0, F0) + dot(F1, F1);
    const V3<T> c = cross(F0, F1);
    const T J = gsqrt(dot(c, c));
    const V3<T> n = c * (T(1) / J);
    const V3<T> G0 = cross(F1, n), G1 = cross(n, F0);
    const T A = k * (T(1) - T(1) / (Ic + T(1)));
    const T B = k * (J - T(5) / T(3));
    const V3<T> P0 = F0 * A + G0 * B, P1 = F1 * A + G1 * B;
    f[1] = (P0 * D[0] + P1 * D[1]) * (-area);
    f[2] = (P0 * D[2] + P1 * D[3]) * (-area);
    f[0] = -(f[1] + f[2]);
}

template <typename T>
__device__ __forceinline__ void tri_adjoint(const V3<T> x[3], const T D[4], T area, T k, const V3<T> fb[3], V3<T> f[3],
                                            V3<T> xb[3], T& gk) {
    const V3<T> d0 = x[1] - x[0], d1 = x[2] - x[0];
    const V3<T> F0 = d0 * D[0] + d1 * D[2];
    const V3<T> F1 = d0 * D[1] + d1 * D[3];
    const T Ic = dot(F0, F0) + dot(F1, F1);
    const V3<T> c = cross(F0, F1);
    const T J = gsqrt(dot(c, c));
    const T iJ = T(1) / J;
    const V3<T> n = c * iJ;
    const V3<T> G0 = cross(F1, n), G1 = cross(n, F0);
    const T ip = T(1) / (Ic + T(1));
    const T A = k * (T(1) - ip);
    const T B = k * (J - T(5) / T(3));
    const V3<T> P0 = F0 * A + G0 * B, P1 = F1 * A + G1 * B;
    f[1] = (P0 * D[0] + P1 * D[1]) * (-area);
    f[2] = (P0 * D[2] + P1 * D[3]) * (-area);
    f[0] = -(f[1] + f[2]);
    const V3<T> Hb0 = fb[1] - fb[0], Hb1 = fb[2] - fb[0];
    const V3<T> Pb0 = (Hb0 * D[0] + Hb1 * D[2]) * (-area);
    const V3<T> Pb1 = (Hb0 * D[1] + Hb1 * D[3]) * (-area);
    const T Ab = dot(Pb0, F0) + dot(Pb1, F1);
    const T Bb = dot(Pb0, G0) + dot(Pb1, G1);
    gk = (T(1) - ip) * Ab + (J - T(5) / T(3)) * Bb;
    const T Icb = Ab * k * ip * ip;
    const T Jb = Bb * k;
    V3<T> Fb0 = Pb0 * A + F0 * (T(2) * Icb);
    V3<T> Fb1 = Pb1 * A + F1 * (T(2) * Icb);
    const V3<T> Gb0 = Pb0 * B, Gb1 = Pb1 * B;
    // G0 = F1 x n, G1 = n x F0
    Fb1 += cross(n, Gb0);
    V3<T> nb = cross(Gb0, F1);
    nb += cross(F0, Gb1);
    Fb0 += cross(Gb1, n);
    // n = c / |c|, J = |c|
    const V3<T> cb = (nb - n * dot(n, nb)) * iJ + n * Jb;
    // c = F0 x F1
    Fb0 += cross(F1, cb);
    Fb1 += cross(cb, F0);
    xb[1] = Fb0 * D[0] + Fb1 * D[1];
    xb[2] = Fb0 * D[2] + Fb1 * D[3];
    xb[0] = -(xb[1] + xb[2]);
}

// ------------------------------------------------------------- bending ---
// Wings x0, x1; edge E = x3 - x2; N1 = (x0-x2)x(x0-x3), N2 = (x1-x3)x(x1-x2).
// Bridson's directions u0 = |E| N1/|N1|^2, u1 = |E| N2/|N2|^2,
// u2 = s0 N1/|N1|^2 + s1 N2/|N2|^2, u3 = -(s2 N1/|N1|^2 + s3 N2/|N2|^2) with
// s0 = (x0-x3).E/|E|, s1 = (x1-x3).E/|E|, s2 = (x0-x2).E/|E|, s3 = (x1-x2).E/|E|;
// they equal d phi/dx_i for phi = atan2(-((N1 x N2).E)/|E|, N1.N2).
// f_i = -k_b |E|^2/(|N1|+|N2|) sin((phi - phi0)/2) u_i.
template <typename T>
struct HingeGeo {
    V3<T> E, N1, N2, a1, a2, Eh, u[4];
    T el, n1, n2, s[4], phi;
};

template <typename T>
__device__ __forceinline__ void hinge_geo(const V3<T> x[4], HingeGeo<T>& h) {
    h.E = x[3] - x[2];
    h.N1 = cross(x[0] - x[2], x[0] - x[3]);
    h.N2 = cross(x[1] - x[3], x[1] - x[2]);
    h.el = gsqrt(dot(h.E, h.E));
    const T n1sq = dot(h.N1, h.N1), n2sq = dot(h.N2, h.N2);
    h.n1 = gsqrt(n1sq);
    h.n2 = gsqrt(n2sq);
    h.a1 = h.N1 * (T(1) / n1sq);
    h.a2 = h.N2 * (T(1) / n2sq);
    h.Eh = h.E * (T(1) / h.el);
    h.s[0] = dot(x[0] - x[3], h.Eh);
    h.s[1] = dot(x[1] - x[3], h.Eh);
    h.s[2] = dot(x[0] - x[2], h.Eh);
    h.s[3] = dot(x[1] - x[2], h.Eh);
    h.u[0] = h.a1 * h.el;
    h.u[1] = h.a2 * h.el;
    h.u[2] = h.a1 * h.s[0] + h.a2 * h.s[1];
    h.u[3] = -(h.a1 * h.s[2] + h.a2 * h.s[3]);
    h.phi = gatan2(-dot(cross(h.N1, h.N2), h.Eh), dot(h.N1, h.N2));
}

// Bending force with actuation a: the half-angle term is sin((phi - phi0)/2 + a).
template <typename T>
__device__ __forceinline__ void hinge_force(const V3<T> x[4], T phi0, T kb, T act, V3<T> f[4]) {
    HingeGeo<T> h;
    hinge_geo(x, h);
    const T sc = h.el * h.el / (h.n1 + h.n2);
    const T mag = -kb * sc * gsin(T(0.5) * (h.phi - phi0) + act);
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = h.u[i] * mag;
}

// Reverse mode of hinge_force: position adjoints xb and d/da of <fb, f> (gact).
template <typename T>
__device__ __forceinline__ void hinge_adjoint(const V3<T> x[4], T phi0, T kb, T act, const V3<T> fb[4], V3<T> f[4],
                                              V3<T> xb[4], T& gact) {
    HingeGeo<T> h;
    hinge_geo(x, h);
    const T q = h.n1 + h.n2;
    const T sc = h.el * h.el / q;
    const T psi = T(0.5) * (h.phi - phi0) + act;
    const T sn = gsin(psi), cs = gcos(psi);
    const T mag = -kb * sc * sn;
    T magb = T(0);
    V3<T> ub[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[i] = h.u[i] * mag;
        ub[i] = fb[i] * mag;
        magb += dot(fb[i], h.u[i]);
    }
    const T scb = -kb * sn * magb;
    const T psib = -kb * sc * cs * magb;
    const T phib = T(0.5) * psib;
    gact = psib;
    // phi: its gradient is u (exact identity of the dihedral angle)
#pragma unroll
    for (int i = 0; i < 4; ++i) xb[i] = h.u[i] * phib;
    // sc = el^2 / (|N1| + |N2|)
    T elb = scb * T(2) * h.el / q;
    const T qb = -scb * sc / q;
    V3<T> N1b = h.N1 * (qb / h.n1);
    V3<T> N2b = h.N2 * (qb / h.n2);
    // u0 = el a1, u1 = el a2, u2 = s0 a1 + s1 a2, u3 = -(s2 a1 + s3 a2)
    elb += dot(ub[0], h.a1) + dot(ub[1], h.a2);
    V3<T> a1b = ub[0] * h.el + ub[2] * h.s[0] - ub[3] * h.s[2];
    V3<T> a2b = ub[1] * h.el + ub[2] * h.s[1] - ub[3] * h.s[3];
    const T sb0 = dot(ub[2], h.a1), sb1 = dot(ub[2], h.a2);
    const T sb2 = -dot(ub[3], h.a1), sb3 = -dot(ub[3], h.a2);
    // s0 = (x0-x3).Eh, s1 = (x1-x3).Eh, s2 = (x0-x2).Eh, s3 = (x1-x2).Eh
    xb[0] += h.Eh * (sb0 + sb2);
    xb[1] += h.Eh * (sb1 + sb3);
    xb[2] -= h.Eh * (sb2 + sb3);
    xb[3] -= h.Eh * (sb0 + sb1);
    const V3<T> Ehb = (x[0] - x[3]) * sb0 + (x[1] - x[3]) * sb1 + (x[0] - x[2]) * sb2 + (x[1] - x[2]) * sb3;
    // Eh = E / el, el = |E|
    const V3<T> Eb = (Ehb - h.Eh * dot(h.Eh, Ehb)) * (T(1) / h.el) + h.Eh * elb;
    // a = N / |N|^2
    const T n1sq = h.n1 * h.n1, n2sq = h.n2 * h.n2;
    N1b += a1b * (T(1) / n1sq) - h.N1 * (T(2) * dot(a1b, h.N1) / (n1sq * n1sq));
    N2b += a2b * (T(1) / n2sq) - h.N2 * (T(2) * dot(a2b, h.N2) / (n2sq * n2sq));
    // E = x3 - x2
    xb[3] += Eb;
    xb[2] -= Eb;
    // N1 = p x q with p = x0 - x2, q = x0 - x3
    {
        const V3<T> p = x[0] - x[2], qv = x[0] - x[3];
        const V3<T> pb = cross(qv, N1b), qb2 = cross(N1b, p);
        xb[0] += pb + qb2;
        xb[2] -= pb;
        xb[3] -= qb2;
    }
    // N2 = p x q with p = x1 - x3, q = x1 - x2
    {
        const V3<T> p = x[1] - x[3], qv = x[1] - x[2];
        const V3<T> pb = cross(qv, N2b), qb2 = cross(N2b, p);
        xb[1] += pb + qb2;
        xb[3] -= pb;
        xb[2] -= qb2;
    }
}

// ----------------------------------------------------------------- air ---
// Lift/drag on one triangle (App. A.1 thin shells; flat-plate reading): u = mean
// corner velocity (still air), N = (x1 - x0) x (x2 - x0), A = |N|/2, n = N/|N|,
// s = n.u, q = |u|^2:
//   F = -A (k_d |s| u + k_l s (q n - s u) / sqrt(q))     (lift term 0 at q = 0)
// and every corner receives F / 3.  |s| takes slope +1 at s = 0.
template <typename T>
__device__ __forceinline__ V3<T> air_total(const V3<T> x[3], const V3<T> v[3], T kd, T kl) {
    const V3<T> N = cross(x[1] - x[0], x[2] - x[0]);
    const T nn = gsqrt(dot(N, N));
    const V3<T> n = N * (T(1) / nn);
    const T A = T(0.5) * nn;
    const V3<T> u = (v[0] + v[1] + v[2]) * (T(1) / T(3));
    const T s = dot(n, u), q = dot(u, u);
    V3<T> F = u * (-(kd * A * gabs(s)));
    if (q > T(0)) F += (n * q - u * s) * (-(kl * A * s / gsqrt(q)));
    return F;
}

// Reverse mode of air_total for G, the adjoint of F (the mean of the corners'
// adjoints, as each corner receives F / 3).  With gu = G.u, gn = G.n and
// P = s q gn - s^2 gu the scalar <G, F> = -k_d A |s| gu - k_l A P / sqrt(q); its
// partials in A, s, q, n and u (direct) are chained through s = n.u, q = u.u,
// n = N/|N|, A = |N|/2 and N = a x b.  Returns F; adds the position adjoints to
// xb and writes each corner's velocity adjoint (ubar / 3) to vbc.
template <typename T>
__device__ __forceinline__ V3<T> air_adjoint(const V3<T> x[3], const V3<T> v[3], T kd, T kl, V3<T> G, V3<T> xb[3],
                                             V3<T>& vbc) {
    const V3<T> a = x[1] - x[0], b = x[2] - x[0];
    const V3<T> N = cross(a, b);
    const T nn = gsqrt(dot(N, N));
    const T inn = T(1) / nn;
    const V3<T> n = N * inn;
    const T A = T(0.5) * nn;
    const V3<T> u = (v[0] + v[1] + v[2]) * (T(1) / T(3));
    const T s = dot(n, u), q = dot(u, u);
    const T as = gabs(s), sg = s < T(0) ? T(-1) : T(1);
    const T gu = dot(G, u), gn = dot(G, n);
    V3<T> F = u * (-(kd * A * as));
    T Ab = -kd * as * gu;          // d/dA
    T sb = -kd * A * sg * gu;      // d/ds
    T qb = T(0);                   // d/dq
    V3<T> nb = zero3<T>();         // d/dn through gn
    V3<T> ub = G * (-kd * A * as); // d/du through gu
    if (q > T(0)) {
        const T r = gsqrt(q), ir = T(1) / r;
        F += (n * q - u * s) * (-(kl * A * s * ir));
        const T P = s * q * gn - s * s * gu;
        Ab += -kl * P * ir;
        sb += -kl * A * (q * gn - T(2) * s * gu) * ir;
        qb += -kl * A * s * ir * (T(0.5) * gn + s * gu / (T(2) * q));
        nb += G * (-kl * A * s * r);
        ub += G * (kl * A * s * s * ir);
    }
    nb += u * sb;
    ub += n * sb + u * (T(2) * qb);
    const V3<T> Nb = (nb - n * dot(nb, n)) * inn + n * (T(0.5) * Ab);
    const V3<T> abar = cross(b, Nb), bbar = cross(Nb, a);
    xb[1] += abar;
    xb[2] += bbar;
    xb[0] -= abar + bbar;
    vbc = ub * (T(1) / T(3));
    return F;
}

// ------------------------------------------------------ block reduction ---
template <typename T, int N>
__device__ __forceinline__ void block_sum(T v[N], T out[N]) {
    __shared__ T red[16][N];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += __shfl_down(v[k], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) red[wid][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < N; ++k) {
            T s = T(0);
            for (int w = 0; w < nw; ++w) s += red[w][k];
            out[k] = s;
        }
    }
}

// ------------------------------------------------------------- kernels ---
// A 4-vector in LDS, read and written as one 16-byte (FP32) access.
template <typename T>
struct alignas(4 * sizeof(T)) L4 {
    T x, y, z, w;
};
template <typename T>
__device__ __forceinline__ V3<T> v3(const L4<T>& a) {
    return mk3(a.x, a.y, a.z);
}
template <typename T>
__device__ __forceinline__ L4<T> l4(V3<T> v, T w) {
    return L4<T>{v.x, v.y, v.z, w};
}

// LDS accessors of the fused kernels (SoA rows of length n).
template <typename T>
__device__ __forceinline__ V3<T> lds3(const T* a, int n, int i) {
    return mk3(a[i], a[n + i], a[2 * n + i]);
}
template <typename T>
__device__ __forceinline__ void lds_st3(T* a, int n, int i, V3<T> v) {
    a[i] = v.x;
    a[n + i] = v.y;
    a[2 * n + i] = v.z;
}

// A tile particle's record (particle index, corner run, partial slot): three
// consecutive 32-bit words, one 12-byte load.
typedef int gi4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ gi4 ld_tp(const int32_t* tp, int64_t i) {
    const __attribute__((address_space(1))) int32_t* r = (const __attribute__((address_space(1))) int32_t*)(tp + 3 * i);
    return gi4{r[0], r[1], r[2], 0};
}

// Element pass: one workgroup per planned element tile.  The positions of the
// tile's particles are staged in LDS once (instead of one gather per corner), as
// 16-byte 4-vectors like the corner contributions (one LDS access per corner);
// each element writes its corners' forces at their positions in the tile's
// particle-sorted corner order; after one barrier each tile particle sums its
// contiguous run of corners in that fixed order and writes one partial.  No
// atomics; the result does not depend on the block size.
// AIR: the variant launched for models with a lift/drag body (the other compiles
// without any of that code).
template <typename T, bool AIR>
__device__ __forceinline__ void elem_fwd_tile(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd, const Tile tl,
                                              unsigned char* smem) {
    const ModelDev<T>& M = md[tl.model];
    const StepDev<T>& S = sd[tl.model];
    const int64_t np = M.np;
    const int m = tl.pad, tid = threadIdx.x, nth = blockDim.x;
    // triangle tiles of bodies with air also stage the velocities (lift/drag)
    const bool air = AIR && tl.kind == TILE_TRI && M.bodies[tl.body].air_on != 0;
    L4<T>* xs = reinterpret_cast<L4<T>*>(smem);  // [m] tile-particle positions
    L4<T>* vs = xs + m;                          // [m] velocities (air tiles)
    L4<T>* cs = xs + (air ? 2 * m : m);          // [corners] corner forces, particle-sorted
    gi4 mine = {0, 0, 0, 0};                     // this thread's first tile particle
    for (int j = tid; j < m; j += nth) {
        const gi4 r = ld_tp(M.tp, (int64_t)tl.id + j);
        if (j == tid) mine = r;
        xs[j] = l4(tl.kind == TILE_TET ? load_disp(M, S.x, S.x_abs, (int64_t)r.x) : load_pos(M, S.x, S.x_abs, (int64_t)r.x),
                   T(0));
        if (air) vs[j] = l4(ld3(S.v, np, (int64_t)r.x), T(0));
    }
    __syncthreads();
    for (int l = threadIdx.x; l < tl.count; l += blockDim.x) {
        const int64_t e = tl.begin + l;
        if (tl.kind == TILE_TET) {
            uint32_t cd[4];
            V3<T> x[4], f[4];
            T D[9];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                cd[c] = gld(M.tet_code, c * M.ne + e);
                x[c] = v3(xs[cd[c] & 0xffffu]);
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) D[k] = gld(M.tet_dinv, k * M.ne + e);
            const T act = S.act ? gld(S.act, e) : T(0);
            T J1;
            tet_force(x, D, gld(M.tet_vol, e), gld(S.mu, e), gld(S.lam, e), act, f, J1);
            if (J1 <= T(-1)) raise_flag(M, tl.body, 1);
#pragma unroll
            for (int c = 0; c < 4; ++c) cs[cd[c] >> 16] = l4(f[c], T(0));
        } else if (tl.kind == TILE_TRI) {
            uint32_t cd[3];
            V3<T> x[3], f[3];
            T D[4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cd[c] = gld(M.tri_code, c * M.nt + e);
                x[c] = v3(xs[cd[c] & 0xffffu]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) D[k] = gld(M.tri_dinv, k * M.nt + e);
            tri_force(x, D, gld(M.tri_area, e), gld(S.ktri, e), f);
            if (air) {
                V3<T> v[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = v3(vs[cd[c] & 0xffffu]);
                const V3<T> F = air_total(x, v, S.air[2 * tl.body], S.air[2 * tl.body + 1]) * (T(1) / T(3));
#pragma unroll
                for (int c = 0; c < 3; ++c) f[c] += F;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) cs[cd[c] >> 16] = l4(f[c], T(0));
        } else {
            uint32_t cd[4];
            V3<T> x[4], f[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                cd[c] = gld(M.hin_code, c * M.nh + e);
                x[c] = v3(xs[cd[c] & 0xffffu]);
            }
            hinge_force(x, gld(M.hin_phi0, e), M.bodies[tl.body].kb, S.hact ? gld(S.hact, e) : T(0), f);
#pragma unroll
            for (int c = 0; c < 4; ++c) cs[cd[c] >> 16] = l4(f[c], T(0));
        }
    }
    __syncthreads();
    for (int j = tid; j < m; j += nth) {
        const gi4 r = j == tid ? mine : ld_tp(M.tp, (int64_t)tl.id + j);
        const int r0 = r.y & 0xffff, rn = r.y >> 16;
        V3<T> f = zero3<T>();
        for (int k = 0; k < rn; ++k) f += v3(cs[r0 + k]);
        st_fslot(M.fslots, r.z, f.x, f.y, f.z);
    }
}

template <typename T, bool AIR>
__global__ void __launch_bounds__(512) k_elem_fwd(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd,
                                                   const Tile* __restrict__ tiles) {
    extern __shared__ __align__(16) unsigned char smem[];
    elem_fwd_tile<T, AIR>(md, sd, tiles[blockIdx.x], smem);
}

template <typename T>
__device__ __forceinline__ void part_fwd_tile(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd, const Tile tl) {
    const ModelDev<T>& M = md[tl.model];
    const StepDev<T>& S = sd[tl.model];
    const BodyDev<T>& B = M.bodies[tl.body];
    const int64_t np = M.np;
    const T dt = B.dt;
    T pl[4], cp[4];
    const bool contact = B.contact_on != 0;
    if (contact) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pl[k] = B.plane[k];
            cp[k] = S.contact[4 * tl.body + k];
        }
    }
    const V3<T> g = mk3(B.g[0], B.g[1], B.g[2]);
    for (int64_t l = threadIdx.x; l < tl.count; l += blockDim.x) {
        const int64_t i = tl.begin + l;
        // every load that does not depend on another is issued first
        const int64_t li = i - B.p0;
        const int64_t gb = M.gbase[B.g0 + (li >> 6)];
        const int32_t deg = M.pdeg[i];
        const V3<T> u = load_disp(M, S.x, S.x_abs, i), v = ld3(S.v, np, i);
        const T rg = contact ? gld(M.rgap, i) : T(0);
        const T w = inv_mass(M, S, i);
        V3<T> f = zero3<T>();
        sum_fslots(M.fslots, gb + (li & 63), deg, f);
        if (S.ckx) {
            st3(S.ckx, np, i, u);
            st3(S.ckv, np, i, v);
        }
        if (contact) f += contact_force_gap(gap_of(rg, pl, u), v, pl, cp);
        const T gate = w > T(0) ? T(1) : T(0);
        const V3<T> vn = v + (f * w + g * gate) * dt;
        const V3<T> un = u + vn * dt;
        if (!finite_pair(un, vn)) raise_flag(M, tl.body, 0);
        st3(S.vo, np, i, vn);
        st3(S.xo, np, i, S.xo_abs ? ld3(M.rest, np, i) + un : un);
    }
}

template <typename T>
__global__ void __launch_bounds__(512) k_part_fwd(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd,
                                                   const Tile* __restrict__ tiles) {
    part_fwd_tile<T>(md, sd, tiles[blockIdx.x]);
}

// Adjoint force of a particle: fbar = dt w (vbar+ + dt xbar+), with one explicit
// fused multiply-add per component so that every kernel forming it from the same
// adjoint state gets the same bits.
__device__ __forceinline__ float gfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double gfma(double a, double b, double c) { return fma(a, b, c); }
template <typename T>
__device__ __forceinline__ V3<T> fbar_of(V3<T> xb, V3<T> vb, T dt, T w) {
    const T s = dt * w;
    return mk3(gfma(xb.x, dt, vb.x) * s, gfma(xb.y, dt, vb.y) * s, gfma(xb.z, dt, vb.z) * s);
}
// Adjoint force of particle p at this adjoint step: the one the previous adjoint
// step's particle pass stored (S.fb), or formed from the adjoint state.
template <typename T>
__device__ __forceinline__ V3<T> corner_fbar(const ModelDev<T>& M, const StepDev<T>& S, int64_t p, T dt) {
    if (S.fb) return ld3(S.fb, M.np, p);
    return fbar_of(ld3(S.xb, M.np, p), ld3(S.vb, M.np, p), dt, inv_mass(M, S, p));
}

// Adjoint element pass, same tiling: the tile particles' positions and adjoint
// forces fbar are staged in LDS; each element writes (xbar contribution, f.fbar)
// of its corners in particle-sorted order; each tile particle sums its run into
// one partial.  Element-owned parameter gradients are read-modify-writes by the
// element's own thread.  Bodies with air: triangle tiles also stage velocities
// and sum each particle's velocity adjoint into a second partial (vslots); the
// body's other tiles write zero there, so every partial the particle pass reads
// is written.
template <typename T, bool AIR>
__device__ __forceinline__ void elem_adj_tile(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd, const Tile tl,
                                              unsigned char* smem) {
    const ModelDev<T>& M = md[tl.model];
    const StepDev<T>& S = sd[tl.model];
    const int64_t np = M.np;
    const T dt = M.bodies[tl.body].dt;
    const int m = tl.pad, tid = threadIdx.x, nth = blockDim.x;
    const bool air_body = AIR && M.bodies[tl.body].air_on != 0;
    const bool air = air_body && tl.kind == TILE_TRI;
    L4<T>* xs = reinterpret_cast<L4<T>*>(smem);  // [m] tile-particle positions
    L4<T>* fbs = xs + m;                         // [m] tile-particle adjoint forces
    L4<T>* vs = fbs + m;                         // [m] velocities (air tiles)
    L4<T>* cs = fbs + (air ? 2 * m : m);         // [corners] corner (xbar, f.fbar), particle-sorted
    L4<T>* cv = cs + 3 * tl.count;               // [corners] corner vbar (air tiles)
    gi4 mine = {0, 0, 0, 0};                     // this thread's first tile particle
    for (int j = tid; j < m; j += nth) {
        const gi4 r = ld_tp(M.tp, (int64_t)tl.id + j);
        if (j == tid) mine = r;
        const int64_t p = r.x;
        xs[j] = l4(tl.kind == TILE_TET ? load_disp(M, S.x, S.x_abs, p) : load_pos(M, S.x, S.x_abs, p), T(0));
        fbs[j] = l4(corner_fbar(M, S, p, dt), T(0));
        if (air) vs[j] = l4(ld3(S.v, np, p), T(0));
    }
    __syncthreads();
    for (int l = threadIdx.x; l < tl.count; l += blockDim.x) {
        const int64_t e = tl.begin + l;
        if (tl.kind == TILE_TET) {
            uint32_t cd[4];
            V3<T> x[4], f[4], fb[4], xb[4];
            T D[9];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                cd[c] = gld(M.tet_code, c * M.ne + e);
                x[c] = v3(xs[cd[c] & 0xffffu]);
                fb[c] = v3(fbs[cd[c] & 0xffffu]);
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) D[k] = gld(M.tet_dinv, k * M.ne + e);
            const T act = S.act ? gld(S.act, e) : T(0);
            // the accumulated gradients are read before the adjoint is computed, so
            // their loads overlap with the element's other loads
            const T gmu0 = S.g_mu ? gld(S.g_mu, e) : T(0), glam0 = S.g_lam ? gld(S.g_lam, e) : T(0),
                    gact0 = S.g_act ? gld(S.g_act, e) : T(0);
            T gmu, glam, gact;
            tet_adjoint(x, D, gld(M.tet_vol, e), gld(S.mu, e), gld(S.lam, e), act, fb, f, xb, gmu, glam, gact);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                cs[cd[c] >> 16] = l4(xb[c], dot(f[c], fb[c]));
            }
            if (S.g_mu) gst(S.g_mu, e, gmu0 + gmu);
            if (S.g_lam) gst(S.g_lam, e, glam0 + glam);
            if (S.g_act) gst(S.g_act, e, gact0 + gact);
        } else if (tl.kind == TILE_TRI) {
            uint32_t cd[3];
            V3<T> x[3], f[3], fb[3], xb[3];
            T D[4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cd[c] = gld(M.tri_code, c * M.nt + e);
                x[c] = v3(xs[cd[c] & 0xffffu]);
                fb[c] = v3(fbs[cd[c] & 0xffffu]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) D[k] = gld(M.tri_dinv, k * M.nt + e);
            const T gk0 = S.g_ktri ? gld(S.g_ktri, e) : T(0);
            T gk;
            tri_adjoint(x, D, gld(M.tri_area, e), gld(S.ktri, e), fb, f, xb, gk);
            if (air) {
                V3<T> v[3], vbc;
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = v3(vs[cd[c] & 0xffffu]);
                const V3<T> G = (fb[0] + fb[1] + fb[2]) * (T(1) / T(3));
                const V3<T> F =
                    air_adjoint(x, v, S.air[2 * tl.body], S.air[2 * tl.body + 1], G, xb, vbc) * (T(1) / T(3));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    f[c] += F;
                    cv[cd[c] >> 16] = l4(vbc, T(0));
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cs[cd[c] >> 16] = l4(xb[c], dot(f[c], fb[c]));
            }
            if (S.g_ktri) gst(S.g_ktri, e, gk0 + gk);
        } else {
            uint32_t cd[4];
            V3<T> x[4], f[4], fb[4], xb[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                cd[c] = gld(M.hin_code, c * M.nh + e);
                x[c] = v3(xs[cd[c] & 0xffffu]);
                fb[c] = v3(fbs[cd[c] & 0xffffu]);
            }
            const T gact0 = S.g_hact ? gld(S.g_hact, e) : T(0);
            T gact;
            hinge_adjoint(x, gld(M.hin_phi0, e), M.bodies[tl.body].kb, S.hact ? gld(S.hact, e) : T(0), fb, f, xb, gact);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                cs[cd[c] >> 16] = l4(xb[c], dot(f[c], fb[c]));
            }
            if (S.g_hact) gst(S.g_hact, e, gact0 + gact);
        }
    }
    __syncthreads();
    for (int j = tid; j < m; j += nth) {
        const gi4 r = j == tid ? mine : ld_tp(M.tp, (int64_t)tl.id + j);
        const int r0 = r.y & 0xffff, rn = r.y >> 16;
        V3<T> xb = zero3<T>();
        T d = T(0);
        for (int k = 0; k < rn; ++k) {
            const L4<T> c = cs[r0 + k];
            xb += v3(c);
            d += c.w;
        }
        st_slot(M.slots, r.z, xb.x, xb.y, xb.z, d);
        if (air_body) {
            V3<T> vb = zero3<T>();
            if (air)
                for (int k = 0; k < rn; ++k) vb += v3(cv[r0 + k]);
            st_slot(M.vslots, r.z, vb.x, vb.y, vb.z, T(0));
        }
    }
}

template <typename T, bool AIR>
__global__ void __launch_bounds__(512) k_elem_adj(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd,
                                                   const Tile* __restrict__ tiles) {
    extern __shared__ __align__(16) unsigned char smem[];
    elem_adj_tile<T, AIR>(md, sd, tiles[blockIdx.x], smem);
}

template <typename T, bool AIR>
__device__ __forceinline__ void part_adj_tile(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd, const Tile tl) {
    const ModelDev<T>& M = md[tl.model];
    const StepDev<T>& S = sd[tl.model];
    const BodyDev<T>& B = M.bodies[tl.body];
    const int64_t np = M.np;
    const T dt = B.dt;
    T pl[4], cp[4];
    const bool contact = B.contact_on != 0;
    if (contact) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pl[k] = B.plane[k];
            cp[k] = S.contact[4 * tl.body + k];
        }
    }
    T gc[4] = {T(0), T(0), T(0), T(0)};
    for (int64_t l = threadIdx.x; l < tl.count; l += blockDim.x) {
        const int64_t i = tl.begin + l;
        // every load that does not depend on another is issued first
        const int64_t li = i - B.p0;
        const int64_t gb = M.gbase[B.g0 + (li >> 6)];
        const int32_t deg = M.pdeg[i];
        const V3<T> xbp = ld3(S.xb, np, i), vbp = ld3(S.vb, np, i);
        const T w = inv_mass(M, S, i);
        V3<T> u = zero3<T>(), v = zero3<T>();
        T rg = T(0);
        if (contact) {
            u = load_disp(M, S.x, S.x_abs, i);
            v = ld3(S.v, np, i);
            rg = gld(M.rgap, i);
        }
        const int64_t base = gb + (li & 63);
        V3<T> xs = zero3<T>();
        T ds = T(0);
        sum_slots(M.slots, base, deg, xs, ds);
        const V3<T> vt = vbp + xbp * dt;
        const V3<T> fb = fbar_of(xbp, vbp, dt, w);
        V3<T> xcb = zero3<T>(), vcb = zero3<T>();
        if (AIR && B.air_on) {  // velocity adjoint of the lift/drag force, same partial slots
            T unused = T(0);
            sum_slots(M.vslots, base, deg, vcb, unused);
        }
        if (contact) {
            const V3<T> fc = contact_adjoint_gap(gap_of(rg, pl, u), v, pl, cp, fb, xcb, vcb, gc);
            ds += dot(fc, fb);
        }
        const V3<T> xbm = xbp + xs + xcb, vbm = vt + vcb;
        if (!finite_pair(xbm, vbm)) raise_flag(M, tl.body, 0);
        st3(S.xbo, np, i, xbm);
        st3(S.vbo, np, i, vbm);
        // the adjoint force of the previous step, for the next adjoint element pass
        if (S.fbo) st3(S.fbo, np, i, fbar_of(xbm, vbm, dt, w));
        if (S.g_mass && w > T(0)) S.g_mass[i] += -w * ds;  // dm = -w^2 dw, dw = dt f.vt = f.fbar / w
    }
    if (contact && S.g_contact) {
        T tot[4];
        block_sum<T, 4>(gc, tot);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 4; ++k) M.cpart[4 * tl.id + k] += tot[k];
    }
}

template <typename T, bool AIR>
__global__ void __launch_bounds__(512) k_part_adj(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd,
                                                   const Tile* __restrict__ tiles) {
    part_adj_tile<T, AIR>(md, sd, tiles[blockIdx.x]);
}

// Persistent execution: workgroup b runs body b through a run of steps.  Each step is
// the body's element tiles one after another, then its particle tiles; where the
// two-pass path has its launch boundaries there are workgroup barriers (the partials
// and states a pass writes are read by other threads of the workgroup in the next,
// all on one CU).  The tiles, their partial slots and their contact rows are
// those of the two-pass launches, so every result is bitwise the same; only the order
// in which tiles run changes, and no result depends on it.
template <typename T>
__global__ void __launch_bounds__(512) k_persist(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ rows,
                                                  int n_rows, const Tile* __restrict__ etiles,
                                                  const Tile* __restrict__ ptiles, const int32_t* __restrict__ toff) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x, nb = gridDim.x;
    const int e0 = toff[b], e1 = toff[b + 1], p0 = toff[nb + 1 + b], p1 = toff[nb + 2 + b];
    for (int r = 0; r < n_rows; ++r) {
        const StepDev<T>* sd = rows + r;  // tiles carry model 0: their record is sd[0]
        const bool adj = sd->adj != 0;
        for (int k = e0; k < e1; ++k) {
            if (adj) elem_adj_tile<T, false>(md, sd, etiles[k], smem);
            else elem_fwd_tile<T, false>(md, sd, etiles[k], smem);
            __syncthreads();  // the next tile reuses the LDS
        }
        __syncthreads();  // (workgroup-scope release and acquire of global memory)
        for (int k = p0; k < p1; ++k) {
            if (adj) part_adj_tile<T, false>(md, sd, ptiles[k]);
            else part_fwd_tile<T>(md, sd, ptiles[k]);
            __syncthreads();  // the contact reduction's LDS
        }
        __syncthreads();  // (workgroup-scope release and acquire of global memory)
    }
}

// Overlapped recompute: one launch runs an adjoint pass (row sd_adj) and a forward pass
// (row sd_fwd).  The two passes belong to independent chains of the checkpointed
// backward (the adjoint steps of one segment, the recompute of the previous segment's
// states) and touch disjoint buffers, so each tile's result is the one its own launch
// would give.  Split layout (particle launches, and element launches of models with few
// tiles): the adjoint tiles in the first workgroups, the forward tiles from workgroup
// span on (the tile count rounded up to a multiple of the 8 XCDs, so each list keeps
// its XCD placement; the workgroups in between return at once).  Paired layout
// (element launches of models with many tiles): workgroup b runs tile b's adjoint pass
// and then its forward pass, so the second pass finds the tile's element records
// (corner codes, Dm^-1, volume, mu, lambda) in cache.
template <typename T>
__global__ void __launch_bounds__(512) k_elem_dual(const ModelDev<T>* __restrict__ md,
                                                    const StepDev<T>* __restrict__ sd_adj,
                                                    const StepDev<T>* __restrict__ sd_fwd,
                                                    const Tile* __restrict__ tiles, int n, int span, int paired) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    if (paired) {
        const Tile tl = tiles[b];
        elem_adj_tile<T, false>(md, sd_adj, tl, smem);
        __syncthreads();  // the forward pass reuses the LDS
        elem_fwd_tile<T, false>(md, sd_fwd, tl, smem);
    } else if (b >= span) {
        elem_fwd_tile<T, false>(md, sd_fwd, tiles[b - span], smem);
    } else if (b < n) {
        elem_adj_tile<T, false>(md, sd_adj, tiles[b], smem);
    }
}
template <typename T>
__global__ void __launch_bounds__(512) k_part_dual(const ModelDev<T>* __restrict__ md,
                                                    const StepDev<T>* __restrict__ sd_adj, const Tile* __restrict__ adj,
                                                    int n_adj, int adj_span, const StepDev<T>* __restrict__ sd_fwd,
                                                    const Tile* __restrict__ fwd) {
    const int b = blockIdx.x;
    if (b >= adj_span) part_fwd_tile<T>(md, sd_fwd, fwd[b - adj_span]);
    else if (b < n_adj) part_adj_tile<T, false>(md, sd_adj, adj[b]);
}

// Serving: the tile at launch position `pos` of a round's element or particle launch.
// The round's tiles are the concatenation of its segments (each query's resident tiles,
// segments in increasing order of their first position `begin`) laid out in XCD order:
// position pos holds tile t = (pos % N_XCD) * G + pos / N_XCD of the concatenation
// (G = grid / N_XCD; fewer than N_XCD tiles keep their order), and positions past the
// total are empty tiles of `empty_kind` reducing into row dummy_id of model 0.  Each
// wavefront finds t's segment from the segments' begins by ballots (see below), then
// loads that segment and the tile: three dependent loads for up to 256 segments.
__device__ __forceinline__ Tile round_tile(const TileSeg* __restrict__ seg, int nseg, int total, int grid, int pos,
                                           int empty_kind, int dummy_id) {
    Tile tl;
    const int nx = 8;  // N_XCD
    const int t = total < nx ? pos : (pos % nx) * (grid / nx) + pos / nx;
    if (t >= total) {
        tl.model = 0;
        tl.body = 0;
        tl.kind = empty_kind;
        tl.count = 0;
        tl.begin = 0;
        tl.id = dummy_id;
        tl.pad = 0;
        return tl;
    }
    // the first SEG_LOOKUP_CHUNKS * 64 begins in one round of independent loads; the
    // segments with begin <= t form a prefix whose length, summed over the ballots,
    // names the segment (a longer table continues chunk by chunk)
    constexpr int SEG_LOOKUP_CHUNKS = 4;
    const int lane = threadIdx.x & 63;
    int bg[SEG_LOOKUP_CHUNKS];
#pragma unroll
    for (int k = 0; k < SEG_LOOKUP_CHUNKS; ++k) {
        const int i = 64 * k + lane;
        bg[k] = i < nseg ? seg[i].begin : INT32_MAX;
    }
    int c = 0;
#pragma unroll
    for (int k = 0; k < SEG_LOOKUP_CHUNKS; ++k) c += __popcll(__ballot(bg[k] <= t));
    for (int b = 64 * SEG_LOOKUP_CHUNKS; b < nseg && c == b; b += 64) {  // uniform trip count
        const int i = b + lane;
        c += __popcll(__ballot(i < nseg && seg[i].begin <= t));
    }
    const TileSeg g = seg[c - 1];  // the same address in every lane
    const Tile* tiles = g.tiles;
    const int sbegin = g.begin, smodel = g.model, sflags = g.flags;
    tl = tiles[t - sbegin];
    tl.model = smodel;
    tl.kind |= sflags;
    return tl;
}

// Serving: one launch over the forward and adjoint element tiles of a round (the
// adjoint ones marked TILE_ADJ), and one over its particle tiles.  Each workgroup runs
// the same element or particle code as the two-pass kernels, for its query's launch
// records; forward and adjoint tiles of a launch belong to different queries, so the
// two kinds of work overlap instead of following each other.  The branch is uniform
// per workgroup.
template <typename T>
__global__ void __launch_bounds__(512) k_elem_mixed(const ModelDev<T>* __restrict__ md,
                                                     const StepDev<T>* __restrict__ sd, const TileSeg* __restrict__ seg,
                                                     int nseg, int total, int grid, int dummy_id) {
    extern __shared__ __align__(16) unsigned char smem[];
    Tile tl = round_tile(seg, nseg, total, grid, blockIdx.x, TILE_TET, dummy_id);
    if (tl.kind & TILE_ADJ) {
        tl.kind &= ~TILE_ADJ;
        elem_adj_tile<T, false>(md, sd, tl, smem);
    } else {
        elem_fwd_tile<T, false>(md, sd, tl, smem);
    }
}
template <typename T>
__global__ void __launch_bounds__(512) k_part_mixed(const ModelDev<T>* __restrict__ md,
                                                     const StepDev<T>* __restrict__ sd, const TileSeg* __restrict__ seg,
                                                     int nseg, int total, int grid, int dummy_id) {
    Tile tl = round_tile(seg, nseg, total, grid, blockIdx.x, TILE_PART, dummy_id);
    if (tl.kind & TILE_ADJ) {
        tl.kind &= ~TILE_ADJ;
        part_adj_tile<T, false>(md, sd, tl);
    } else {
        part_fwd_tile<T>(md, sd, tl);
    }
}

// Batched copy: workgroup b moves piece b, 16 bytes per lane and load when both
// addresses are 16-byte aligned (the staging area and every workspace region are),
// bytes otherwise.
__global__ void __launch_bounds__(256) k_stage_copy(const StageSeg* __restrict__ segs) {
    const StageSeg g = segs[blockIdx.x];
    const char* src = g.src;
    char* dst = g.dst;
    const int64_t n = g.n;
    int64_t done = 0;
    if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0) {
        const int64_t nv = n >> 4;
        uint4* d4 = reinterpret_cast<uint4*>(dst);
        const uint4* s4 = reinterpret_cast<const uint4*>(src);
        for (int64_t i = threadIdx.x; i < nv; i += blockDim.x) d4[i] = src ? s4[i] : make_uint4(0u, 0u, 0u, 0u);
        done = nv << 4;
    }
    for (int64_t i = done + threadIdx.x; i < n; i += blockDim.x) dst[i] = src ? src[i] : (char)0;
}

template <typename T>
__global__ void k_contact_reduce(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd) {
    const ModelDev<T>& M = md[0];
    const StepDev<T>& S = sd[0];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * M.n_bodies || !S.g_contact) return;
    const int b = t >> 2, k = t & 3;
    const BodyDev<T>& B = M.bodies[b];
    if (!B.contact_on) return;
    T s = T(0);
    for (int r = B.pt0; r < B.pt1; ++r) s += M.cpart[4 * r + k];
    S.g_contact[t] += s;
}

template <typename T>
__global__ void __launch_bounds__(512) k_loss_part(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd,
                                                    const Tile* __restrict__ tiles) {
    const Tile tl = tiles[blockIdx.x];
    const ModelDev<T>& M = md[tl.model];
    const StepDev<T>& S = sd[tl.model];
    const BodyDev<T>& B = M.bodies[tl.body];
    const int64_t np = M.np;
    const T scale = T(2) / T(B.np);
    T acc[1] = {T(0)};
    for (int64_t l = threadIdx.x; l < tl.count; l += blockDim.x) {
        const int64_t i = tl.begin + l;
        // displacement input: x = X + u rounded first, exactly as a call's final
        // state is handed to the caller, so the loss of a state kept on the device
        // equals the loss of that state taken out and passed back
        const V3<T> x = S.x_abs ? ld3(S.x, np, i) : ld3(M.rest, np, i) + ld3(S.x, np, i);
        const V3<T> d = x - ld3(S.target, np, i);
        acc[0] += dot(d, d);
        if (S.xbo) st3(S.xbo, np, i, d * scale);
        if (S.vbo) st3(S.vbo, np, i, zero3<T>());
    }
    T tot[1];
    block_sum<T, 1>(acc, tot);
    if (threadIdx.x == 0) M.lpart[tl.id] = tot[0];
}

template <typename T>
__global__ void k_loss_reduce(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd) {
    const ModelDev<T>& M = md[0];
    const StepDev<T>& S = sd[0];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= M.n_bodies) return;
    const BodyDev<T>& B = M.bodies[b];
    T s = T(0);
    for (int r = B.pt0; r < B.pt1; ++r) s += M.lpart[r];
    S.loss[b] = s / T(B.np);
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}


// ------------------------------------------------------------ fused path ---
// One workgroup owns one body for a whole segment of steps.  Positions and
// velocities (forward) or positions and adjoint forces (reverse) of the body's
// particles live in LDS; element contributions are accumulated in LDS colour by
// colour: the elements of a colour share no particle, so each LDS update is
// race-free, and every particle receives its contributions in colour order
// (deterministic).  A workgroup barrier separates colours; nothing else
// synchronises, and every barrier sits in a loop whose trip count is uniform
// over the workgroup.  Each thread loads its element record of the next colour
// before it processes the current one, so record latency overlaps the current
// colour's work and barrier.  Per-element parameters are read from a copy in
// colour order (gathered once per call) and gradients accumulate in colour order
// (scattered back once per call).

// Status flags in the fused kernels: FP32 only.  The FP64 fused kernels (a checking
// build) exceed the register file and spill heavily; with the flag stores added their
// actuation and mu gradients changed (4e-8 in the FP64 actuated test, 8e-15 without), and a
// 256-thread FP64 launch that removes the spills faulted the GPU; neither has a cause
// shown in this code, so the FP64 fused kernels keep the source that passes and raise
// no flags (the two-pass FP64 kernels, which do not spill, do).
template <typename T> constexpr bool FUSED_FLAGS = sizeof(T) == 4;

// Adds v[q] to the LDS accumulators [3][n] of an element's corners li[q]; with
// w, also w[q] to the fourth row (a + 3n).  An element's corners are distinct
// particles (the planner rejects elements that repeat one), so all reads are
// issued before all writes: one LDS round trip per element instead of one per
// corner component.  Each word gets the same single add as a plain `+=`.
template <int NC, typename T>
__device__ __forceinline__ void lds_add_corners(T* a, int n, const int* li, const V3<T>* v, const T* w = nullptr) {
    T c[NC][4];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        c[q][0] = a[li[q]];
        c[q][1] = a[n + li[q]];
        c[q][2] = a[2 * n + li[q]];
        if (w) c[q][3] = a[3 * n + li[q]];
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        a[li[q]] = c[q][0] + v[q].x;
        a[n + li[q]] = c[q][1] + v[q].y;
        a[2 * n + li[q]] = c[q][2] + v[q].z;
        if (w) a[3 * n + li[q]] = c[q][3] + w[q];
    }
}

template <typename T>
struct TetRec {
    int li[4];
    T D[9];
    T V, mu, lam, act;
};
template <typename T>
struct TriRec {
    int li[3];
    T D[4];
    T A, k;
};
template <typename T>
struct HinRec {
    int li[4];
    T phi0, act;
};

template <typename T>
__device__ __forceinline__ void load_rec(const ModelDev<T>& M, int e, TetRec<T>& r) {
#pragma unroll
    for (int q = 0; q < 4; ++q) r.li[q] = gld(M.f_tet_idx, q * M.ne + e);
#pragma unroll
    for (int q = 0; q < 9; ++q) r.D[q] = gld(M.f_tet_dinv, q * M.ne + e);
    r.V = gld(M.f_tet_vol, e);
    r.mu = gld(M.f_par, e);
    r.lam = gld(M.f_par, M.ne + e);
    r.act = gld(M.f_par, 2 * M.ne + e);
}
template <typename T>
__device__ __forceinline__ void load_rec(const ModelDev<T>& M, int e, TriRec<T>& r) {
#pragma unroll
    for (int q = 0; q < 3; ++q) r.li[q] = gld(M.f_tri_idx, q * M.nt + e);
#pragma unroll
    for (int q = 0; q < 4; ++q) r.D[q] = gld(M.f_tri_dinv, q * M.nt + e);
    r.A = gld(M.f_tri_area, e);
    r.k = gld(M.f_ktri, e);
}
template <typename T>
__device__ __forceinline__ void load_rec(const ModelDev<T>& M, int e, HinRec<T>& r) {
#pragma unroll
    for (int q = 0; q < 4; ++q) r.li[q] = gld(M.f_hin_idx, q * M.nh + e);
    r.phi0 = gld(M.f_hin_phi0, e);
    r.act = gld(M.f_hpar, e);
}

// Adjoint records also carry the element's running parameter gradient, read
// with the record so that the per-element read-modify-write does not wait on a
// load issued after the previous element's store.
template <typename T>
struct TetRecA : TetRec<T> {
    T gmu, glam;
};
template <typename T>
struct TriRecA : TriRec<T> {
    T gk;
};
// with the actuation gradients (only in the variant launched when they are requested)
template <typename T>
struct TetRecAct : TetRecA<T> {
    T gact;
};
template <typename T>
struct HinRecAct : HinRec<T> {
    T gact;
};
template <typename T>
__device__ __forceinline__ void load_rec(const ModelDev<T>& M, int e, TetRecA<T>& r) {
    load_rec(M, e, static_cast<TetRec<T>&>(r));
    r.gmu = gld(M.f_g, e);
    r.glam = gld(M.f_g, M.ne + e);
}
template <typename T>
__device__ __forceinline__ void load_rec(const ModelDev<T>& M, int e, TetRecAct<T>& r) {
    load_rec(M, e, static_cast<TetRecA<T>&>(r));
    r.gact = gld(M.f_g, 2 * M.ne + e);
}
template <typename T>
__device__ __forceinline__ void load_rec(const ModelDev<T>& M, int e, TriRecA<T>& r) {
    load_rec(M, e, static_cast<TriRec<T>&>(r));
    r.gk = gld(M.f_gk, e);
}
template <typename T>
__device__ __forceinline__ void load_rec(const ModelDev<T>& M, int e, HinRecAct<T>& r) {
    load_rec(M, e, static_cast<HinRec<T>&>(r));
    r.gact = gld(M.f_gh, e);
}

// Copies the body's colour bounds of all three kinds to LDS (kind k's ncol + 1
// bounds at cb[k]), once per launch: read before every colour, they would
// otherwise put a global-load latency in front of each colour's record loads.
template <typename T>
__device__ __forceinline__ void stage_colour_bounds(const ModelDev<T>& M, const BodyDev<T>& B, int32_t* base,
                                                    int32_t* cb[3]) {
    cb[0] = base;
    cb[1] = cb[0] + B.ncol[0] + 1;
    cb[2] = cb[1] + B.ncol[1] + 1;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        for (int i = threadIdx.x; i <= B.ncol[k]; i += blockDim.x) cb[k][i] = gld(M.coff, (int64_t)B.cbase[k] + i);
}

// Corner contributions of one element: corners li, 3-vectors v (and a scalar w
// per corner for a fourth accumulator row).
template <typename T, int NC>
struct Contrib {
    int li[NC];
    V3<T> v[NC];
    T w[NC];
};

// Processes the colours [0, ncol) of one element kind.  The elements of a colour
// share no particle, so a colour with more elements than the workgroup has
// threads runs in several rounds without a barrier between them; the sweep walks
// the sequence of (colour, round) slots, one element per thread per slot, with a
// workgroup barrier after each colour's last round.  Element contributions do not
// depend on the accumulators (positions and adjoint forces are fixed during a
// sweep), so K slots are taken at a time: first the records of all K are loaded
// and their contributions computed (indices clamped into the colour, so this is
// straight-line code and the K elements overlap), then they are added slot by
// slot.  `compute(e, rec, valid, out)` must not write anything shared unless
// `valid`; `W` adds the fourth accumulator row.
template <int K, int NC, bool W, typename T, typename Rec, typename Compute>
__device__ __forceinline__ void colour_sweep(const ModelDev<T>& M, const int32_t* cb, int ncol, T* acc, int npb,
                                             Compute compute) {
    const int tid = threadIdx.x, nth = blockDim.x;
    int c = 0, round = 0;
    while (c < ncol) {
        int e[K], hi[K];
        bool live[K], last[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            live[k] = c < ncol;
            const int cc = min(c, ncol - 1);
            const int lo = cb[cc];
            hi[k] = cb[cc + 1];
            e[k] = lo + round * nth + tid;
            last[k] = lo + (round + 1) * nth >= hi[k];
            if (live[k]) {
                if (last[k]) {
                    ++c;
                    round = 0;
                } else {
                    ++round;
                }
            }
        }
        Contrib<T, NC> o[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int ek = min(e[k], hi[k] - 1);
            Rec r;
            load_rec(M, ek, r);
            compute(ek, r, live[k] && e[k] < hi[k], o[k]);
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (live[k]) {
                if (e[k] < hi[k]) lds_add_corners<NC>(acc, npb, o[k].li, o[k].v, W ? o[k].w : nullptr);
                if (last[k]) __syncthreads();
            }
    }
}

template <typename T>
__global__ void __launch_bounds__(FUSED_FWD_BLOCK) k_fused_fwd(const ModelDev<T>* __restrict__ md,
                                                               const StepDev<T>* __restrict__ sd,
                                                               const int32_t* __restrict__ order) {
    extern __shared__ __align__(16) unsigned char smem[];
    const ModelDev<T>& M = md[0];
    const StepDev<T>& S = sd[0];
    const int b = order[blockIdx.x];
    const BodyDev<T>& B = M.bodies[b];
    const int npb = (int)B.np;
    const int64_t np = M.np, p0 = B.p0;
    T* xs = reinterpret_cast<T*>(smem);  // [3][npb] displacements from rest
    T* vs = xs + 3 * npb;                // [3][npb] velocities
    T* fs = vs + 3 * npb;                // [3][npb] force accumulators
    int32_t* cb[3];                      // colour bounds, after the particle arrays
    stage_colour_bounds(M, B, reinterpret_cast<int32_t*>(fs + 3 * npb), cb);
    const T dt = B.dt;
    const V3<T> g = mk3(B.g[0], B.g[1], B.g[2]);
    const bool contact = B.contact_on != 0;
    T pl[4], cp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        pl[k] = B.plane[k];
        cp[k] = contact ? S.contact[4 * b + k] : T(0);
    }
    for (int li = threadIdx.x; li < npb; li += blockDim.x) {
        lds_st3(xs, npb, li, load_disp(M, S.x, S.x_abs, p0 + li));
        lds_st3(vs, npb, li, ld3(S.v, np, p0 + li));
    }
    for (int step = 0; step < S.nsteps; ++step) {
        const int t = S.t_base + step;
        const bool ck = S.ckx != nullptr && t % S.ckpt_every == 0;
        for (int li = threadIdx.x; li < npb; li += blockDim.x) {
            if (ck) {
                T* cx = S.ckx + (int64_t)(t / S.ckpt_every) * 6 * np;
                st3(cx, np, p0 + li, lds3(xs, npb, li));
                st3(cx + 3 * np, np, p0 + li, lds3(vs, npb, li));
            }
            lds_st3(fs, npb, li, zero3<T>());
        }
        __syncthreads();
        colour_sweep<FUSED_AHEAD_FWD, 4, false, T, TetRec<T>>(M, cb[0], B.ncol[0], fs, npb,
                                                          [&](int, const TetRec<T>& r, bool, Contrib<T, 4>& o) {
            V3<T> x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                o.li[q] = r.li[q];
                x[q] = lds3(xs, npb, r.li[q]);
            }
            T J1;
            tet_force(x, r.D, r.V, r.mu, r.lam, r.act, o.v, J1);
            if constexpr (FUSED_FLAGS<T>)
                if (J1 <= T(-1)) raise_flag(M, b, 1);
        });
        colour_sweep<FUSED_AHEAD_FWD, 3, false, T, TriRec<T>>(M, cb[1], B.ncol[1], fs, npb,
                                                          [&](int, const TriRec<T>& r, bool, Contrib<T, 3>& o) {
            V3<T> x[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                o.li[q] = r.li[q];
                x[q] = ld3(M.rest, np, p0 + r.li[q]) + lds3(xs, npb, r.li[q]);
            }
            tri_force(x, r.D, r.A, r.k, o.v);
        });
        colour_sweep<FUSED_AHEAD_FWD, 4, false, T, HinRec<T>>(M, cb[2], B.ncol[2], fs, npb,
                                                          [&](int, const HinRec<T>& r, bool, Contrib<T, 4>& o) {
            V3<T> x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                o.li[q] = r.li[q];
                x[q] = ld3(M.rest, np, p0 + r.li[q]) + lds3(xs, npb, r.li[q]);
            }
            hinge_force(x, r.phi0, B.kb, r.act, o.v);
        });
        // contact + semi-implicit Euler on the workgroup's own particles
        for (int li = threadIdx.x; li < npb; li += blockDim.x) {
            const int64_t p = p0 + li;
            V3<T> f = lds3(fs, npb, li);
            V3<T> x = lds3(xs, npb, li);
            V3<T> v = lds3(vs, npb, li);
            if (contact) f += contact_force_gap(gap_of(gld(M.rgap, p), pl, x), v, pl, cp);
            const T w = inv_mass(M, S, p);
            const T gate = w > T(0) ? T(1) : T(0);
            v = v + (f * w + g * gate) * dt;
            x = x + v * dt;
            if constexpr (FUSED_FLAGS<T>)
                if (!finite_pair(x, v)) raise_flag(M, b, 0);
            lds_st3(xs, npb, li, x);
            lds_st3(vs, npb, li, v);
            if (S.seg) {
                T* sx = S.seg + (int64_t)step * 6 * np;
                st3(sx, np, p, x);
                st3(sx + 3 * np, np, p, v);
            }
        }
        __syncthreads();
    }
    if (S.xo)
        for (int li = threadIdx.x; li < npb; li += blockDim.x) {
            const V3<T> u = lds3(xs, npb, li);
            st3(S.xo, np, p0 + li, S.xo_abs ? ld3(M.rest, np, p0 + li) + u : u);
            st3(S.vo, np, p0 + li, lds3(vs, npb, li));
        }
}

// Adjoint steps t0 + nsteps - 1 .. t0 of one body.  The state at t0 is (S.x, S.v),
// later states come from S.seg_in.  The adjoint state is carried in S.xbo / S.vbo
// (each particle's entries are touched only by its own thread).
// ACT: also accumulate the tet / hinge actuation gradients (the variant launched
// only when the call requests them, so the other one moves no bytes for them).
template <typename T, bool ACT>
__global__ void __launch_bounds__(FUSED_ADJ_BLOCK) k_fused_adj(const ModelDev<T>* __restrict__ md,
                                                               const StepDev<T>* __restrict__ sd,
                                                               const int32_t* __restrict__ order) {
    using TetR = typename std::conditional<ACT, TetRecAct<T>, TetRecA<T>>::type;
    using HinR = typename std::conditional<ACT, HinRecAct<T>, HinRec<T>>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const ModelDev<T>& M = md[0];
    const StepDev<T>& S = sd[0];
    const int b = order[blockIdx.x];
    const BodyDev<T>& B = M.bodies[b];
    const int npb = (int)B.np;
    const int64_t np = M.np, p0 = B.p0;
    T* xs = reinterpret_cast<T*>(smem);  // [3][npb] displacements at the step's start
    T* fbs = xs + 3 * npb;               // [3][npb] adjoint force
    T* acc = fbs + 3 * npb;              // [4][npb] xbar contributions, f . fbar
    int32_t* cb[3];                      // colour bounds, after the particle arrays
    stage_colour_bounds(M, B, reinterpret_cast<int32_t*>(acc + 4 * npb), cb);
    const T dt = B.dt;
    const bool contact = B.contact_on != 0;
    const bool want_e = S.g_mu != nullptr || S.g_lam != nullptr || (ACT && S.g_act != nullptr),
               want_k = S.g_ktri != nullptr, want_h = ACT && S.g_hact != nullptr;
    T pl[4], cp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        pl[k] = B.plane[k];
        cp[k] = contact ? S.contact[4 * b + k] : T(0);
    }
    if (S.xbo != S.xb)
        for (int li = threadIdx.x; li < npb; li += blockDim.x) {
            st3(S.xbo, np, p0 + li, ld3(S.xb, np, p0 + li));
            st3(S.vbo, np, p0 + li, ld3(S.vb, np, p0 + li));
        }
    for (int step = S.nsteps - 1; step >= 0; --step) {
        const T* sx = step == 0 ? S.x : S.seg_in + (int64_t)(step - 1) * 6 * np;
        const T* sv = step == 0 ? S.v : sx + 3 * np;
        const int32_t sabs = step == 0 ? S.x_abs : 0;
        for (int li = threadIdx.x; li < npb; li += blockDim.x) {
            lds_st3(xs, npb, li, load_disp(M, sx, sabs, p0 + li));
            const V3<T> vt = ld3(S.vbo, np, p0 + li) + ld3(S.xbo, np, p0 + li) * dt;
            lds_st3(fbs, npb, li, vt * (dt * inv_mass(M, S, p0 + li)));
            lds_st3(acc, npb, li, zero3<T>());
            acc[3 * npb + li] = T(0);
        }
        __syncthreads();
        colour_sweep<FUSED_AHEAD_ADJ, 4, true, T, TetR>(M, cb[0], B.ncol[0], acc, npb,
                                                    [&](int e, const TetR& r, bool valid, Contrib<T, 4>& o) {
            V3<T> x[4], f[4], fb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                o.li[q] = r.li[q];
                x[q] = lds3(xs, npb, r.li[q]);
                fb[q] = lds3(fbs, npb, r.li[q]);
            }
            T gmu, glam, gact;
            tet_adjoint(x, r.D, r.V, r.mu, r.lam, r.act, fb, f, o.v, gmu, glam, gact);
#pragma unroll
            for (int q = 0; q < 4; ++q) o.w[q] = dot(f[q], fb[q]);
            if (want_e && valid) {
                gst(M.f_g, e, r.gmu + gmu);
                gst(M.f_g, M.ne + e, r.glam + glam);
                if constexpr (ACT) gst(M.f_g, 2 * M.ne + e, r.gact + gact);
            }
        });
        colour_sweep<FUSED_AHEAD_ADJ, 3, true, T, TriRecA<T>>(M, cb[1], B.ncol[1], acc, npb,
                                                          [&](int e, const TriRecA<T>& r, bool valid, Contrib<T, 3>& o) {
            V3<T> x[3], f[3], fb[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                o.li[q] = r.li[q];
                x[q] = ld3(M.rest, np, p0 + r.li[q]) + lds3(xs, npb, r.li[q]);
                fb[q] = lds3(fbs, npb, r.li[q]);
            }
            T gk;
            tri_adjoint(x, r.D, r.A, r.k, fb, f, o.v, gk);
#pragma unroll
            for (int q = 0; q < 3; ++q) o.w[q] = dot(f[q], fb[q]);
            if (want_k && valid) gst(M.f_gk, e, r.gk + gk);
        });
        colour_sweep<FUSED_AHEAD_ADJ, 4, true, T, HinR>(M, cb[2], B.ncol[2], acc, npb,
                                                    [&](int e, const HinR& r, bool valid, Contrib<T, 4>& o) {
            V3<T> x[4], f[4], fb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                o.li[q] = r.li[q];
                x[q] = ld3(M.rest, np, p0 + r.li[q]) + lds3(xs, npb, r.li[q]);
                fb[q] = lds3(fbs, npb, r.li[q]);
            }
            T gact;
            hinge_adjoint(x, r.phi0, B.kb, r.act, fb, f, o.v, gact);
#pragma unroll
            for (int q = 0; q < 4; ++q) o.w[q] = dot(f[q], fb[q]);
            if constexpr (ACT)
                if (want_h && valid) gst(M.f_gh, e, r.gact + gact);
        });
        // contact adjoint and the integrator's adjoint on the workgroup's own particles
        T gc[4] = {T(0), T(0), T(0), T(0)};
        for (int li = threadIdx.x; li < npb; li += blockDim.x) {
            const int64_t p = p0 + li;
            const V3<T> xbp = ld3(S.xbo, np, p);
            const V3<T> vt = ld3(S.vbo, np, p) + xbp * dt;
            const V3<T> fb = lds3(fbs, npb, li);
            T ds = acc[3 * npb + li];
            V3<T> xcb = zero3<T>(), vcb = zero3<T>();
            if (contact) {
                const V3<T> fc = contact_adjoint_gap(gap_of(gld(M.rgap, p), pl, lds3(xs, npb, li)), ld3(sv, np, p), pl,
                                                     cp, fb, xcb, vcb, gc);
                ds += dot(fc, fb);
            }
            if constexpr (FUSED_FLAGS<T>) {
                const V3<T> xbm = xbp + lds3(acc, npb, li) + xcb, vbm = vt + vcb;
                if (!finite_pair(xbm, vbm)) raise_flag(M, b, 0);
                st3(S.xbo, np, p, xbm);
                st3(S.vbo, np, p, vbm);
            } else {
                st3(S.xbo, np, p, xbp + lds3(acc, npb, li) + xcb);
                st3(S.vbo, np, p, vt + vcb);
            }
            const T w = inv_mass(M, S, p);
            if (S.g_mass && w > T(0)) gst(S.g_mass, p, gld(S.g_mass, p) - w * ds);
        }
        // This step's contact-parameter gradient, reduced over the workgroup and added
        // by one thread.  (No per-thread accumulator lives across steps: when such a
        // value is spilled, the FP64 build was seen to restore it only in the lanes that
        // ran the contact branch, leaving the other lanes' copies clobbered.)
        if (contact && S.g_contact) {
            T tot[4];
            block_sum<T, 4>(gc, tot);
            if (threadIdx.x == 0)
#pragma unroll
                for (int k = 0; k < 4; ++k) gst(S.g_contact, 4 * b + k, gld(S.g_contact, 4 * b + k) + tot[k]);
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void k_fused_params(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd) {
    const ModelDev<T>& M = md[0];
    const StepDev<T>& S = sd[0];
    const bool clear_e = S.g_mu != nullptr || S.g_lam != nullptr || S.g_act != nullptr,
               clear_k = S.g_ktri != nullptr, clear_h = S.g_hact != nullptr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < M.ne; e += stride) {
        const int32_t o = M.f_tet_orig[e];
        M.f_par[e] = S.mu[o];
        M.f_par[M.ne + e] = S.lam[o];
        M.f_par[2 * M.ne + e] = S.act ? S.act[o] : T(0);
        if (clear_e) {
            M.f_g[e] = T(0);
            M.f_g[M.ne + e] = T(0);
            M.f_g[2 * M.ne + e] = T(0);
        }
    }
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < M.nh; h += stride) {
        M.f_hpar[h] = S.hact ? S.hact[M.f_hin_orig[h]] : T(0);
        if (clear_h) M.f_gh[h] = T(0);
    }
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < M.nt; t += stride) {
        M.f_ktri[t] = S.ktri[M.f_tri_orig[t]];
        if (clear_k) M.f_gk[t] = T(0);
    }
}

template <typename T>
__global__ void k_fused_grads(const ModelDev<T>* __restrict__ md, const StepDev<T>* __restrict__ sd) {
    const ModelDev<T>& M = md[0];
    const StepDev<T>& S = sd[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < M.ne; e += stride) {
        const int32_t o = M.f_tet_orig[e];
        if (S.g_mu) S.g_mu[o] += M.f_g[e];
        if (S.g_lam) S.g_lam[o] += M.f_g[M.ne + e];
        if (S.g_act) S.g_act[o] += M.f_g[2 * M.ne + e];
    }
    if (S.g_hact)
        for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < M.nh; h += stride)
            S.g_hact[M.f_hin_orig[h]] += M.f_gh[h];
    if (S.g_ktri)
        for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < M.nt; t += stride)
            S.g_ktri[M.f_tri_orig[t]] += M.f_gk[t];
}

int check_launch() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace

namespace {
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

// Launches kernel, with the armed timing events (if any) as its start and end.
template <typename K, typename... Args>
void launch_timed(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t stream, Args... args) {
    if (t_ev_start && t_ev_stop) {
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, stream, t_ev_start, t_ev_stop, 0, args...);
        t_ev_start = t_ev_stop = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, args...);
    }
}
}  // namespace

void arm_launch_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}

bool disarm_launch_events() {
    const bool consumed = t_ev_start == nullptr;
    t_ev_start = t_ev_stop = nullptr;
    return consumed;
}

// The element kernels' dynamic LDS can exceed the default limit (FP64 tiles).
// (raised once per kernel and size, outside any steady-state launch sequence)
void allow_lds(const void* kernel, size_t lds, size_t& allowed) {
    if (lds > allowed) {
        (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        allowed = lds;
    }
}
template <typename T, bool AIR>
int launch_elem_fwd_v(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, size_t lds,
                      void* stream) {
    static size_t allowed = 48 * 1024;
    allow_lds(reinterpret_cast<const void*>(&k_elem_fwd<T, AIR>), lds, allowed);
    launch_timed(k_elem_fwd<T, AIR>, dim3(ntiles), dim3(block), lds, (hipStream_t)stream, md, sd, tiles);
    return check_launch();
}
template <typename T>
int launch_elem_fwd(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, size_t lds,
                    bool air, void* stream) {
    if (ntiles <= 0) return 0;
    return air ? launch_elem_fwd_v<T, true>(md, sd, tiles, ntiles, block, lds, stream)
               : launch_elem_fwd_v<T, false>(md, sd, tiles, ntiles, block, lds, stream);
}
template <typename T>
int launch_part_fwd(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, int,
                    void* stream) {
    if (ntiles <= 0) return 0;
    launch_timed(k_part_fwd<T>, dim3(ntiles), dim3(block), 0, (hipStream_t)stream, md, sd, tiles);
    return check_launch();
}
template <typename T, bool AIR>
int launch_elem_adj_v(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, size_t lds,
                      void* stream) {
    static size_t allowed = 48 * 1024;
    allow_lds(reinterpret_cast<const void*>(&k_elem_adj<T, AIR>), lds, allowed);
    launch_timed(k_elem_adj<T, AIR>, dim3(ntiles), dim3(block), lds, (hipStream_t)stream, md, sd, tiles);
    return check_launch();
}
template <typename T>
int launch_elem_adj(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, size_t lds,
                    bool air, void* stream) {
    if (ntiles <= 0) return 0;
    return air ? launch_elem_adj_v<T, true>(md, sd, tiles, ntiles, block, lds, stream)
               : launch_elem_adj_v<T, false>(md, sd, tiles, ntiles, block, lds, stream);
}
template <typename T>
int launch_part_adj(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, int,
                    bool air, void* stream) {
    if (ntiles <= 0) return 0;
    if (air)
        launch_timed(k_part_adj<T, true>, dim3(ntiles), dim3(block), 0, (hipStream_t)stream, md, sd, tiles);
    else
        launch_timed(k_part_adj<T, false>, dim3(ntiles), dim3(block), 0, (hipStream_t)stream, md, sd, tiles);
    return check_launch();
}
template <typename T>
int launch_persist(const ModelDev<T>* md, const StepDev<T>* rows, int n_rows, const Tile* etiles, const Tile* ptiles,
                   const int32_t* toff, int n_bodies, int block, size_t lds, void* stream) {
    if constexpr (std::is_same<T, double>::value) {
        // FP32 only: with all four tile passes in one kernel the FP64 build spills
        return (int)hipErrorNotSupported;
    } else {
        static size_t allowed = 48 * 1024;
        if (n_rows <= 0 || n_bodies <= 0) return 0;
        allow_lds(reinterpret_cast<const void*>(&k_persist<T>), lds, allowed);
        hipLaunchKernelGGL(k_persist<T>, dim3(n_bodies), dim3(block), lds, (hipStream_t)stream, md, rows, n_rows,
                           etiles, ptiles, toff);
        return check_launch();
    }
}
template <typename T>
int launch_dual(const ModelDev<T>* md, const StepDev<T>* sd_adj, const StepDev<T>* sd_fwd, const Tile* etiles,
                int n_etiles, const Tile* ptiles, int n_ptiles, int block, int pblock, size_t lds, bool particles,
                bool paired, void* stream) {
    static size_t allowed = 48 * 1024;
    const int nx = 8;  // XCDs: workgroup b runs on XCD b % 8
    const int espan = (n_etiles + nx - 1) / nx * nx, pspan = (n_ptiles + nx - 1) / nx * nx;
    if (!particles) {
        if (n_etiles <= 0) return 0;
        allow_lds(reinterpret_cast<const void*>(&k_elem_dual<T>), lds, allowed);
        launch_timed(k_elem_dual<T>, dim3(paired ? n_etiles : espan + n_etiles), dim3(block), lds, (hipStream_t)stream,
                     md, sd_adj, sd_fwd, etiles, n_etiles, espan, paired ? 1 : 0);
        return check_launch();
    }
    if (n_ptiles <= 0) return 0;
    launch_timed(k_part_dual<T>, dim3(pspan + n_ptiles), dim3(pblock), 0, (hipStream_t)stream, md, sd_adj, ptiles,
                 n_ptiles, pspan, sd_fwd, ptiles);
    return check_launch();
}
int launch_stage_copy(const StageSeg* segs, int n_segs, void* stream) {
    if (n_segs <= 0) return 0;
    hipLaunchKernelGGL(k_stage_copy, dim3(n_segs), dim3(256), 0, (hipStream_t)stream, segs);
    return check_launch();
}
template <typename T>
int launch_mixed(const ModelDev<T>* md, const StepDev<T>* sd, const TileSeg* eseg, int n_eseg, int e_total, int e_grid,
                 const TileSeg* pseg, int n_pseg, int p_total, int p_grid, int dummy_id, int block, size_t lds,
                 void* stream) {
    static size_t allowed = 48 * 1024;
    if (e_grid > 0) {
        allow_lds(reinterpret_cast<const void*>(&k_elem_mixed<T>), lds, allowed);
        hipLaunchKernelGGL(k_elem_mixed<T>, dim3(e_grid), dim3(block), lds, (hipStream_t)stream, md, sd, eseg, n_eseg,
                           e_total, e_grid, dummy_id);
        if (int rc = check_launch()) return rc;
    }
    if (p_grid > 0)
        hipLaunchKernelGGL(k_part_mixed<T>, dim3(p_grid), dim3(block), 0, (hipStream_t)stream, md, sd, pseg, n_pseg,
                           p_total, p_grid, dummy_id);
    return check_launch();
}
template <typename T>
int launch_fill(T* p, int64_t n, T value, void* stream) {
    if (n <= 0) return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, p, n, value);
    return check_launch();
}
template <typename T>
int launch_contact_reduce(const ModelDev<T>* md, const StepDev<T>* sd, int n_bodies, void* stream) {
    const int n = 4 * n_bodies;
    hipLaunchKernelGGL(k_contact_reduce<T>, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, md, sd);
    return check_launch();
}
template <typename T>
int launch_loss(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, int,
                int n_bodies, void* stream) {
    hipLaunchKernelGGL(k_loss_part<T>, dim3(ntiles), dim3(block), 0, (hipStream_t)stream, md, sd, tiles);
    int rc = check_launch();
    if (rc) return rc;
    hipLaunchKernelGGL(k_loss_reduce<T>, dim3((n_bodies + 255) / 256), dim3(256), 0, (hipStream_t)stream, md, sd);
    return check_launch();
}

template <typename T>
int launch_fused_fwd(const ModelDev<T>* md, const StepDev<T>* sd, const int32_t* order, int n_bodies, size_t lds,
                     void* stream) {
    if (n_bodies <= 0) return 0;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused_fwd<T>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(k_fused_fwd<T>, dim3(n_bodies), dim3(FUSED_FWD_BLOCK), lds, (hipStream_t)stream, md, sd, order);
    return check_launch();
}
template <typename T, bool ACT>
int launch_fused_adj_v(const ModelDev<T>* md, const StepDev<T>* sd, const int32_t* order, int n_bodies, size_t lds,
                       void* stream) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused_adj<T, ACT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_fused_adj<T, ACT>), dim3(n_bodies), dim3(FUSED_ADJ_BLOCK), lds, (hipStream_t)stream, md, sd,
                       order);
    return check_launch();
}
template <typename T>
int launch_fused_adj(const ModelDev<T>* md, const StepDev<T>* sd, const int32_t* order, int n_bodies, size_t lds,
                     bool act, void* stream) {
    if (n_bodies <= 0) return 0;
    return act ? launch_fused_adj_v<T, true>(md, sd, order, n_bodies, lds, stream)
               : launch_fused_adj_v<T, false>(md, sd, order, n_bodies, lds, stream);
}

template <typename T>
hipError_t fused_static_lds(bool adjoint, size_t* bytes) {
    *bytes = 0;
    const void* fs[2] = {reinterpret_cast<const void*>(&k_fused_fwd<T>), nullptr};
    if (adjoint) {
        fs[0] = reinterpret_cast<const void*>(&k_fused_adj<T, false>);
        fs[1] = reinterpret_cast<const void*>(&k_fused_adj<T, true>);
    }
    for (const void* f : fs) {
        if (!f) continue;
        hipFuncAttributes a;
        const hipError_t e = hipFuncGetAttributes(&a, f);
        if (e != hipSuccess) return e;
        if (a.sharedSizeBytes > *bytes) *bytes = a.sharedSizeBytes;
    }
    return hipSuccess;
}
template <typename T>
int launch_fused_params(const ModelDev<T>* md, const StepDev<T>* sd, void* stream) {
    hipLaunchKernelGGL(k_fused_params<T>, dim3(1024), dim3(256), 0, (hipStream_t)stream, md, sd);
    return check_launch();
}
template <typename T>
int launch_fused_grads(const ModelDev<T>* md, const StepDev<T>* sd, void* stream) {
    hipLaunchKernelGGL(k_fused_grads<T>, dim3(1024), dim3(256), 0, (hipStream_t)stream, md, sd);
    return check_launch();
}

#define GSIM_INSTANTIATE(T)                                                                                          \
    template int launch_elem_fwd<T>(const ModelDev<T>*, const StepDev<T>*, const Tile*, int, int, size_t, bool, void*); \
    template int launch_part_fwd<T>(const ModelDev<T>*, const StepDev<T>*, const Tile*, int, int, int, void*);     \
    template int launch_elem_adj<T>(const ModelDev<T>*, const StepDev<T>*, const Tile*, int, int, size_t, bool, void*); \
    template int launch_part_adj<T>(const ModelDev<T>*, const StepDev<T>*, const Tile*, int, int, int, bool, void*); \
    template int launch_fill<T>(T*, int64_t, T, void*);                                                             \
    template int launch_persist<T>(const ModelDev<T>*, const StepDev<T>*, int, const Tile*, const Tile*, const int32_t*, \
                                   int, int, size_t, void*);                                                        \
    template int launch_dual<T>(const ModelDev<T>*, const StepDev<T>*, const StepDev<T>*, const Tile*, int, const Tile*, \
                                int, int, int, size_t, bool, bool, void*);                                        \
    template int launch_mixed<T>(const ModelDev<T>*, const StepDev<T>*, const TileSeg*, int, int, int, const TileSeg*, \
                                 int, int, int, int, int, size_t, void*);                                           \
    template int launch_contact_reduce<T>(const ModelDev<T>*, const StepDev<T>*, int, void*);                       \
    template int launch_loss<T>(const ModelDev<T>*, const StepDev<T>*, const Tile*, int, int, int, int, void*);     \
    template int launch_fused_fwd<T>(const ModelDev<T>*, const StepDev<T>*, const int32_t*, int, size_t, void*);     \
    template int launch_fused_adj<T>(const ModelDev<T>*, const StepDev<T>*, const int32_t*, int, size_t, bool, void*); \
    template int launch_fused_params<T>(const ModelDev<T>*, const StepDev<T>*, void*);                               \
    template int launch_fused_grads<T>(const ModelDev<T>*, const StepDev<T>*, void*);                               \
    template hipError_t fused_static_lds<T>(bool, size_t*);

GSIM_INSTANTIATE(float)
GSIM_INSTANTIATE(double)

}  // namespace gsim
