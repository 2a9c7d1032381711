// Rigid bodies (App. A.1 "Rigid bodies" and "Contact"; App. A.2 semi-implicit
// Euler; App. A adjoint) on CDNA4.
//
// State per body s = [x (3), r (4) = (w, i, j, k), v (3), omega (3)]: centre-of-mass
// position, body-to-world orientation quaternion, linear and angular velocity
// (world frame).  Parameters: mass m, body-frame inertia about the centre of mass
// I = [Ixx, Iyy, Izz, Ixy, Ixz, Iyz], contact [k_e, k_d, k_f, mu_f].  One step:
//   a_k = R(r) p_k, y_k = x + a_k, w_k = v + omega x a_k  (body-frame vertices p_k)
//   f_k = ground contact of the point (y_k, w_k), F = sum f_k, tau = sum a_k x f_k
//   Iw = R I R^T, alpha = Iw^-1 (tau - omega x (Iw omega))
//   v+ = v + dt (F / m + g), omega+ = omega + dt alpha, x+ = x + dt v+
//   r+ = normalise(r + dt/2 [0, omega+] (x) r)
//
// One wavefront per body: each lane holds up to RIGID_VPL of the body's vertices in
// registers, the vertex sums F and tau are wave butterfly reductions (every lane ends
// with bitwise the same totals, so every lane integrates the same state and no lane
// waits on another), and the whole rollout is one launch: the forward walks the steps
// storing every state (13 values per body per step), the adjoint walks them back.
// Nothing is shared between waves, so there are no barriers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "gsim.h"
#include "gsim_device.h"
#include "gsim_host.h"

namespace gsim {
namespace {

constexpr int RIGID_WAVES = 4;                              // bodies per workgroup
constexpr int RIGID_VPL = GSIM_RIGID_MAX_VERTS / 64;        // vertices per lane

template <typename T>
struct RigidBodyDev {
    int64_t v0;  // first vertex in the SoA vertex arrays
    int32_t nv;
    int32_t contact_on;
    T dt;
    T g[3];
    T plane[4];
};

template <typename T>
struct RigidArgs {
    const RigidBodyDev<T>* bodies;
    const T* verts;  // SoA [3][n_verts]
    int64_t n_verts;
    int32_t nb, n_steps;
    const T* mass;     // [nb]
    const T* inertia;  // [nb][6]
    const T* contact;  // [nb][4]
    const T* s0;       // forward: [nb][13]
    T* traj;           // [(n_steps + 1)][nb][13]
    const T* sbar;     // adjoint: [nb][13] adjoint of the final state
    T* sbar0;          // adjoint of the initial state
    T* g_mass;
    T* g_inertia;
    T* g_contact;
};

template <typename T, int N>
__device__ __forceinline__ void wave_sum(T v[N]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, 64);
}

template <typename T>
__device__ __forceinline__ void quat_rot(const T q[4], T R[9]) {
    const T w = q[0], a = q[1], b = q[2], c = q[3];
    R[0] = T(1) - T(2) * (b * b + c * c); R[1] = T(2) * (a * b - w * c);        R[2] = T(2) * (a * c + w * b);
    R[3] = T(2) * (a * b + w * c);        R[4] = T(1) - T(2) * (a * a + c * c); R[5] = T(2) * (b * c - w * a);
    R[6] = T(2) * (a * c - w * b);        R[7] = T(2) * (b * c + w * a);        R[8] = T(1) - T(2) * (a * a + b * b);
}

// Adjoint of quat_rot: adds dR/dq^T Rb to qb.
template <typename T>
__device__ __forceinline__ void quat_rot_adjoint(const T q[4], const T Rb[9], T qb[4]) {
    const T w = q[0], a = q[1], b = q[2], c = q[3];
    qb[0] += T(2) * (-c * Rb[1] + b * Rb[2] + c * Rb[3] - a * Rb[5] - b * Rb[6] + a * Rb[7]);
    qb[1] += T(2) * (b * Rb[1] + c * Rb[2] + b * Rb[3] - T(2) * a * Rb[4] - w * Rb[5] + c * Rb[6] + w * Rb[7] -
                     T(2) * a * Rb[8]);
    qb[2] += T(2) * (-T(2) * b * Rb[0] + a * Rb[1] + w * Rb[2] + a * Rb[3] + c * Rb[5] - w * Rb[6] + c * Rb[7] -
                     T(2) * b * Rb[8]);
    qb[3] += T(2) * (-T(2) * c * Rb[0] - w * Rb[1] + a * Rb[2] + w * Rb[3] - T(2) * c * Rb[4] + b * Rb[5] +
                     a * Rb[6] + b * Rb[7]);
}

template <typename T>
__device__ __forceinline__ V3<T> mv(const T M[9], V3<T> v) {
    return mk3(M[0] * v.x + M[1] * v.y + M[2] * v.z, M[3] * v.x + M[4] * v.y + M[5] * v.z,
               M[6] * v.x + M[7] * v.y + M[8] * v.z);
}
template <typename T>
__device__ __forceinline__ V3<T> mtv(const T M[9], V3<T> v) {  // M^T v
    return mk3(M[0] * v.x + M[3] * v.y + M[6] * v.z, M[1] * v.x + M[4] * v.y + M[7] * v.z,
               M[2] * v.x + M[5] * v.y + M[8] * v.z);
}

// Per-body quantities of one step that both the forward and the adjoint use.
template <typename T>
struct RigidFwd {
    T R[9], T1[9], Iw[9], inv[9];
    V3<T> F, tau, L, alpha, vn, wn;
    T q0, qn;
    V3<T> qv;
};

// Vertex forces (this lane's vertices, summed over the wave) and the integration.
template <typename T>
__device__ __forceinline__ void rigid_forward(const RigidBodyDev<T>& B, const V3<T> p[RIGID_VPL], int lane,
                                              const T s[13], T m, const T I[6], const T c[4], RigidFwd<T>& f) {
    const V3<T> x = mk3(s[0], s[1], s[2]);
    const V3<T> v = mk3(s[7], s[8], s[9]);
    const V3<T> w = mk3(s[10], s[11], s[12]);
    quat_rot(&s[3], f.R);
    T acc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if (B.contact_on) {
#pragma unroll
        for (int j = 0; j < RIGID_VPL; ++j) {
            if (lane + 64 * j >= B.nv) break;
            const V3<T> a = mv(f.R, p[j]);
            const V3<T> fk = contact_force(x + a, v + cross(w, a), B.plane, c);
            const V3<T> tk = cross(a, fk);
            acc[0] += fk.x; acc[1] += fk.y; acc[2] += fk.z;
            acc[3] += tk.x; acc[4] += tk.y; acc[5] += tk.z;
        }
        wave_sum<T, 6>(acc);
    }
    f.F = mk3(acc[0], acc[1], acc[2]);
    f.tau = mk3(acc[3], acc[4], acc[5]);
    const T Ib[9] = {I[0], I[3], I[4], I[3], I[1], I[5], I[4], I[5], I[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            f.T1[3 * i + j] = f.R[3 * i] * Ib[j] + f.R[3 * i + 1] * Ib[3 + j] + f.R[3 * i + 2] * Ib[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            f.Iw[3 * i + j] = f.T1[3 * i] * f.R[3 * j] + f.T1[3 * i + 1] * f.R[3 * j + 1] + f.T1[3 * i + 2] * f.R[3 * j + 2];
    const T* M = f.Iw;
    const T det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                  M[2] * (M[3] * M[7] - M[4] * M[6]);
    const T id = T(1) / det;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int r1 = (j + 1) % 3, r2 = (j + 2) % 3, c1 = (i + 1) % 3, c2 = (i + 2) % 3;
            f.inv[3 * i + j] = (M[3 * r1 + c1] * M[3 * r2 + c2] - M[3 * r1 + c2] * M[3 * r2 + c1]) * id;
        }
    f.L = mv(f.Iw, w);
    f.alpha = mv(f.inv, f.tau - cross(w, f.L));
    f.vn = v + (f.F * (T(1) / m) + mk3(B.g[0], B.g[1], B.g[2])) * B.dt;
    f.wn = w + f.alpha * B.dt;
    const V3<T> u = mk3(s[4], s[5], s[6]);
    const T hd = T(0.5) * B.dt;
    f.q0 = s[3] - hd * dot(f.wn, u);
    f.qv = u + (f.wn * s[3] + cross(f.wn, u)) * hd;
    f.qn = gsqrt(f.q0 * f.q0 + dot(f.qv, f.qv));
}

template <typename T>
__device__ __forceinline__ void rigid_next(const T s[13], const RigidFwd<T>& f, T dt, T out[13]) {
    const V3<T> xn = mk3(s[0], s[1], s[2]) + f.vn * dt;
    const T iq = T(1) / f.qn;
    out[0] = xn.x; out[1] = xn.y; out[2] = xn.z;
    out[3] = f.q0 * iq; out[4] = f.qv.x * iq; out[5] = f.qv.y * iq; out[6] = f.qv.z * iq;
    out[7] = f.vn.x; out[8] = f.vn.y; out[9] = f.vn.z;
    out[10] = f.wn.x; out[11] = f.wn.y; out[12] = f.wn.z;
}

template <typename T>
__device__ __forceinline__ void load_body(const RigidArgs<T>& A, const RigidBodyDev<T>& B, int b, int lane,
                                          V3<T> p[RIGID_VPL], T& m, T I[6], T c[4]) {
#pragma unroll
    for (int j = 0; j < RIGID_VPL; ++j) {
        const int k = lane + 64 * j;
        p[j] = k < B.nv ? ld3(A.verts, A.n_verts, B.v0 + k) : zero3<T>();
    }
    m = A.mass[b];
#pragma unroll
    for (int i = 0; i < 6; ++i) I[i] = A.inertia[6 * b + i];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = A.contact[4 * b + i];
}

template <typename T>
__global__ __launch_bounds__(64 * RIGID_WAVES) void k_rigid_fwd(RigidArgs<T> A) {
    const int lane = threadIdx.x & 63;
    // the body index is wave-uniform: keep it (and every address built from it) in
    // scalar registers
    const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * RIGID_WAVES + (int)(threadIdx.x >> 6));
    if (b >= A.nb) return;  // whole wavefronts only: nothing below synchronises waves
    const RigidBodyDev<T> B = A.bodies[b];
    V3<T> p[RIGID_VPL];
    T m, I[6], c[4], s[13];
    load_body(A, B, b, lane, p, m, I, c);
#pragma unroll
    for (int i = 0; i < 13; ++i) s[i] = A.s0[13 * b + i];
    if (lane < 13) A.traj[13 * b + lane] = s[lane];
    for (int t = 0; t < A.n_steps; ++t) {
        RigidFwd<T> f;
        rigid_forward(B, p, lane, s, m, I, c, f);
        T out[13];
        rigid_next(s, f, B.dt, out);
#pragma unroll
        for (int i = 0; i < 13; ++i) s[i] = out[i];
        if (lane < 13) A.traj[(int64_t)(t + 1) * 13 * A.nb + 13 * b + lane] = s[lane];
    }
}

// Reverse of one step at state s for the adjoint sb of the step's output: sb becomes
// the adjoint of s; the parameter adjoints are added to gm, gI, gc.
template <typename T>
__device__ __forceinline__ void rigid_step_adjoint(const RigidBodyDev<T>& B, const V3<T> p[RIGID_VPL], int lane,
                                                   const T s[13], T m, const T I[6], const T c[4], T sb[13], T& gm,
                                                   T gI[6], T gc[4]) {
    RigidFwd<T> f;
    rigid_forward(B, p, lane, s, m, I, c, f);
    const T dt = B.dt, hd = T(0.5) * dt;
    const V3<T> x = mk3(s[0], s[1], s[2]);
    const V3<T> v = mk3(s[7], s[8], s[9]);
    const V3<T> w = mk3(s[10], s[11], s[12]);
    const V3<T> u = mk3(s[4], s[5], s[6]);
    // r+ = q / |q|
    const T iq = T(1) / f.qn;
    const T rn[4] = {f.q0 * iq, f.qv.x * iq, f.qv.y * iq, f.qv.z * iq};
    const T rdot = rn[0] * sb[3] + rn[1] * sb[4] + rn[2] * sb[5] + rn[3] * sb[6];
    const T q0b = (sb[3] - rn[0] * rdot) * iq;
    const V3<T> qvb = mk3(sb[4] - rn[1] * rdot, sb[5] - rn[2] * rdot, sb[6] - rn[3] * rdot) * iq;
    // q0 = r0 - dt/2 wn.u,  qv = u + dt/2 (r0 wn + wn x u)
    T rb[4];
    rb[0] = q0b + hd * dot(f.wn, qvb);
    const V3<T> ub = qvb - f.wn * (hd * q0b) + cross(qvb, f.wn) * hd;
    rb[1] = ub.x; rb[2] = ub.y; rb[3] = ub.z;
    V3<T> wnb = mk3(sb[10], sb[11], sb[12]) + (u * (-q0b) + qvb * s[3] + cross(u, qvb)) * hd;
    // x+ = x + dt v+
    const V3<T> xb0 = mk3(sb[0], sb[1], sb[2]);
    const V3<T> vnb = mk3(sb[7], sb[8], sb[9]) + xb0 * dt;
    // v+ = v + dt (F / m + g)
    const T im = T(1) / m;
    const V3<T> Fb = vnb * (dt * im);
    gm += -dt * im * im * dot(f.F, vnb);
    // omega+ = omega + dt alpha,  alpha = inv h,  h = tau - omega x L,  L = Iw omega
    V3<T> wb = wnb;
    const V3<T> alphab = wnb * dt;
    const V3<T> hb = mtv(f.inv, alphab);
    const V3<T> taub = hb;
    wb -= cross(f.L, hb);
    const V3<T> Lb = cross(w, hb);
    wb += mtv(f.Iw, Lb);
    // Iw-bar = -hb alpha^T + Lb omega^T
    T Iwb[9];
    const T al[3] = {f.alpha.x, f.alpha.y, f.alpha.z}, om[3] = {w.x, w.y, w.z};
    const T hbv[3] = {hb.x, hb.y, hb.z}, Lbv[3] = {Lb.x, Lb.y, Lb.z};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Iwb[3 * i + j] = -hbv[i] * al[j] + Lbv[i] * om[j];
    // Iw = T1 R^T, T1 = R Ib
    T Rb[9], T1b[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T1b[3 * i + k] = Iwb[3 * i] * f.R[k] + Iwb[3 * i + 1] * f.R[3 + k] + Iwb[3 * i + 2] * f.R[6 + k];
            Rb[3 * i + k] = Iwb[i] * f.T1[k] + Iwb[3 + i] * f.T1[3 + k] + Iwb[6 + i] * f.T1[6 + k];
        }
    const T Ib[9] = {I[0], I[3], I[4], I[3], I[1], I[5], I[4], I[5], I[2]};
    T Ibb[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Rb[3 * i + k] += T1b[3 * i] * Ib[3 * k] + T1b[3 * i + 1] * Ib[3 * k + 1] + T1b[3 * i + 2] * Ib[3 * k + 2];
            Ibb[3 * i + k] = f.R[i] * T1b[k] + f.R[3 + i] * T1b[3 + k] + f.R[6 + i] * T1b[6 + k];
        }
    gI[0] += Ibb[0];
    gI[1] += Ibb[4];
    gI[2] += Ibb[8];
    gI[3] += Ibb[1] + Ibb[3];
    gI[4] += Ibb[2] + Ibb[6];
    gI[5] += Ibb[5] + Ibb[7];
    // vertices: F = sum f_k, tau = sum a_k x f_k, f_k = contact(y_k, w_k)
    T acc[22];
#pragma unroll
    for (int i = 0; i < 22; ++i) acc[i] = T(0);
    if (B.contact_on) {
#pragma unroll
        for (int j = 0; j < RIGID_VPL; ++j) {
            if (lane + 64 * j >= B.nv) break;
            const V3<T> a = mv(f.R, p[j]);
            const V3<T> y = x + a, wk = v + cross(w, a);
            // the force itself first (a_k-bar needs it), then its adjoint
            const V3<T> fk = contact_force(y, wk, B.plane, c);
            const V3<T> fkb = Fb + cross(taub, a);
            V3<T> yb = zero3<T>(), wkb = zero3<T>();
            T gck[4] = {T(0), T(0), T(0), T(0)};
            contact_adjoint(y, wk, B.plane, c, fkb, yb, wkb, gck);
            const V3<T> ab = cross(fk, taub) + yb + cross(wkb, w);
            const V3<T> wa = cross(a, wkb);
            acc[0] += yb.x; acc[1] += yb.y; acc[2] += yb.z;
            acc[3] += wkb.x; acc[4] += wkb.y; acc[5] += wkb.z;
            acc[6] += wa.x; acc[7] += wa.y; acc[8] += wa.z;
            const T pk[3] = {p[j].x, p[j].y, p[j].z}, abv[3] = {ab.x, ab.y, ab.z};
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) acc[9 + 3 * i + k] += abv[i] * pk[k];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[18 + k] += gck[k];
        }
        wave_sum<T, 22>(acc);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) Rb[i] += acc[9 + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) gc[k] += acc[18 + k];
    quat_rot_adjoint(&s[3], Rb, rb);
    const V3<T> xb = xb0 + mk3(acc[0], acc[1], acc[2]);
    const V3<T> vb = vnb + mk3(acc[3], acc[4], acc[5]);
    wb += mk3(acc[6], acc[7], acc[8]);
    sb[0] = xb.x; sb[1] = xb.y; sb[2] = xb.z;
    sb[3] = rb[0]; sb[4] = rb[1]; sb[5] = rb[2]; sb[6] = rb[3];
    sb[7] = vb.x; sb[8] = vb.y; sb[9] = vb.z;
    sb[10] = wb.x; sb[11] = wb.y; sb[12] = wb.z;
}

template <typename T>
__global__ __launch_bounds__(64 * RIGID_WAVES) void k_rigid_adj(RigidArgs<T> A) {
    const int lane = threadIdx.x & 63;
    // the body index is wave-uniform: keep it (and every address built from it) in
    // scalar registers
    const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * RIGID_WAVES + (int)(threadIdx.x >> 6));
    if (b >= A.nb) return;
    const RigidBodyDev<T> B = A.bodies[b];
    V3<T> p[RIGID_VPL];
    T m, I[6], c[4], sb[13];
    load_body(A, B, b, lane, p, m, I, c);
#pragma unroll
    for (int i = 0; i < 13; ++i) sb[i] = A.sbar[13 * b + i];
    for (int t = A.n_steps - 1; t >= 0; --t) {
        T s[13];
#pragma unroll
        for (int i = 0; i < 13; ++i) s[i] = A.traj[(int64_t)t * 13 * A.nb + 13 * b + i];
        // this step's parameter adjoints, added to the outputs at once (no
        // accumulator lives across steps)
        T gm = T(0), gI[6] = {T(0), T(0), T(0), T(0), T(0), T(0)}, gc[4] = {T(0), T(0), T(0), T(0)};
        rigid_step_adjoint(B, p, lane, s, m, I, c, sb, gm, gI, gc);
        if (lane == 0) {
            if (A.g_mass) A.g_mass[b] += gm;
            if (A.g_inertia)
#pragma unroll
                for (int i = 0; i < 6; ++i) A.g_inertia[6 * b + i] += gI[i];
            if (A.g_contact && B.contact_on)
#pragma unroll
                for (int i = 0; i < 4; ++i) A.g_contact[4 * b + i] += gc[i];
        }
    }
    if (lane < 13) A.sbar0[13 * b + lane] = sb[lane];
}

// Mean squared distance of each body's world vertices to target points, and (if
// sbar) its gradient with respect to x and r (v, omega entries zero).
template <typename T>
__global__ __launch_bounds__(64 * RIGID_WAVES) void k_rigid_loss(RigidArgs<T> A, const T* __restrict__ state,
                                                                 const T* __restrict__ target, T* __restrict__ loss,
                                                                 T* __restrict__ sbar) {
    const int lane = threadIdx.x & 63;
    // the body index is wave-uniform: keep it (and every address built from it) in
    // scalar registers
    const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * RIGID_WAVES + (int)(threadIdx.x >> 6));
    if (b >= A.nb) return;
    const RigidBodyDev<T> B = A.bodies[b];
    T s[13], R[9];
#pragma unroll
    for (int i = 0; i < 13; ++i) s[i] = state[13 * b + i];
    quat_rot(&s[3], R);
    const V3<T> x = mk3(s[0], s[1], s[2]);
    T acc[13];
#pragma unroll
    for (int i = 0; i < 13; ++i) acc[i] = T(0);
#pragma unroll
    for (int j = 0; j < RIGID_VPL; ++j) {
        const int k = lane + 64 * j;
        if (k >= B.nv) break;
        const V3<T> pk = ld3(A.verts, A.n_verts, B.v0 + k);
        const int64_t q = 3 * (B.v0 + k);  // target is [n_verts][3]
        const V3<T> d = x + mv(R, pk) - mk3(target[q], target[q + 1], target[q + 2]);
        acc[0] += dot(d, d);
        acc[1] += d.x; acc[2] += d.y; acc[3] += d.z;
        const T dv[3] = {d.x, d.y, d.z}, pv[3] = {pk.x, pk.y, pk.z};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[4 + 3 * i + q] += dv[i] * pv[q];
    }
    wave_sum<T, 13>(acc);
    const T inv = T(1) / (T)B.nv;
    if (lane == 0) loss[b] = acc[0] * inv;
    if (sbar) {
        T Rb[9], rb[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int i = 0; i < 9; ++i) Rb[i] = T(2) * inv * acc[4 + i];
        quat_rot_adjoint(&s[3], Rb, rb);
        T out[13] = {T(2) * inv * acc[1], T(2) * inv * acc[2], T(2) * inv * acc[3], rb[0], rb[1], rb[2], rb[3],
                     T(0), T(0), T(0), T(0), T(0), T(0)};
        if (lane < 13) sbar[13 * b + lane] = out[lane];
    }
}

}  // namespace
}  // namespace gsim

using namespace gsim;

// ------------------------------------------------------------------ host ---
struct gsim_rigid {
    int dtype = GSIM_F32;
    int nb = 0;
    int64_t n_verts = 0;
    char* ws = nullptr;
    size_t bodies_off = 0, verts_off = 0;
};

namespace {

size_t rigid_align(size_t o) { return (o + 255) & ~size_t(255); }

int rigid_check_desc(const gsim_rigid_desc* d, int64_t* n_verts) {
    if (!d) return fail(GSIM_E_INVALID, "NULL description");
    if (d->dtype != GSIM_F32 && d->dtype != GSIM_F64) return fail(GSIM_E_INVALID, "dtype must be GSIM_F32 or GSIM_F64");
    if (d->n_bodies < 1) return fail(GSIM_E_INVALID, "n_bodies must be >= 1");
    if (!d->vert_off || !d->verts || !d->dt || !d->gravity) return fail(GSIM_E_INVALID, "NULL array in the description");
    if (d->vert_off[0] != 0) return fail(GSIM_E_INVALID, "vert_off[0] must be 0");
    for (int b = 0; b < d->n_bodies; ++b) {
        const int64_t nv = d->vert_off[b + 1] - d->vert_off[b];
        if (nv < 1 || nv > GSIM_RIGID_MAX_VERTS)
            return fail(GSIM_E_UNSUPPORTED, "body %d has %lld vertices (1..%d)", b, (long long)nv, GSIM_RIGID_MAX_VERTS);
        if (!(d->dt[b] > 0) || !std::isfinite(d->dt[b])) return fail(GSIM_E_INVALID, "dt of body %d must be > 0", b);
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(d->gravity[3 * b + k])) return fail(GSIM_E_NONFINITE, "gravity of body %d", b);
        if (d->ground) {
            const double* pl = &d->ground[4 * b];
            const double nn = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
            if (!(nn > 0) || !std::isfinite(nn) || !std::isfinite(pl[3])) return fail(GSIM_E_INVALID, "plane of body %d", b);
        }
    }
    *n_verts = d->vert_off[d->n_bodies];
    for (int64_t i = 0; i < 3 * *n_verts; ++i)
        if (!std::isfinite(d->verts[i])) return fail(GSIM_E_NONFINITE, "vertex %lld is not finite", (long long)(i / 3));
    return GSIM_OK;
}

template <typename T>
size_t rigid_bytes(int nb, int64_t n_verts, size_t* bodies_off, size_t* verts_off) {
    size_t o = 0;
    *bodies_off = o;
    o = rigid_align(o + sizeof(RigidBodyDev<T>) * nb);
    *verts_off = o;
    o = rigid_align(o + 3 * sizeof(T) * std::max<int64_t>(n_verts, 1));
    return o;
}

template <typename T>
int rigid_upload(const gsim_rigid_desc* d, gsim_rigid* R, hipStream_t s) {
    std::vector<RigidBodyDev<T>> bodies(R->nb);
    for (int b = 0; b < R->nb; ++b) {
        RigidBodyDev<T>& B = bodies[b];
        std::memset(&B, 0, sizeof B);
        B.v0 = d->vert_off[b];
        B.nv = (int32_t)(d->vert_off[b + 1] - d->vert_off[b]);
        B.contact_on = d->contact_on ? (d->contact_on[b] ? 1 : 0) : 0;
        B.dt = (T)d->dt[b];
        for (int k = 0; k < 3; ++k) B.g[k] = (T)d->gravity[3 * b + k];
        double pl[4] = {0.0, 1.0, 0.0, 0.0};
        if (d->ground)
            for (int k = 0; k < 4; ++k) pl[k] = d->ground[4 * b + k];
        const double nn = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
        for (int k = 0; k < 4; ++k) B.plane[k] = (T)(pl[k] / nn);
    }
    std::vector<T> verts(3 * std::max<int64_t>(R->n_verts, 1), T(0));
    for (int64_t i = 0; i < R->n_verts; ++i)
        for (int k = 0; k < 3; ++k) verts[k * R->n_verts + i] = (T)d->verts[3 * i + k];
    hipError_t e = hipMemcpyAsync(R->ws + R->bodies_off, bodies.data(), sizeof(RigidBodyDev<T>) * R->nb,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(R->ws + R->verts_off, verts.data(), verts.size() * sizeof(T), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GSIM_OK : hip_fail(e, "rigid upload");
}

template <typename T>
RigidArgs<T> rigid_args(const gsim_rigid* R, const gsim_rigid_params* p, int n_steps) {
    RigidArgs<T> A;
    std::memset(&A, 0, sizeof A);
    A.bodies = reinterpret_cast<const RigidBodyDev<T>*>(R->ws + R->bodies_off);
    A.verts = reinterpret_cast<const T*>(R->ws + R->verts_off);
    A.n_verts = R->n_verts;
    A.nb = R->nb;
    A.n_steps = n_steps;
    if (p) {
        A.mass = (const T*)p->mass;
        A.inertia = (const T*)p->inertia;
        A.contact = (const T*)p->contact;
    }
    return A;
}

int rigid_check_params(const gsim_rigid* R, const gsim_rigid_params* p, int n_steps) {
    if (!R) return fail(GSIM_E_INVALID, "NULL rigid model");
    if (!p || !p->mass || !p->inertia || !p->contact) return fail(GSIM_E_INVALID, "mass, inertia and contact are required");
    if (n_steps < 0) return fail(GSIM_E_INVALID, "n_steps must be >= 0");
    return GSIM_OK;
}

int rigid_launched(const char* what) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GSIM_OK : hip_fail(e, what);
}

}  // namespace

extern "C" {

int gsim_rigid_sizes(const gsim_rigid_desc* desc, size_t* workspace_bytes) {
    int64_t nv = 0;
    if (int rc = rigid_check_desc(desc, &nv)) return rc;
    if (!workspace_bytes) return fail(GSIM_E_INVALID, "NULL output");
    size_t a, b;
    *workspace_bytes = desc->dtype == GSIM_F64 ? rigid_bytes<double>(desc->n_bodies, nv, &a, &b)
                                                : rigid_bytes<float>(desc->n_bodies, nv, &a, &b);
    return GSIM_OK;
}

int gsim_rigid_init(const gsim_rigid_desc* desc, void* d_workspace, size_t bytes, void* stream, gsim_rigid** out) {
    int64_t nv = 0;
    if (int rc = rigid_check_desc(desc, &nv)) return rc;
    if (!d_workspace || !out) return fail(GSIM_E_INVALID, "NULL workspace or output");
    if (((uintptr_t)d_workspace) & 255) return fail(GSIM_E_INVALID, "workspace must be 256-byte aligned");
    gsim_rigid* R = new (std::nothrow) gsim_rigid();
    if (!R) return fail(GSIM_E_INVALID, "out of host memory");
    R->dtype = desc->dtype;
    R->nb = desc->n_bodies;
    R->n_verts = nv;
    R->ws = (char*)d_workspace;
    const size_t need = desc->dtype == GSIM_F64 ? rigid_bytes<double>(R->nb, nv, &R->bodies_off, &R->verts_off)
                                                : rigid_bytes<float>(R->nb, nv, &R->bodies_off, &R->verts_off);
    if (bytes < need) {
        delete R;
        return fail(GSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", bytes, need);
    }
    const int rc = desc->dtype == GSIM_F64 ? rigid_upload<double>(desc, R, (hipStream_t)stream)
                                           : rigid_upload<float>(desc, R, (hipStream_t)stream);
    if (rc) {
        delete R;
        return rc;
    }
    *out = R;
    return GSIM_OK;
}

int gsim_rigid_destroy(gsim_rigid* R) {
    delete R;
    return GSIM_OK;
}

int gsim_rigid_rollout(gsim_rigid* R, const gsim_rigid_params* p, const void* s0, int n_steps, void* traj,
                       void* stream) {
    if (int rc = rigid_check_params(R, p, n_steps)) return rc;
    if (!s0 || !traj) return fail(GSIM_E_INVALID, "NULL state or trajectory");
    const dim3 grid((R->nb + RIGID_WAVES - 1) / RIGID_WAVES), block(64 * RIGID_WAVES);
    if (R->dtype == GSIM_F64) {
        RigidArgs<double> A = rigid_args<double>(R, p, n_steps);
        A.s0 = (const double*)s0;
        A.traj = (double*)traj;
        hipLaunchKernelGGL(k_rigid_fwd<double>, grid, block, 0, (hipStream_t)stream, A);
    } else {
        RigidArgs<float> A = rigid_args<float>(R, p, n_steps);
        A.s0 = (const float*)s0;
        A.traj = (float*)traj;
        hipLaunchKernelGGL(k_rigid_fwd<float>, grid, block, 0, (hipStream_t)stream, A);
    }
    return rigid_launched("rigid rollout");
}

int gsim_rigid_loss(gsim_rigid* R, const void* state, const void* target, void* loss, void* state_bar, void* stream) {
    if (!R || !state || !target || !loss) return fail(GSIM_E_INVALID, "NULL argument");
    const dim3 grid((R->nb + RIGID_WAVES - 1) / RIGID_WAVES), block(64 * RIGID_WAVES);
    if (R->dtype == GSIM_F64)
        hipLaunchKernelGGL(k_rigid_loss<double>, grid, block, 0, (hipStream_t)stream, rigid_args<double>(R, nullptr, 0),
                           (const double*)state, (const double*)target, (double*)loss, (double*)state_bar);
    else
        hipLaunchKernelGGL(k_rigid_loss<float>, grid, block, 0, (hipStream_t)stream, rigid_args<float>(R, nullptr, 0),
                           (const float*)state, (const float*)target, (float*)loss, (float*)state_bar);
    return rigid_launched("rigid loss");
}

int gsim_rigid_rollout_backward(gsim_rigid* R, const gsim_rigid_params* p, const void* traj, int n_steps,
                                const void* adj_final, void* adj_init, const gsim_rigid_grads* g, void* stream) {
    if (int rc = rigid_check_params(R, p, n_steps)) return rc;
    if (!traj || !adj_final || !adj_init) return fail(GSIM_E_INVALID, "NULL trajectory or adjoint");
    if (adj_final == adj_init) return fail(GSIM_E_INVALID, "adj_final and adj_init must not alias");
    const dim3 grid((R->nb + RIGID_WAVES - 1) / RIGID_WAVES), block(64 * RIGID_WAVES);
    if (R->dtype == GSIM_F64) {
        RigidArgs<double> A = rigid_args<double>(R, p, n_steps);
        A.traj = (double*)traj;
        A.sbar = (const double*)adj_final;
        A.sbar0 = (double*)adj_init;
        if (g) {
            A.g_mass = (double*)g->mass;
            A.g_inertia = (double*)g->inertia;
            A.g_contact = (double*)g->contact;
        }
        hipLaunchKernelGGL(k_rigid_adj<double>, grid, block, 0, (hipStream_t)stream, A);
    } else {
        RigidArgs<float> A = rigid_args<float>(R, p, n_steps);
        A.traj = (float*)traj;
        A.sbar = (const float*)adj_final;
        A.sbar0 = (float*)adj_init;
        if (g) {
            A.g_mass = (float*)g->mass;
            A.g_inertia = (float*)g->inertia;
            A.g_contact = (float*)g->contact;
        }
        hipLaunchKernelGGL(k_rigid_adj<float>, grid, block, 0, (hipStream_t)stream, A);
    }
    return rigid_launched("rigid adjoint");
}

}  // extern "C"
