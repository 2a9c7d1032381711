// Open-loop actuation controller (App. "MPC controller architecture"; Sec. 5.3):
// N phase-shifted sinusoids of the simulation time -> one bias-free fully
// connected layer -> tanh, one actuation per output element per step.
//
//   s_k(t)    = sin(omega (t0 + t) dt + 2 pi k / N)
//   act[t][e] = scale tanh(sum_k W[k][e] s_k(t))
//
// The N signals share one frequency and differ only in phase, so
//   sum_k W[k][e] s_k(t) = A_e sin(omega tau) + B_e cos(omega tau),
//   A_e = sum_k W[k][e] cos(2 pi k / N),   B_e = sum_k W[k][e] sin(2 pi k / N)
// (sin(x + p) = sin x cos p + cos x sin p): each thread forms its element's A, B
// once and then spends two FMAs per step on the layer.  The backward accumulates
// the two sums  sum_t zbar_t sin(omega tau_t)  and  sum_t zbar_t cos(omega tau_t)
// and maps them back to the N weights with the same phase table.
//
// Both kernels stream: one thread per output element walks the steps, so every
// row access of act / act_grad is one coalesced 1 KB (FP32) wavefront access; the
// (sin, cos) table of a chunk of steps is computed once per workgroup (FP64,
// rounded to the dtype) into LDS and read as broadcasts.  The backward issues the
// loads of CTRL_BATCH steps before using any of them, so each wave keeps several
// HBM reads in flight.  Forward: reads W once, writes n_steps rows.  Backward:
// recomputes the layer from W (cheaper than re-reading act), reads n_steps rows of
// act_grad, and adds its N sums per element to W_grad.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gsim.h"
#include "gsim_host.h"

namespace {

constexpr int CTRL_BLOCK = 256;
constexpr int CTRL_CHUNK = 128;  // steps per LDS table
constexpr int CTRL_BATCH = 8;    // backward: act_grad loads issued together
constexpr int MAXN = GSIM_CTRL_MAX_SIGNALS;

struct CtrlArgs {
    int n_signals;
    double omega, dt, scale;
    int64_t n, t0, n_steps;
};

template <typename T>
struct SC {
    T s, c;
};

// (sin, cos) of omega tau for steps tc .. tc + CTRL_CHUNK - 1 of the call.
template <typename T>
__device__ void ctrl_table(const CtrlArgs& a, int64_t tc, SC<T>* tab) {
    for (int t = threadIdx.x; t < CTRL_CHUNK; t += blockDim.x) {
        const double x = a.omega * ((double)(a.t0 + tc + t) * a.dt);
        tab[t].s = (T)sin(x);
        tab[t].c = (T)cos(x);
    }
}

// Phase table cos / sin(2 pi k / N) (FP64 rounded to T) into LDS, then this
// thread's A, B from its weights.  Contains a barrier: every thread calls it.
template <typename T>
__device__ void ctrl_coeffs(const CtrlArgs& a, const T* __restrict__ W, int64_t e, bool live, T* cp, T* sp, T& A,
                            T& B) {
    const double two_pi = 6.283185307179586476925287;
    if (threadIdx.x < a.n_signals) {
        const double p = two_pi * (double)threadIdx.x / (double)a.n_signals;
        cp[threadIdx.x] = (T)cos(p);
        sp[threadIdx.x] = (T)sin(p);
    }
    __syncthreads();
    A = T(0);
    B = T(0);
#pragma unroll
    for (int k = 0; k < MAXN; ++k)
        if (live && k < a.n_signals) {
            const T w = W[(int64_t)k * a.n + e];
            A += w * cp[k];
            B += w * sp[k];
        }
}

template <typename T>
__global__ __launch_bounds__(CTRL_BLOCK) void k_ctrl_fwd(CtrlArgs a, const T* __restrict__ W, T* __restrict__ act) {
    __shared__ SC<T> tab[CTRL_CHUNK];
    __shared__ T cp[MAXN], sp[MAXN];
    const int64_t e = (int64_t)blockIdx.x * CTRL_BLOCK + threadIdx.x;
    const bool live = e < a.n;
    const T scale = (T)a.scale;
    T A, B;
    ctrl_coeffs<T>(a, W, e, live, cp, sp, A, B);
    for (int64_t tc = 0; tc < a.n_steps; tc += CTRL_CHUNK) {
        __syncthreads();  // the previous chunk's table is no longer read
        ctrl_table<T>(a, tc, tab);
        __syncthreads();
        const int nt = (int)(a.n_steps - tc < CTRL_CHUNK ? a.n_steps - tc : CTRL_CHUNK);
        if (live)
            for (int t = 0; t < nt; ++t) {
                const SC<T> q = tab[t];
                act[(tc + t) * a.n + e] = scale * tanh(A * q.s + B * q.c);
            }
    }
}

template <typename T>
__global__ __launch_bounds__(CTRL_BLOCK) void k_ctrl_bwd(CtrlArgs a, const T* __restrict__ W,
                                                         const T* __restrict__ g, T* __restrict__ gW) {
    __shared__ SC<T> tab[CTRL_CHUNK];
    __shared__ T cp[MAXN], sp[MAXN];
    const int64_t e = (int64_t)blockIdx.x * CTRL_BLOCK + threadIdx.x;
    const bool live = e < a.n;
    const T scale = (T)a.scale;
    T A, B;
    ctrl_coeffs<T>(a, W, e, live, cp, sp, A, B);
    T gA = T(0), gB = T(0);
    for (int64_t tc = 0; tc < a.n_steps; tc += CTRL_CHUNK) {
        __syncthreads();
        ctrl_table<T>(a, tc, tab);
        __syncthreads();
        const int nt = (int)(a.n_steps - tc < CTRL_CHUNK ? a.n_steps - tc : CTRL_CHUNK);
        if (live)
            for (int t0 = 0; t0 < nt; t0 += CTRL_BATCH) {
                T gv[CTRL_BATCH];
#pragma unroll
                for (int j = 0; j < CTRL_BATCH; ++j)
                    gv[j] = t0 + j < nt ? g[(tc + t0 + j) * a.n + e] : T(0);
#pragma unroll
                for (int j = 0; j < CTRL_BATCH; ++j)
                    if (t0 + j < nt) {
                        const SC<T> q = tab[t0 + j];
                        const T y = tanh(A * q.s + B * q.c);
                        const T dz = gv[j] * scale * (T(1) - y * y);
                        gA += dz * q.s;
                        gB += dz * q.c;
                    }
            }
    }
    if (live)
#pragma unroll
        for (int k = 0; k < MAXN; ++k)
            if (k < a.n_signals) gW[(int64_t)k * a.n + e] += gA * cp[k] + gB * sp[k];
}

int check_ctrl(int dtype, const gsim_controller* c, int64_t n, int64_t t0, int64_t n_steps, CtrlArgs& a) {
    if (dtype != GSIM_F32 && dtype != GSIM_F64) return gsim::fail(GSIM_E_INVALID, "dtype must be GSIM_F32 or GSIM_F64");
    if (!c) return gsim::fail(GSIM_E_INVALID, "NULL controller");
    if (c->n_signals < 1 || c->n_signals > MAXN)
        return gsim::fail(GSIM_E_INVALID, "n_signals must be in [1, %d]", MAXN);
    if (n < 0 || t0 < 0 || n_steps < 0) return gsim::fail(GSIM_E_INVALID, "n, t0 and n_steps must be >= 0");
    if (!std::isfinite(c->omega) || !std::isfinite(c->dt) || !std::isfinite(c->scale))
        return gsim::fail(GSIM_E_INVALID, "omega, dt and scale must be finite");
    a.n_signals = c->n_signals;
    a.omega = c->omega;
    a.dt = c->dt;
    a.scale = c->scale;
    a.n = n;
    a.t0 = t0;
    a.n_steps = n_steps;
    return GSIM_OK;
}

int launched(const char* what) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GSIM_OK : gsim::hip_fail(e, what);
}

}  // namespace

extern "C" {

int gsim_controller_forward(int dtype, const gsim_controller* ctrl, const void* W, int64_t n, int64_t t0,
                            int64_t n_steps, void* act, void* stream) {
    CtrlArgs a;
    int rc = check_ctrl(dtype, ctrl, n, t0, n_steps, a);
    if (rc) return rc;
    if (n == 0 || n_steps == 0) return GSIM_OK;
    if (!W || !act) return gsim::fail(GSIM_E_INVALID, "NULL W or act");
    const dim3 grid((unsigned)((n + CTRL_BLOCK - 1) / CTRL_BLOCK));
    if (dtype == GSIM_F32)
        hipLaunchKernelGGL(k_ctrl_fwd<float>, grid, dim3(CTRL_BLOCK), 0, (hipStream_t)stream, a, (const float*)W,
                           (float*)act);
    else
        hipLaunchKernelGGL(k_ctrl_fwd<double>, grid, dim3(CTRL_BLOCK), 0, (hipStream_t)stream, a, (const double*)W,
                           (double*)act);
    return launched("controller forward launch");
}

int gsim_controller_backward(int dtype, const gsim_controller* ctrl, const void* W, const void* act_grad, int64_t n,
                             int64_t t0, int64_t n_steps, void* W_grad, void* stream) {
    CtrlArgs a;
    int rc = check_ctrl(dtype, ctrl, n, t0, n_steps, a);
    if (rc) return rc;
    if (n == 0 || n_steps == 0) return GSIM_OK;
    if (!W || !act_grad || !W_grad) return gsim::fail(GSIM_E_INVALID, "NULL W, act_grad or W_grad");
    const dim3 grid((unsigned)((n + CTRL_BLOCK - 1) / CTRL_BLOCK));
    if (dtype == GSIM_F32)
        hipLaunchKernelGGL(k_ctrl_bwd<float>, grid, dim3(CTRL_BLOCK), 0, (hipStream_t)stream, a, (const float*)W,
                           (const float*)act_grad, (float*)W_grad);
    else
        hipLaunchKernelGGL(k_ctrl_bwd<double>, grid, dim3(CTRL_BLOCK), 0, (hipStream_t)stream, a, (const double*)W,
                           (const double*)act_grad, (double*)W_grad);
    return launched("controller backward launch");
}

}  // extern "C"
