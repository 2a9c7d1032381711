// Open-loop actuation controller (App. "MPC controller architecture"; Sec. 5.3):
// N phase-shifted sinusoids of the simulation time -> one bias-free fully
// connected layer -> tanh, one actuation per output element per step.
//
//   s_k(t)    = sin(omega (t0 + t) dt + 2 pi k / N)
//   act[t][e] = scale tanh(sum_k W[k][e] s_k(t))
//
// Both kernels are streaming and HBM-bound: one thread per output element keeps
// its N weights in registers and walks the steps, so every row access of act /
// act_grad is one coalesced 1 KB (FP32) wavefront access; the signal table of a
// chunk of steps is computed once per workgroup into LDS and read as broadcasts.
// Forward: reads W once, writes n_steps rows.  Backward: recomputes the layer
// from W (cheaper than re-reading act), reads n_steps rows of act_grad, and adds
// its N sums per element to W_grad.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gsim.h"
#include "gsim_host.h"

namespace {

constexpr int CTRL_BLOCK = 256;
constexpr int CTRL_CHUNK = 64;  // steps per LDS signal table
constexpr int MAXN = GSIM_CTRL_MAX_SIGNALS;

struct CtrlArgs {
    int n_signals;
    double omega, dt, scale;
    int64_t n, t0, n_steps;
};

// s[t][k] for steps tc .. tc + CTRL_CHUNK - 1 of the call (FP64, rounded to T).
template <typename T>
__device__ void ctrl_signals(const CtrlArgs& a, int64_t tc, T (*s)[MAXN]) {
    const double two_pi = 6.283185307179586476925287;
    for (int i = threadIdx.x; i < CTRL_CHUNK * a.n_signals; i += blockDim.x) {
        const int t = i / a.n_signals, k = i - t * a.n_signals;
        const double tau = (double)(a.t0 + tc + t) * a.dt;
        s[t][k] = (T)sin(a.omega * tau + two_pi * (double)k / (double)a.n_signals);
    }
}

template <typename T>
__global__ __launch_bounds__(CTRL_BLOCK) void k_ctrl_fwd(CtrlArgs a, const T* __restrict__ W, T* __restrict__ act) {
    __shared__ T s[CTRL_CHUNK][MAXN];
    const int64_t e = (int64_t)blockIdx.x * CTRL_BLOCK + threadIdx.x;
    const bool live = e < a.n;
    const int N = a.n_signals;
    const T scale = (T)a.scale;
    T w[MAXN];
#pragma unroll
    for (int k = 0; k < MAXN; ++k) w[k] = (live && k < N) ? W[(int64_t)k * a.n + e] : T(0);
    for (int64_t tc = 0; tc < a.n_steps; tc += CTRL_CHUNK) {
        __syncthreads();  // the previous chunk's table is no longer read
        ctrl_signals<T>(a, tc, s);
        __syncthreads();
        const int nt = (int)(a.n_steps - tc < CTRL_CHUNK ? a.n_steps - tc : CTRL_CHUNK);
        if (live)
            for (int t = 0; t < nt; ++t) {
                T z = T(0);
#pragma unroll
                for (int k = 0; k < MAXN; ++k)
                    if (k < N) z += w[k] * s[t][k];
                act[(tc + t) * a.n + e] = scale * tanh(z);
            }
    }
}

template <typename T>
__global__ __launch_bounds__(CTRL_BLOCK) void k_ctrl_bwd(CtrlArgs a, const T* __restrict__ W,
                                                         const T* __restrict__ g, T* __restrict__ gW) {
    __shared__ T s[CTRL_CHUNK][MAXN];
    const int64_t e = (int64_t)blockIdx.x * CTRL_BLOCK + threadIdx.x;
    const bool live = e < a.n;
    const int N = a.n_signals;
    const T scale = (T)a.scale;
    T w[MAXN], acc[MAXN];
#pragma unroll
    for (int k = 0; k < MAXN; ++k) {
        w[k] = (live && k < N) ? W[(int64_t)k * a.n + e] : T(0);
        acc[k] = T(0);
    }
    for (int64_t tc = 0; tc < a.n_steps; tc += CTRL_CHUNK) {
        __syncthreads();
        ctrl_signals<T>(a, tc, s);
        __syncthreads();
        const int nt = (int)(a.n_steps - tc < CTRL_CHUNK ? a.n_steps - tc : CTRL_CHUNK);
        if (live)
            for (int t = 0; t < nt; ++t) {
                T z = T(0);
#pragma unroll
                for (int k = 0; k < MAXN; ++k)
                    if (k < N) z += w[k] * s[t][k];
                const T y = tanh(z);
                const T dz = g[(tc + t) * a.n + e] * scale * (T(1) - y * y);
#pragma unroll
                for (int k = 0; k < MAXN; ++k)
                    if (k < N) acc[k] += dz * s[t][k];
            }
    }
    if (live)
#pragma unroll
        for (int k = 0; k < MAXN; ++k)
            if (k < N) gW[(int64_t)k * a.n + e] += acc[k];
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
