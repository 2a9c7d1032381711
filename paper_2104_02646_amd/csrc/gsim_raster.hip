// Soft silhouette renderer (SoftRas-style; the paper renders its meshes with a
// differentiable soft rasterizer so that losses sit on pixels, Sec. 3 and the
// rendering appendix) and its adjoint, on CDNA4.
//
// Each vertex X is projected by a 3x4 camera matrix P to pixel coordinates
// u = P0.[X,1] / P2.[X,1], v = P1.[X,1] / P2.[X,1].  Triangle j covers pixel p
// (centre (col + 0.5, row + 0.5)) with probability D_j = sigmoid(x_j),
// x_j = +-d_j^2 / sigma (d_j: distance from p to the triangle's edges; + inside);
// the image is I = 1 - prod_j (1 - D_j) = 1 - T with the transmittance
// T = 1 / prod_j (1 + exp(x_j)) (as 1 - sigmoid(x) = 1 / (1 + e^x)).  Terms of
// pixels outside a triangle with d^2 > CUT sigma (D < 1e-6) are dropped.
//
// Adjoint: dI / dx_j = T D_j (prod over the other triangles times D_j (1 - D_j)),
// which needs no division by 1 - D_j, and d(d^2) / d(endpoint) of the nearest edge
// point q = s0 + t (s1 - s0) is -2 (1 - t) (p - q) and -2 t (p - q).
//
// Kernels: projection (one thread per vertex); triangle records (one thread per
// triangle: widened box, corners, orientation, reciprocal edge lengths, and each
// chunk's box); forward (an 8 x 8 pixel tile per workgroup; the records of the
// triangles whose widened box reaches the tile are compacted through LDS in order,
// RCHUNK at a time, and split over the workgroup's RSLICE wavefronts); triangle adjoint
// (16 lanes per triangle over the pixels of its widened box, the transmittance
// recomputed by the forward kernels first); vertex gather (one thread per vertex
// summing its triangle corners in a fixed order, then through the projection).  No
// atomics anywhere: results are bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "gsim.h"
#include "gsim_device.h"
#include "gsim_host.h"

namespace gsim {
namespace {

constexpr int RT = 8;             // pixel tile edge: one wavefront's 8 x 8 pixels
constexpr int RSLICE = 8;         // wavefronts per tile, each over every 8th kept triangle
constexpr int RCHUNK = 512;       // triangles staged per LDS chunk (one per thread)
constexpr int RREC = 16;          // values per triangle record
constexpr int RLANES = 16;        // lanes per triangle in the adjoint
const double RCUT = 13.815510557964274;  // -ln(1e-6)

// Per-triangle record, written once per frame: [0..3] bounding box widened by the
// cut-off distance (xmin, xmax, ymin, ymax); [4..9] screen corners a, b, c;
// [10] orientation (+1, -1, 0 for a degenerate triangle); [11..13] reciprocal
// squared lengths of the edges ab, bc, ca; [14, 15] unused.
template <typename T>
struct RasterArgs {
    const int32_t* tris;   // [nt][3]
    const int32_t* coff;   // [nv + 1] vertex -> corner list
    const int32_t* cent;   // [3 nt] corner = 3 tri + k
    T* uvw;                // [nv][3]: u, v, P2.[X,1]
    T* trans;              // [H][W]
    T* cg;                 // [nt][6] screen-space gradient of each corner
    T* trec;               // [nt][RREC] triangle records
    T* cbox;               // [ceil(nt / RCHUNK)][4] widened box of each chunk of triangles
    int64_t nv, nt;
    int32_t H, W;
    T P[12];
    T isigma, cut;         // 1 / sigma; cut = CUT sigma
};

template <typename T>
struct alignas(16) Rec {
    T v[RREC];
};

template <typename T>
__device__ __forceinline__ T cr2(T ax, T ay, T bx, T by) {
    return ax * by - ay * bx;
}

// Squared distance from p to segment s0 -> s1 (inv: 1 / |s1 - s0|^2) and the
// parameter t of the nearest point.
template <typename T>
__device__ __forceinline__ T seg_d2(T px, T py, T ax, T ay, T bx, T by, T inv, T& t) {
    const T ex = bx - ax, ey = by - ay, wx = px - ax, wy = py - ay;
    t = fmin(fmax((wx * ex + wy * ey) * inv, T(0)), T(1));  // (a zero-length edge: t = 0)
    const T dx = wx - t * ex, dy = wy - t * ey;
    return dx * dx + dy * dy;
}

// Signed scaled distance x = +-d^2 / sigma of pixel p to the triangle of record q;
// returns false when the term is dropped.  edge / t: the nearest edge (0: ab,
// 1: bc, 2: ca; the first minimum) and its parameter.
template <typename T>
__device__ __forceinline__ bool tri_term(T px, T py, const T* q, T isigma, T cut, T& x, int& edge, T& t) {
    const T ax = q[4], ay = q[5], bx = q[6], by = q[7], cx = q[8], cy = q[9], s = q[10];
    const T e0 = s * cr2(bx - ax, by - ay, px - ax, py - ay);
    const T e1 = s * cr2(cx - bx, cy - by, px - bx, py - by);
    const T e2 = s * cr2(ax - cx, ay - cy, px - cx, py - cy);
    const bool inside = s != T(0) && e0 >= T(0) && e1 >= T(0) && e2 >= T(0);
    T t0, t1, t2;
    const T d0 = seg_d2(px, py, ax, ay, bx, by, q[11], t0);
    const T d1 = seg_d2(px, py, bx, by, cx, cy, q[12], t1);
    const T d2 = seg_d2(px, py, cx, cy, ax, ay, q[13], t2);
    T d = d0;
    edge = 0;
    t = t0;
    if (d1 < d) { d = d1; edge = 1; t = t1; }
    if (d2 < d) { d = d2; edge = 2; t = t2; }
    if (!inside && d > cut) return false;
    x = (inside ? d : -d) * isigma;
    return true;
}

__device__ __forceinline__ float sigm(float x) { return 1.f / (1.f + expf(-x)); }
__device__ __forceinline__ double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

template <typename T>
__global__ __launch_bounds__(256) void k_raster_project(RasterArgs<T> A, const T* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.nv) return;
    const V3<T> X = ld3(x, A.nv, i);
    const T n0 = A.P[0] * X.x + A.P[1] * X.y + A.P[2] * X.z + A.P[3];
    const T n1 = A.P[4] * X.x + A.P[5] * X.y + A.P[6] * X.z + A.P[7];
    const T dn = A.P[8] * X.x + A.P[9] * X.y + A.P[10] * X.z + A.P[11];
    A.uvw[3 * i] = n0 / dn;
    A.uvw[3 * i + 1] = n1 / dn;
    A.uvw[3 * i + 2] = dn;
}

// One thread per triangle: its record, and the union of the widened boxes of each
// chunk of RCHUNK triangles (so a tile can skip whole chunks).
template <typename T>
__global__ __launch_bounds__(RCHUNK) void k_raster_tri_prep(RasterArgs<T> A) {
    __shared__ T red[4][RCHUNK];
    const int64_t j = (int64_t)blockIdx.x * RCHUNK + threadIdx.x;
    const T r = sqrt(A.cut);
    T b[4] = {T(INFINITY), T(-INFINITY), T(INFINITY), T(-INFINITY)};
    // a triangle with a corner index outside [0, nv) (possible only with a caller's
    // device-side list, which the host cannot check) is not read: its record keeps an
    // empty box, so it covers no pixel and no chunk box grows for it
    bool valid = j < A.nt;
    int32_t ci[3] = {0, 0, 0};
    if (valid)
        for (int k = 0; k < 3; ++k) {
            ci[k] = A.tris[3 * j + k];
            valid = valid && ci[k] >= 0 && ci[k] < A.nv;
        }
    if (j < A.nt && !valid) {
#pragma unroll
        for (int k = 0; k < RREC; ++k) A.trec[RREC * j + k] = k < 4 ? b[k] : T(0);
    }
    if (valid) {
        T q[RREC];
        for (int k = 0; k < 3; ++k) {
            const int32_t i = ci[k];
            q[4 + 2 * k] = A.uvw[3 * i];
            q[5 + 2 * k] = A.uvw[3 * i + 1];
        }
        const T ax = q[4], ay = q[5], bx = q[6], by = q[7], cx = q[8], cy = q[9];
        b[0] = fmin(fmin(ax, bx), cx) - r;
        b[1] = fmax(fmax(ax, bx), cx) + r;
        b[2] = fmin(fmin(ay, by), cy) - r;
        b[3] = fmax(fmax(ay, by), cy) + r;
        const T area = cr2(bx - ax, by - ay, cx - ax, cy - ay);
        q[0] = b[0];
        q[1] = b[1];
        q[2] = b[2];
        q[3] = b[3];
        q[10] = area > T(0) ? T(1) : (area < T(0) ? T(-1) : T(0));
        q[11] = T(1) / ((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
        q[12] = T(1) / ((cx - bx) * (cx - bx) + (cy - by) * (cy - by));
        q[13] = T(1) / ((ax - cx) * (ax - cx) + (ay - cy) * (ay - cy));
        q[14] = T(0);
        q[15] = T(0);
#pragma unroll
        for (int k = 0; k < RREC; ++k) A.trec[RREC * j + k] = q[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = b[k];
    __syncthreads();
    for (int h = RCHUNK / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + h]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + h]);
            red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + h]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) A.cbox[4 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// One 8 x 8 pixel tile per workgroup of RSLICE wavefronts; writes the
// transmittance and (if not null) the image.  Each chunk of RCHUNK triangle
// records is tested against the tile (its box widened by the cut-off distance) and
// the kept ones are compacted into LDS in triangle order; wavefront w then takes
// kept triangles w, w + RSLICE, ... for all 64 pixels, with the product
// Q_w = prod (1 + exp(x_j)) per pixel (T = 1 / prod_w Q_w, multiplied in wavefront
// order: a fixed order, so results are bitwise repeatable).
template <typename T>
__global__ __launch_bounds__(64 * RSLICE) void k_raster_fwd(RasterArgs<T> A, T* __restrict__ image) {
    __shared__ __align__(16) T rec[RCHUNK][RREC];
    __shared__ T qw[RSLICE][64];
    __shared__ int wcount[RSLICE];
    static_assert(RCHUNK == 64 * RSLICE, "one record per thread per chunk");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = blockIdx.x * RT + (lane & 7), row = blockIdx.y * RT + (lane >> 3);
    const T px = (T)col + T(0.5), py = (T)row + T(0.5);
    // the tile's pixel-centre extent
    const T tx0 = (T)(blockIdx.x * RT) + T(0.5), tx1 = tx0 + T(RT - 1);
    const T ty0 = (T)(blockIdx.y * RT) + T(0.5), ty1 = ty0 + T(RT - 1);
    T Q = T(1);
    for (int64_t c0 = 0; c0 < A.nt; c0 += RCHUNK) {
        // whole chunk out of reach: skip (uniform over the workgroup, before any barrier)
        const T* cb = A.cbox + 4 * (c0 / RCHUNK);
        if ((cb[1] < tx0) | (cb[0] > tx1) | (cb[3] < ty0) | (cb[2] > ty1)) continue;
        const int64_t j = c0 + threadIdx.x;
        T q[RREC];
        bool keep = false;
        if (j < A.nt) {
#pragma unroll
            for (int k = 0; k < RREC; ++k) q[k] = A.trec[RREC * j + k];
            keep = !((q[1] < tx0) | (q[0] > tx1) | (q[3] < ty0) | (q[2] > ty1));
        }
        const unsigned long long m = __ballot(keep);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        __syncthreads();  // the previous chunk's records and counts are no longer read
        if (lane == 0) wcount[wave] = __popcll(m);
        __syncthreads();
        int base = 0, total = 0;
#pragma unroll
        for (int w = 0; w < RSLICE; ++w) {
            base += w < wave ? wcount[w] : 0;
            total += wcount[w];
        }
        if (keep) {
#pragma unroll
            for (int k = 0; k < RREC; ++k) rec[base + before][k] = q[k];
        }
        __syncthreads();
        // whole records through registers, the next one loaded while this one is used
        Rec<T> cur = *(const Rec<T>*)rec[wave < total ? wave : 0];
        for (int k = wave; k < total; k += RSLICE) {
            const int kn = k + RSLICE < total ? k + RSLICE : k;
            const Rec<T> nxt = *(const Rec<T>*)rec[kn];
            const T* r = cur.v;
            if (!((px < r[0]) | (px > r[1]) | (py < r[2]) | (py > r[3]))) {
                T x, t;
                int e;
                if (tri_term(px, py, r, A.isigma, A.cut, x, e, t)) Q = fma(Q, exp(x), Q);  // Q (1 + e^x)
            }
            cur = nxt;
        }
    }
    qw[wave][lane] = Q;
    __syncthreads();
    if (wave == 0 && col < A.W && row < A.H) {
        T P = qw[0][lane];
#pragma unroll
        for (int w = 1; w < RSLICE; ++w) P *= qw[w][lane];
        const T tr = T(1) / P;
        A.trans[(int64_t)row * A.W + col] = tr;
        if (image) image[(int64_t)row * A.W + col] = T(1) - tr;
    }
}

// RLANES lanes per triangle: d <Ibar, I> / d (screen corners) over the pixels of
// its widened box, strided over the lanes, then a butterfly sum over the lanes
// (fixed order).  Needs the transmittance of the same x (the forward runs first).
template <typename T>
__global__ __launch_bounds__(256) void k_raster_tri_adj(RasterArgs<T> A, const T* __restrict__ ibar) {
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = gid / RLANES;
    const int sub = (int)(gid % RLANES);
    const bool live = j < A.nt;  // the lanes of a triangle are all live or all not
    T q[RREC];
#pragma unroll
    for (int k = 0; k < RREC; ++k) q[k] = live ? A.trec[RREC * (live ? j : 0) + k] : T(0);
    // pixel index range whose centres lie inside the widened box, clamped into the
    // image before any conversion to int (far or non-finite corners stay in range)
    const int c0 = (int)fmin(T(A.W), fmax(T(0), ceil(q[0] - T(0.5))));
    const int c1 = (int)fmax(T(-1), fmin(T(A.W - 1), floor(q[1] - T(0.5))));
    const int r0 = (int)fmin(T(A.H), fmax(T(0), ceil(q[2] - T(0.5))));
    const int r1 = (int)fmax(T(-1), fmin(T(A.H - 1), floor(q[3] - T(0.5))));
    const int bw = c1 >= c0 ? c1 - c0 + 1 : 0;
    const int npx = live && r1 >= r0 ? bw * (r1 - r0 + 1) : 0;
    T g[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    for (int p = sub; p < npx; p += RLANES) {
        const int row = r0 + p / bw, col = c0 + p % bw;
        const T px = (T)col + T(0.5), py = (T)row + T(0.5);
        T x, t;
        int e;
        if (!tri_term(px, py, q, A.isigma, A.cut, x, e, t)) continue;
        const int64_t pi = (int64_t)row * A.W + col;
        const T gx = ibar[pi] * A.trans[pi] * sigm(x);
        if (gx == T(0)) continue;
        // x = +-d2 / sigma; d2 = |p - q|^2, q on edge e = (s0, s1)
        const T sgn = x >= T(0) ? T(1) : T(-1);
        const int i0 = e, i1 = e == 2 ? 0 : e + 1;
        const T s0x = q[4 + 2 * i0], s0y = q[5 + 2 * i0], s1x = q[4 + 2 * i1], s1y = q[5 + 2 * i1];
        const T qx = s0x + t * (s1x - s0x), qy = s0y + t * (s1y - s0y);
        const T k = gx * sgn * A.isigma * T(-2);
        const T a = k * (T(1) - t), b = k * t;
        if (e == 0) {
            g[0] += a * (px - qx); g[1] += a * (py - qy); g[2] += b * (px - qx); g[3] += b * (py - qy);
        } else if (e == 1) {
            g[2] += a * (px - qx); g[3] += a * (py - qy); g[4] += b * (px - qx); g[5] += b * (py - qy);
        } else {
            g[4] += a * (px - qx); g[5] += a * (py - qy); g[0] += b * (px - qx); g[1] += b * (py - qy);
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int h = RLANES / 2; h > 0; h >>= 1) g[k] += __shfl_xor(g[k], h);
    if (live && sub == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) A.cg[6 * j + k] = g[k];
    }
}

// One thread per vertex: sum its corners' screen gradients (fixed order), then
// through the projection; adds to xbar (SoA [3][nv]).
template <typename T>
__global__ __launch_bounds__(256) void k_raster_vertex_adj(RasterArgs<T> A, T* __restrict__ xbar) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.nv) return;
    T gu = T(0), gv = T(0);
    for (int32_t k = A.coff[i]; k < A.coff[i + 1]; ++k) {
        const int32_t c = A.cent[k];
        gu += A.cg[6 * (c / 3) + 2 * (c % 3)];
        gv += A.cg[6 * (c / 3) + 2 * (c % 3) + 1];
    }
    const T u = A.uvw[3 * i], v = A.uvw[3 * i + 1], dn = A.uvw[3 * i + 2];
    const T id = T(1) / dn;
#pragma unroll
    for (int k = 0; k < 3; ++k) xbar[k * A.nv + i] += (gu * (A.P[k] - u * A.P[8 + k]) + gv * (A.P[4 + k] - v * A.P[8 + k])) * id;
}

}  // namespace
}  // namespace gsim

using namespace gsim;

// ------------------------------------------------------------------ host ---
struct gsim_raster {
    int dtype = GSIM_F32;
    int64_t nv = 0, nt = 0;
    int H = 0, W = 0;
    char* ws = nullptr;
    size_t o_tris = 0, o_coff = 0, o_cent = 0, o_uvw = 0, o_trans = 0, o_cg = 0, o_trec = 0, o_cbox = 0;
};

namespace {

size_t raster_layout(gsim_raster* R, size_t tsize) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        o = (o + 255) & ~size_t(255);
        const size_t at = o;
        o += std::max<size_t>(bytes, 1);
        return at;
    };
    R->o_tris = take(12 * (size_t)R->nt);
    R->o_coff = take(4 * (size_t)(R->nv + 1));
    R->o_cent = take(12 * (size_t)R->nt);
    R->o_uvw = take(3 * tsize * (size_t)R->nv);
    R->o_trans = take(tsize * (size_t)R->H * R->W);
    R->o_cg = take(6 * tsize * (size_t)R->nt);
    R->o_trec = take(RREC * tsize * (size_t)R->nt);
    R->o_cbox = take(4 * tsize * (size_t)((R->nt + RCHUNK - 1) / RCHUNK));
    return (o + 255) & ~size_t(255);
}

int raster_check(int dtype, int64_t nv, int64_t nt, int H, int W) {
    if (dtype != GSIM_F32 && dtype != GSIM_F64) return fail(GSIM_E_INVALID, "dtype must be GSIM_F32 or GSIM_F64");
    if (nv < 1 || nt < 1 || nt > (int64_t)INT32_MAX / 3 || nv >= INT32_MAX)
        return fail(GSIM_E_INVALID, "n_verts and n_tris must be >= 1 (and below 2^31 / 3 triangles)");
    if (H < 1 || W < 1 || (int64_t)H * W > (int64_t)1 << 28) return fail(GSIM_E_INVALID, "bad image size");
    return GSIM_OK;
}

template <typename T>
RasterArgs<T> raster_args(const gsim_raster* R, const gsim_camera* cam) {
    RasterArgs<T> A;
    std::memset(&A, 0, sizeof A);
    A.tris = (const int32_t*)(R->ws + R->o_tris);
    A.coff = (const int32_t*)(R->ws + R->o_coff);
    A.cent = (const int32_t*)(R->ws + R->o_cent);
    A.uvw = (T*)(R->ws + R->o_uvw);
    A.trans = (T*)(R->ws + R->o_trans);
    A.cg = (T*)(R->ws + R->o_cg);
    A.trec = (T*)(R->ws + R->o_trec);
    A.cbox = (T*)(R->ws + R->o_cbox);
    A.nv = R->nv;
    A.nt = R->nt;
    A.H = R->H;
    A.W = R->W;
    for (int k = 0; k < 12; ++k) A.P[k] = (T)cam->P[k];
    A.isigma = (T)(1.0 / cam->sigma);
    A.cut = (T)(RCUT * cam->sigma);
    return A;
}

int cam_check(const gsim_camera* cam) {
    if (!cam) return fail(GSIM_E_INVALID, "NULL camera");
    if (!(cam->sigma > 0) || !std::isfinite(cam->sigma)) return fail(GSIM_E_INVALID, "sigma must be > 0");
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(cam->P[k])) return fail(GSIM_E_NONFINITE, "camera matrix");
    return GSIM_OK;
}

int raster_cam_check(const gsim_raster* R, const gsim_camera* cam) {
    if (!R || !cam) return fail(GSIM_E_INVALID, "NULL renderer or camera");
    if (!(cam->sigma > 0) || !std::isfinite(cam->sigma)) return fail(GSIM_E_INVALID, "sigma must be > 0");
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(cam->P[k])) return fail(GSIM_E_NONFINITE, "camera matrix");
    return GSIM_OK;
}

template <typename T>
int raster_forward(gsim_raster* R, const gsim_camera* cam, const T* x, T* image, hipStream_t s) {
    RasterArgs<T> A = raster_args<T>(R, cam);
    hipLaunchKernelGGL(k_raster_project<T>, dim3((unsigned)((R->nv + 255) / 256)), dim3(256), 0, s, A, x);
    hipLaunchKernelGGL(k_raster_tri_prep<T>, dim3((unsigned)((R->nt + RCHUNK - 1) / RCHUNK)), dim3(RCHUNK), 0, s, A);
    hipLaunchKernelGGL(k_raster_fwd<T>, dim3((R->W + RT - 1) / RT, (R->H + RT - 1) / RT), dim3(64 * RSLICE), 0, s,
                       A, image);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GSIM_OK : hip_fail(e, "raster forward");
}

template <typename T>
int raster_backward(gsim_raster* R, const gsim_camera* cam, const T* x, const T* ibar, T* xbar, hipStream_t s) {
    int rc = raster_forward<T>(R, cam, x, nullptr, s);  // transmittance and projection of this x
    if (rc) return rc;
    RasterArgs<T> A = raster_args<T>(R, cam);
    hipLaunchKernelGGL(k_raster_tri_adj<T>, dim3((unsigned)((R->nt * RLANES + 255) / 256)), dim3(256), 0, s, A, ibar);
    hipLaunchKernelGGL(k_raster_vertex_adj<T>, dim3((unsigned)((R->nv + 255) / 256)), dim3(256), 0, s, A, xbar);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GSIM_OK : hip_fail(e, "raster backward");
}

// ------------------------------------------- forward without allocation ---
// Scratch of gsim_raster_forward_noalloc: one static device array per GPU (each device
// the library runs on holds its own copy until the process ends).  In host code
// `scratch` names a host-side stand-in, not device memory: its device address is taken
// once per device with hipGetSymbolAddress and only that address is passed on.
static __device__ __align__(256) unsigned char scratch[GSIM_RASTER_SCRATCH_BYTES];

const int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch (looked up on the first call on it).
int scratch_ptr(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(GSIM_E_UNSUPPORTED, "device %d: at most %d devices", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "scratch address");
        g_scratch_ptr[dev] = (char*)p;
    }
    *out = g_scratch_ptr[dev];
    return GSIM_OK;
}

// Offsets of the forward's scratch (projected vertices, transmittance, triangle
// records, chunk boxes) from one base; returns the bytes it needs.
size_t raster_fwd_layout(gsim_raster* R, size_t tsize) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        o = (o + 255) & ~size_t(255);
        const size_t at = o;
        o += std::max<size_t>(bytes, 1);
        return at;
    };
    R->o_uvw = take(3 * tsize * (size_t)R->nv);
    R->o_trans = take(tsize * (size_t)R->H * R->W);
    R->o_trec = take(RREC * tsize * (size_t)R->nt);
    R->o_cbox = take(4 * tsize * (size_t)((R->nt + RCHUNK - 1) / RCHUNK));
    return (o + 255) & ~size_t(255);
}

template <typename T>
int raster_forward_noalloc(gsim_raster* R, const int32_t* d_tris, const gsim_camera* cam, const T* x, T* image,
                           hipStream_t s) {
    RasterArgs<T> A = raster_args<T>(R, cam);
    A.tris = d_tris;  // the caller's device list (coff, cent, cg: only the adjoint uses them)
    A.coff = A.cent = nullptr;
    A.cg = nullptr;
    hipLaunchKernelGGL(k_raster_project<T>, dim3((unsigned)((R->nv + 255) / 256)), dim3(256), 0, s, A, x);
    hipLaunchKernelGGL(k_raster_tri_prep<T>, dim3((unsigned)((R->nt + RCHUNK - 1) / RCHUNK)), dim3(RCHUNK), 0, s, A);
    hipLaunchKernelGGL(k_raster_fwd<T>, dim3((R->W + RT - 1) / RT, (R->H + RT - 1) / RT), dim3(64 * RSLICE), 0, s,
                       A, image);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GSIM_OK : hip_fail(e, "raster forward (no allocation)");
}

}  // namespace

extern "C" {

int gsim_raster_forward_noalloc(int dtype, int64_t n_verts, int64_t n_tris, const int32_t* d_tris, int height,
                                int width, const gsim_camera* camera, const void* x, void* image, void* stream) {
    if (int rc = raster_check(dtype, n_verts, n_tris, height, width)) return rc;
    if (int rc = cam_check(camera)) return rc;
    if (!d_tris || !x || !image) return fail(GSIM_E_INVALID, "NULL triangle list, positions or image");
    gsim_raster R;  // host-side description only (no workspace of its own)
    R.dtype = dtype;
    R.nv = n_verts;
    R.nt = n_tris;
    R.H = height;
    R.W = width;
    const size_t need = raster_fwd_layout(&R, dtype == GSIM_F64 ? 8 : 4);
    if (need > (size_t)GSIM_RASTER_SCRATCH_BYTES)
        return fail(GSIM_E_WORKSPACE, "%lld vertices, %lld triangles at %dx%d need %zu bytes of scratch; the static "
                    "scratch holds %d (use gsim_raster_init with a workspace)", (long long)n_verts, (long long)n_tris,
                    height, width, need, GSIM_RASTER_SCRATCH_BYTES);
    if (int rc = scratch_ptr(&R.ws)) return rc;
    return dtype == GSIM_F64
               ? raster_forward_noalloc<double>(&R, d_tris, camera, (const double*)x, (double*)image, (hipStream_t)stream)
               : raster_forward_noalloc<float>(&R, d_tris, camera, (const float*)x, (float*)image, (hipStream_t)stream);
}

int gsim_raster_sizes(int dtype, int64_t n_verts, int64_t n_tris, int height, int width, size_t* workspace_bytes) {
    if (int rc = raster_check(dtype, n_verts, n_tris, height, width)) return rc;
    if (!workspace_bytes) return fail(GSIM_E_INVALID, "NULL output");
    gsim_raster R;
    R.nv = n_verts;
    R.nt = n_tris;
    R.H = height;
    R.W = width;
    *workspace_bytes = raster_layout(&R, dtype == GSIM_F64 ? 8 : 4);
    return GSIM_OK;
}

int gsim_raster_init(int dtype, int64_t n_verts, int64_t n_tris, const int32_t* tris, int height, int width,
                     void* d_workspace, size_t bytes, void* stream, gsim_raster** out) {
    if (int rc = raster_check(dtype, n_verts, n_tris, height, width)) return rc;
    if (!tris || !d_workspace || !out) return fail(GSIM_E_INVALID, "NULL argument");
    if (((uintptr_t)d_workspace) & 255) return fail(GSIM_E_INVALID, "workspace must be 256-byte aligned");
    for (int64_t k = 0; k < 3 * n_tris; ++k)
        if (tris[k] < 0 || tris[k] >= n_verts) return fail(GSIM_E_TOPOLOGY, "triangle %lld index out of range", (long long)(k / 3));
    gsim_raster* R = new (std::nothrow) gsim_raster();
    if (!R) return fail(GSIM_E_INVALID, "out of host memory");
    R->dtype = dtype;
    R->nv = n_verts;
    R->nt = n_tris;
    R->H = height;
    R->W = width;
    R->ws = (char*)d_workspace;
    const size_t need = raster_layout(R, dtype == GSIM_F64 ? 8 : 4);
    if (bytes < need) {
        delete R;
        return fail(GSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", bytes, need);
    }
    // vertex -> corner lists (corner = 3 tri + k), in increasing corner order
    std::vector<int32_t> coff(n_verts + 1, 0), cent(3 * n_tris);
    for (int64_t k = 0; k < 3 * n_tris; ++k) coff[tris[k] + 1]++;
    for (int64_t i = 0; i < n_verts; ++i) coff[i + 1] += coff[i];
    std::vector<int32_t> fill(coff.begin(), coff.end() - 1);
    for (int64_t k = 0; k < 3 * n_tris; ++k) cent[fill[tris[k]]++] = (int32_t)k;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(R->ws + R->o_tris, tris, 12 * (size_t)n_tris, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(R->ws + R->o_coff, coff.data(), 4 * coff.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(R->ws + R->o_cent, cent.data(), 4 * cent.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete R;
        return hip_fail(e, "raster upload");
    }
    *out = R;
    return GSIM_OK;
}

int gsim_raster_destroy(gsim_raster* R) {
    delete R;
    return GSIM_OK;
}

int gsim_raster_forward(gsim_raster* R, const gsim_camera* cam, const void* x, void* image, void* stream) {
    if (int rc = raster_cam_check(R, cam)) return rc;
    if (!x || !image) return fail(GSIM_E_INVALID, "NULL x or image");
    return R->dtype == GSIM_F64 ? raster_forward<double>(R, cam, (const double*)x, (double*)image, (hipStream_t)stream)
                                : raster_forward<float>(R, cam, (const float*)x, (float*)image, (hipStream_t)stream);
}

int gsim_raster_backward(gsim_raster* R, const gsim_camera* cam, const void* x, const void* image_bar, void* x_bar,
                         void* stream) {
    if (int rc = raster_cam_check(R, cam)) return rc;
    if (!x || !image_bar || !x_bar) return fail(GSIM_E_INVALID, "NULL argument");
    return R->dtype == GSIM_F64
               ? raster_backward<double>(R, cam, (const double*)x, (const double*)image_bar, (double*)x_bar,
                                         (hipStream_t)stream)
               : raster_backward<float>(R, cam, (const float*)x, (const float*)image_bar, (float*)x_bar,
                                        (hipStream_t)stream);
}

}  // extern "C"
