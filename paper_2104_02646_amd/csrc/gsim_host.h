// Host-side objects of libgsim shared by the C-ABI runtime (gsim_api.cpp) and
// the serving engine (gsim_engine.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "gsim.h"
#include "gsim_internal.h"

// ------------------------------------------------------------------ plan ---
struct gsim_plan {
    int dtype = 32;
    int nb = 0;
    int64_t np = 0, ne = 0, nt = 0, nh = 0, nslot = 0;
    std::vector<int64_t> poff, eoff, toff, hoff;   // per-body ranges
    std::vector<int32_t> tet_idx;                  // SoA [4][ne]
    std::vector<double> tet_dinv, tet_vol;         // SoA [9][ne], [ne]
    std::vector<int32_t> tri_idx;                  // [3][nt]
    std::vector<double> tri_dinv, tri_area;        // [4][nt], [nt]
    std::vector<int32_t> hin_idx;                  // [4][nh]
    std::vector<double> hin_phi0;                  // [nh]
    // two-pass element tiles (see build_tiles): tiles in plan order, corner codes
    // per kind, per-tile-particle index / corner run / partial slot
    std::vector<gsim::Tile> etiles;
    std::vector<uint32_t> tet_code, tri_code, hin_code;  // SoA [corners][n]
    std::vector<int32_t> tp_id, tp_run, tp_slot;
    int tile_elems = gsim::ETILE;                  // elements per two-pass element tile
    int64_t etile_words[2] = {0, 0};               // largest tile's LDS words, forward / adjoint
    std::vector<int32_t> gbase;                    // [n_slices] sliced-ELL slice bases of the partials
    std::vector<int32_t> pdeg;                     // [np] partials per particle (tiles touching it)
    std::vector<int32_t> body_g0;                  // [nb] first slice of each body
    // colour-ordered element copies for the fused path: within each body and kind,
    // elements sorted by (colour, index); no two elements of a colour share a particle
    bool fused_ok = false;                         // every kind of every body coloured with <= 128 colours
    bool coloured = false;                         // the fused path's colouring was made (not for serving queries)
    std::vector<int32_t> ftet, ftri, fhin;         // fused position -> element index
    std::vector<int32_t> coff;                     // colour boundaries (fused element positions)
    std::vector<int32_t> cbase, ncol;              // [nb][3] first entry in coff, number of colours
    std::vector<uint8_t> pinned;                   // [np]
    std::vector<double> rest;                      // [np][3] rest positions (state positions are relative to them)
    std::vector<double> dt, grav, plane, kb;       // per body
    std::vector<uint8_t> contact_on;               // per body
    std::vector<uint8_t> air_on;                   // per body: lift/drag on its triangles
    bool any_air = false;
};

namespace gsim {

const int N_XCD = 8;  // workgroups are dispatched round-robin over the XCDs
const int MAX_LANES = 4;      // concurrent launch lanes of the two-pass path
const int DEFAULT_LANES = 2;  // lanes of a new model with that many bodies or more

struct Layout {
    size_t model, bodies, etiles, ptiles;
    size_t tet_code, tet_dinv, tet_vol;
    size_t tri_code, tri_dinv, tri_area;
    size_t hin_code, hin_phi0;
    size_t tp;
    size_t gbase, pdeg, pinned, slots, fslots, vslots, cpart, lpart;  // vslots: only when a body has air
    size_t rest, rgap;  // rest positions [3][np], rest ground gaps [np]
    size_t bflag;       // [nb][2] int32 body status words
    size_t fbuf, abuf;  // forward / adjoint internal ping-pong states
    size_t fbar;        // [2][3][np] adjoint forces handed from one adjoint step to the next
    // fused path: colour-ordered element records, colour bounds, body launch order
    size_t f_tet_idx, f_tet_dinv, f_tet_vol, f_tet_orig, f_tri_idx, f_tri_dinv, f_tri_area, f_tri_orig;
    size_t f_hin_idx, f_hin_phi0, f_hin_orig, coff, border, f_par, f_ktri, f_g, f_gk, f_hpar, f_gh;
    size_t ntiles, toff;  // persistent execution: natural-order tiles, per-body ranges [2][nb + 1]
    size_t table;
    int64_t table_cap;
    size_t total;
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
};

// Records an error message for gsim_last_error() and returns `code`.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// Workgroups are dispatched round-robin over the 8 XCDs (block b on XCD b % 8).
// Permutes a natural-order tile list so that consecutive tiles (which share
// particles, hence L2 lines) land on the same XCD; pads with empty tiles.
void xcd_order(const std::vector<Tile>& nat, int empty_kind, int dummy_id, std::vector<Tile>& out, int& grid);

// Where the host-to-device copies of a model's set-up go.  Without one, each copy is a
// hipMemcpyAsync on the set-up stream and the set-up ends with a synchronisation of
// that stream (the host arrays are temporaries).  The serving engine passes its
// staging area instead: copy() takes the bytes at once (the source may be freed on
// return) and zero() records a zero fill; both land on the device, in stream order,
// before any later launch on that stream reads them.
struct UploadSink {
    virtual ~UploadSink() = default;
    virtual hipError_t copy(void* dst, const void* src, size_t n) = 0;
    virtual hipError_t zero(void* dst, size_t n) = 0;
};

template <typename T>
int model_init(const gsim_plan* P, int max_steps, int K, void* d_ws, size_t bytes, void* stream, gsim_model** out,
               UploadSink* sink = nullptr);

// gsim_plan_create, optionally without the fused path's colouring (a model of such a
// plan runs the two-pass path only; its colour-ordered records are not made).
int plan_create(const gsim_model_desc* desc, gsim_plan** out, bool fused);

}  // namespace gsim

struct gsim_model {
    int dtype = 32;
    int nb = 0;
    int64_t np = 0, ne = 0, nt = 0, nh = 0;
    int max_steps = 0, K = 1;
    char* ws = nullptr;
    gsim::Layout L{};
    std::vector<int64_t> poff, eoff, toff, hoff;
    int exec = GSIM_EXEC_PLAIN;
    int block = 256, items = 1;    // element passes: threads per element tile (items: unused, tiles are planned)
    int pblock = 256, pitems = 1;  // particle passes
    int n_etiles = 0, n_ptiles = 0;   // launched grid sizes (including XCD padding)
    int n_etiles_nat = 0;             // natural-order element tiles (persistent execution)
    // launch lanes: with L > 1, the bodies are split into L groups of about equal
    // work whose passes run on L streams (the caller's and lane_stream[1 .. L-1])
    // between a fork and a join; lane l's tiles are [lane_e[l], lane_e[l + 1]) of
    // the element list and [lane_p[l], lane_p[l + 1]) of the particle list.  Within a
    // lane the tiles of bodies with air come last, from lane_e_air[l] / lane_p_air[l]:
    // they run the kernel variant with lift/drag, the others the plain one, so a
    // body's arithmetic never depends on the rest of its batch.
    int lanes = 1;
    int lane_e[gsim::MAX_LANES + 1] = {}, lane_p[gsim::MAX_LANES + 1] = {};
    int lane_e_air[gsim::MAX_LANES] = {}, lane_p_air[gsim::MAX_LANES] = {};
    hipStream_t lane_stream[gsim::MAX_LANES] = {};
    hipEvent_t ev_fork = nullptr, ev_join[gsim::MAX_LANES] = {};
    int n_ptile_rows = 0;             // real particle tiles (contact / loss partial rows)
    // overlapped recompute (gsim_model_set_overlap): the caller's second segment buffer;
    // tail_*: the checkpointed rollout whose last segment's states seg2 holds (none: null)
    void* seg2 = nullptr;
    size_t seg2_bytes = 0;
    const void* tail_ckpt = nullptr;
    const void* tail_seg2 = nullptr;
    int tail_n = 0;
    std::vector<char> bodies_host;    // BodyDev<T>[nb] as last uploaded
    char* stage = nullptr;            // pinned copy of the launch table as last uploaded
    hipEvent_t stage_evt = nullptr;   // completes when the last table upload has read `stage`
    std::vector<gsim::Tile> etiles_nat, ptiles_nat;  // natural-order tiles (planned / current tile size)
    std::vector<gsim::Tile> etiles_plan;             // element tiles of the plan
    int64_t etile_words[2] = {0, 0};                 // largest element tile's LDS words, forward / adjoint
    std::vector<char> md_host;                       // ModelDev<T> as uploaded
    std::map<long long, gsim::GraphEntry> graphs;
    // per-kernel timing: HIP events around each launch of the kernels in timing_mask
    int timing_mask = 0;
    std::vector<hipEvent_t> evt_pool;
    struct Pending {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    double timing_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t timing_n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // fused path
    bool fused_ok = false;   // colouring succeeded for every body and kind
    bool any_air = false;    // some body has lift/drag (not modelled by the fused path)
    std::vector<uint8_t> air_on;  // per body
    int64_t max_body_np = 0;  // particles of the largest body
    size_t fused_dyn[2] = {0, 0};  // dynamic LDS bytes of the fused forward / adjoint launch (max over bodies)
};
