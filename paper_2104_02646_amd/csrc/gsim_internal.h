// Internal layouts shared by the HIP kernels and the host runtime of libgsim.
//
// Device data of one model (all inside the caller-owned workspace):
//   rest positions X [3][np] and rest ground gaps [np]: positions in every state
//     buffer the library owns (internal ping-pong states, checkpoints, segments)
//     are displacements u = x - X, so deformation is resolved in FP32 however far
//     the body is from the origin; the caller's states are absolute;
//   element records, SoA over elements of each kind:
//     tets    idx[4][ne] (int32, model-global particle index), dinv[9][ne] (Dm^-1
//             row-major), vol[ne], slot[4][ne] (corner -> gather slot)
//     tris    idx[3][nt], dinv[4][nt], area[nt], slot[3][nt]
//     hinges  idx[4][nh] (wing0, wing1, edge0, edge1), phi0[nh], slot[4][nh]
//   gather table in sliced-ELL form: the particles of a body are cut into
//     slices of 64 (one wavefront); slice g stores its particles' corner slots
//     interleaved, so corner k of lane j sits at gbase[g] + 64 k + j and one
//     wavefront load of "corner k" is one contiguous 1 KB (FP32) access;
//     pdeg[p] = number of element corners of particle p (summed in order k = 0..);
//   slots[nslot][4]: one 4-vector per element corner, written once per pass by
//     the element kernel (forward: the corner force; adjoint: the corner's
//     position-adjoint contribution and f_corner . fbar for the mass gradient).
// Each kernel launch reads its per-launch pointers (state in/out, adjoints,
// parameters, gradients) from a StepDev record in device memory, so a launch
// sequence can be captured once into a hipGraph and replayed with new buffers.
#pragma once
#include <stdint.h>

namespace gsim {

enum TileKind : int32_t { TILE_TET = 0, TILE_TRI = 1, TILE_HINGE = 2, TILE_PART = 3 };
// Serving's combined launches: the kind of an adjoint tile carries this bit.
const int32_t TILE_ADJ = 0x100;


// One workgroup's share of a pass: `count` consecutive items of one kind of one body.
struct Tile {
    int32_t model;  // index into the ModelDev / StepDev arrays of the launch
    int32_t body;   // body index inside the model
    int32_t kind;   // TileKind
    int32_t count;  // items in this tile
    int64_t begin;  // first item (model-global element or particle index)
    int32_t id;     // particle tiles: row of the contact-gradient partial buffer;
                    // element tiles: first tile particle
    int32_t pad;    // element tiles: number of tile particles
};

// Serving: one query's share of a round's pass: its `count` tiles (resident on the
// device since admission) become the round's tiles [begin, begin + count), with the
// launch's model index `model` and `flags` (TILE_ADJ or 0) OR-ed into their kind.
struct TileSeg {
    const Tile* tiles;
    int32_t begin, count, model, flags;
};

// One piece of a batched device copy: n bytes from src to dst, or zeros when src is
// null; the host splits each copy into pieces of at most STAGE_PIECE bytes.
struct StageSeg {
    const char* src;
    char* dst;
    int64_t n;
};
const int64_t STAGE_PIECE = 64 << 10;

template <typename T>
struct BodyDev {
    int64_t p0, np;      // particle range
    int32_t pt0, pt1;    // particle-tile id range (contact-gradient partials)
    int32_t contact_on;  // ground contact active
    int32_t g0;          // first gather slice of the body
    int32_t air_on;      // lift/drag on the body's triangles
    int32_t cbase[3];    // fused path: first colour boundary of each element kind in coff
    int32_t ncol[3];     // fused path: colours of each element kind
    T dt;
    T g[3];
    T plane[4];          // n.x = d
    T kb;                // bending stiffness
};

template <typename T>
struct ModelDev {
    int64_t np, ne, nt, nh, nslot;
    int32_t n_bodies, n_ptiles;
    // element records (SoA over elements); corner codes: tile-local particle |
    // position in the tile's particle-sorted corner order << 16
    const uint32_t* tet_code;
    const T* tet_dinv;
    const T* tet_vol;
    const uint32_t* tri_code;
    const T* tri_dinv;
    const T* tri_area;
    const uint32_t* hin_code;
    const T* hin_phi0;
    // tile particles (Tile.id = first, Tile.pad = count), one 16-byte record each:
    // particle index, corner run (first sorted corner | count << 16), partial slot, 0
    const int32_t* tp;
    const int32_t* gbase;  // [n_slices] first partial slot of each 64-particle slice
    const int32_t* pdeg;   // [np] partials per particle
    const uint8_t* pinned;
    const T* rest;  // [3][np] rest positions X: the state holds displacements u = x - X
    const T* rgap;  // [np] rest ground gap n.X - d of each particle (its body's plane)
    const BodyDev<T>* bodies;
    int32_t* bflag;  // [n_bodies][2] status words, set to 1 by the kernels: [0] a state or
                     // adjoint value stopped being finite, [1] a tet inverted (J <= 0)
    T* slots;   // [nslot][4] per-(tile, particle) partial sums of the adjoint passes
    T* fslots;  // [nslot][3] per-(tile, particle) forces of the forward passes
    T* vslots;  // [nslot][4] velocity-adjoint partials of air tiles (null when no body has air)
    T* cpart;   // [n_ptiles][4] contact-gradient partial sums
    T* lpart;   // [n_ptiles] loss partial sums
    // fused path: element records in colour order (same SoA layouts, corner indices
    // local to the element's body), the original element index of each position
    // (for parameters and gradients), colour bounds
    const int32_t* f_tet_idx;
    const T* f_tet_dinv;
    const T* f_tet_vol;
    const int32_t* f_tet_orig;
    const int32_t* f_tri_idx;
    const T* f_tri_dinv;
    const T* f_tri_area;
    const int32_t* f_tri_orig;
    const int32_t* f_hin_idx;
    const T* f_hin_phi0;
    const int32_t* f_hin_orig;
    const int32_t* coff;
    T* f_par;   // [3][ne] mu, lambda, actuation in colour order (gathered per call)
    T* f_ktri;  // [nt] membrane stiffness in colour order
    T* f_g;     // [3][ne] mu-bar, lambda-bar, actuation-bar in colour order (scattered back per call)
    T* f_gk;    // [nt] k-bar in colour order
    T* f_hpar;  // [nh] hinge actuation in colour order
    T* f_gh;    // [nh] hinge actuation-bar in colour order
};

template <typename T>
struct StepDev {
    const T* x;   // state at the start of the step, SoA [3][np]
    const T* v;
    T* xo;        // forward: state at the end of the step
    T* vo;
    T* ckx;       // forward: optional copy of the input state (checkpoint)
    T* ckv;
    const T* xb;  // adjoint of the step output
    const T* vb;
    T* xbo;       // adjoint of the step input
    T* vbo;
    const T* fb;  // adjoint: this step's adjoint force dt w (vbar+ + dt xbar+), stored by the
                  // previous adjoint step's particle pass (null: formed from xb, vb)
    T* fbo;       // particle adjoint: store the previous step's adjoint force here (or null)
    const T* mu;
    const T* lam;
    const T* act;
    const T* ktri;
    const T* mass;
    const T* contact;  // [n_bodies][4]
    const T* hact;     // [nh] hinge actuation (this step's), may be null
    const T* air;      // [n_bodies][2] k_drag, k_lift (bodies with air_on)
    T* g_mu;
    T* g_lam;
    T* g_ktri;
    T* g_mass;
    T* g_contact;      // [n_bodies][4]
    T* g_act;          // [ne] tet actuation gradient (this step's slot), may be null
    T* g_hact;         // [nh] hinge actuation gradient, may be null
    const T* target;   // loss target, SoA [3][np]
    T* loss;           // [n_bodies]
    // fused path
    T* seg;            // forward: store the state after every step here ([step][x|v][3][np])
    const T* seg_in;   // adjoint: states t0+1.. of the segment (the state at t0 is x, v)
    int32_t nsteps;    // steps run by one fused launch
    int32_t t_base;    // absolute index of its first step (checkpoint slots)
    int32_t ckpt_every;
    int32_t x_abs;     // x holds absolute positions (the caller's state), not displacements
    int32_t xo_abs;    // forward: write absolute positions to xo (the caller's state)
    int32_t adj;       // the row is an adjoint step (read by persistent execution)
};

// Kernel timing: when a pair of events is armed, the next launch of the element and
// particle passes records them as that kernel's own start and end (HIP's extended
// launch), so their elapsed time is the kernel's execution, without the event packets
// around it; the launch disarms them.  Returns whether the pair was consumed.
void arm_launch_events(hipEvent_t start, hipEvent_t stop);
bool disarm_launch_events();

// Host-side launch helpers (defined in gsim_kernels.hip).  `stream` is a hipStream_t;
// `air` selects the kernel variant that models lift/drag (models with an air body).
// element passes: one workgroup (block threads) per element tile, `lds` bytes of
// dynamic LDS (the largest tile's: forward 4 words per tile particle + 4 per
// corner, adjoint 8 + 4)
template <typename T>
int launch_elem_fwd(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, size_t lds,
                    bool air, void* stream);
template <typename T>
int launch_part_fwd(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, int items,
                    void* stream);
template <typename T>
int launch_elem_adj(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, size_t lds,
                    bool air, void* stream);
template <typename T>
int launch_part_adj(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, int items,
                    bool air, void* stream);
template <typename T>
int launch_fill(T* p, int64_t n, T value, void* stream);
// Persistent execution of steps rows[0 .. n_rows): workgroup b runs body b's element
// tiles etiles[toff[b] .. toff[b + 1]) one after another, then its particle tiles
// ptiles[toff[nb + 1 + b] .. toff[nb + 2 + b]), for every row in turn (forward, or
// adjoint where row.adj is set); `lds` covers the largest element tile of either kind.
template <typename T>
int launch_persist(const ModelDev<T>* md, const StepDev<T>* rows, int n_rows, const Tile* etiles, const Tile* ptiles,
                   const int32_t* toff, int n_bodies, int block, size_t lds, void* stream);
// Overlapped recompute: one element launch (particles = false) or one particle launch
// (true) running the adjoint pass of row sd_adj and the forward pass of row sd_fwd
// over the same tile list (models without lift/drag).  Split layout: the forward tiles
// start at the adjoint count rounded up to a multiple of 8, so both keep their XCD
// placement; paired layout (element launch with `paired`): one workgroup per tile runs
// both passes of its tile, adjoint first.  `lds` covers both element passes.
template <typename T>
int launch_dual(const ModelDev<T>* md, const StepDev<T>* sd_adj, const StepDev<T>* sd_fwd, const Tile* etiles,
                int n_etiles, const Tile* ptiles, int n_ptiles, int block, int pblock, size_t lds, bool particles,
                bool paired, void* stream);
// One workgroup per piece: the pieces' copies and zero fills in one launch (the serving
// engine's query set-up, staged through one host-to-device copy).
int launch_stage_copy(const StageSeg* segs, int n_segs, void* stream);
// Serving: one launch over a round's forward and adjoint element tiles (adjoint ones
// marked TILE_ADJ), then one over its particle tiles; each workgroup finds its tile from
// the round's segment tables (position pos of the XCD order of the concatenation: tile
// t = (pos % N_XCD) * G + pos / N_XCD, G = grid / N_XCD, grid = the total rounded up to
// N_XCD; fewer than N_XCD tiles keep their order; positions past the total are empty
// tiles reducing into row dummy_id of model 0).  `lds` covers both element kinds.
template <typename T>
int launch_mixed(const ModelDev<T>* md, const StepDev<T>* sd, const TileSeg* eseg, int n_eseg, int e_total, int e_grid,
                 const TileSeg* pseg, int n_pseg, int p_total, int p_grid, int dummy_id, int block, size_t lds,
                 void* stream);
template <typename T>
int launch_contact_reduce(const ModelDev<T>* md, const StepDev<T>* sd, int n_bodies, void* stream);
template <typename T>
int launch_loss(const ModelDev<T>* md, const StepDev<T>* sd, const Tile* tiles, int ntiles, int block, int items,
                int n_bodies, void* stream);
// Fused path: one workgroup per body (bodies in `order`), the whole segment of steps
// in one launch; `lds` bytes of dynamic LDS.
template <typename T>
int launch_fused_fwd(const ModelDev<T>* md, const StepDev<T>* sd, const int32_t* order, int n_bodies, size_t lds,
                     void* stream);
// act: the variant that also accumulates the actuation gradients
template <typename T>
int launch_fused_adj(const ModelDev<T>* md, const StepDev<T>* sd, const int32_t* order, int n_bodies, size_t lds,
                     bool act, void* stream);
// two-pass element tiles: at most ETILE consecutive elements of one kind of one
// body, and at most ETILE_WORDS words of adjoint LDS (8 per tile particle, 4 per
// corner; triangle tiles of bodies with air: 12 and 8)
const int ETILE = 256, ETILE_WORDS = 16384;

const int FUSED_FWD_BLOCK = 1024, FUSED_ADJ_BLOCK = 512;
// dynamic LDS per particle of the largest body: x, v, f (forward); fbar, xbar-acc, f.fbar (adjoint)
const int FUSED_FWD_LDS_WORDS = 9, FUSED_ADJ_LDS_WORDS = 10;
// fused sweeps: elements computed per thread before their contributions are added
constexpr int FUSED_AHEAD_FWD = 2, FUSED_AHEAD_ADJ = 2;
// per-call parameter gather into colour order (and gradient-buffer clear), and the
// scatter of colour-ordered gradients back to element order
template <typename T>
int launch_fused_params(const ModelDev<T>* md, const StepDev<T>* sd, void* stream);
template <typename T>
int launch_fused_grads(const ModelDev<T>* md, const StepDev<T>* sd, void* stream);
// static LDS bytes of the fused forward (adjoint = false) or adjoint kernel
template <typename T>
hipError_t fused_static_lds(bool adjoint, size_t* bytes);

}  // namespace gsim
