/*
 * gsim.h -- C-ABI of the MI355X differentiable simulation step.
 *
 * The library implements one time step of a deformable-body simulator and the
 * reverse-mode adjoint of that step, as stated in "gradSim: differentiable
 * simulation for system identification and visuomotor control" (ICLR 2021):
 *
 *   state      s = [q, u]: particle positions x and velocities v (Sec. 2.1);
 *   parameters theta: per-tet Lame parameters mu, lambda (App. A.1, App. B.1),
 *              per-triangle membrane stiffness k (App. A.1 thin shells),
 *              per-particle mass m, per-body contact parameters
 *              [k_e, k_d, k_f, mu_f] (App. A.1 "Contact");
 *   step       the semi-implicit Euler relation g(s-, s+, theta) = 0 (App. A.2):
 *              v+ = v- + dt (M^-1 f(s-) + g), x+ = x- + dt v+ ;
 *   backward   the discrete adjoint (App. A, implicit-function theorem, with the
 *              App. A.2 step Jacobians): from dl/ds+ it produces dl/ds- and
 *              accumulates dl/dtheta.
 *
 * Forces f(s) are the sum of: stable Neo-Hookean constant-strain tets, with
 * alpha = 1 + 3 mu/(4 lambda) + actuation; Neo-Hookean constant-strain
 * membrane triangles with mu = lambda = k and alpha2 = 5/3; dihedral bending
 * f = -k_b |E|^2/(|N1|+|N2|) sin((phi - phi0)/2 + a) dphi/dx with Bridson's
 * directions; penalty ground contact lambda_n = k_e C + k_d Cdot along the
 * plane normal and relaxed-Coulomb friction (isotropic cone, stick when
 * k_f |u_t| <= mu_f |lambda_n|).  Gravity is an acceleration on particles
 * that are not pinned.
 *
 * Conventions
 *   - Every call returns an int status: GSIM_OK (0) or a negative GSIM_E_*.
 *     gsim_last_error() returns a thread-local message for the last failure.
 *   - Device arrays are caller-owned (the library never allocates device
 *     memory).  Floating arrays have the model's dtype (float or double).
 *   - Particle state is SoA: x[3][n_particles] (all x components, then y,
 *     then z), same for v.  Bodies are contiguous particle ranges.
 *   - Launches are asynchronous on the given stream (hipStream_t passed as
 *     void*; NULL = the default stream).  Validation errors return
 *     synchronously.  Successive calls on one model must be stream-ordered
 *     (same stream, or synchronised by the caller): the model's workspace is
 *     reused by every call.
 *   - Parameter gradients ACCUMULATE into caller buffers (zero them first).
 *     The mass gradient is with respect to m (not 1/m) and is 0 for pinned
 *     particles.
 *   - No C++ exception crosses this ABI.  Distinct models are independent.
 */
#ifndef GSIM_H
#define GSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GSIM_OK = 0,
    GSIM_E_INVALID = -1,     /* bad argument (NULL pointer, size, dtype, ...) */
    GSIM_E_TOPOLOGY = -2,    /* index out of range or element crossing bodies */
    GSIM_E_DEGENERATE = -3,  /* zero-volume tet / zero-area triangle / zero-length hinge edge */
    GSIM_E_WORKSPACE = -4,   /* workspace / buffer too small for the request */
    GSIM_E_HIP = -5,         /* a HIP runtime call failed (message has the HIP error) */
    GSIM_E_NONFINITE = -6,   /* non-finite input value */
    GSIM_E_UNSUPPORTED = -7  /* request outside what the library implements */
};

enum { GSIM_F32 = 32, GSIM_F64 = 64 };

/* Execution strategies for rollouts (gsim_model_set_exec). */
enum {
    GSIM_EXEC_PLAIN = 0,   /* two kernel launches per step (element pass, particle pass) */
    GSIM_EXEC_GRAPH = 1,   /* the same launches captured once into a hipGraph and replayed
                              (needs a non-default stream) */
    GSIM_EXEC_FUSED = 2,   /* one workgroup per body keeps the body in LDS and runs a whole
                              checkpoint segment of steps per launch (forward rollout: one
                              launch; backward: two launches per segment).  Needs every
                              body's particles to fit in LDS (36 B each for FP32) */
    GSIM_EXEC_PERSIST = 3  /* one workgroup per body runs every step of a call's run of
                              steps (a rollout: one launch; a backward: one launch) through
                              the two-pass path's element and particle tiles, with workgroup
                              barriers in place of launch boundaries: bitwise the two-pass
                              results; for bodies of few tiles, whose steps are bound by
                              launch latency.  FP32 models without lift/drag */
};

const char* gsim_last_error(void);
int gsim_version(int* major, int* minor);

/* ------------------------------------------------------------------------ */
/* MODEL DESCRIPTION (host memory, read only during gsim_plan_create)        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dtype;                         /* GSIM_F32 or GSIM_F64 */
    int n_bodies;                      /* >= 1 */
    int64_t n_particles, n_tets, n_tris, n_hinges;
    const int64_t* body_particle_off;  /* [n_bodies+1], body b owns particles [off[b], off[b+1]) */
    const int64_t* body_tet_off;       /* [n_bodies+1] or NULL when n_tets == 0 */
    const int64_t* body_tri_off;       /* [n_bodies+1] or NULL when n_tris == 0 */
    const int64_t* body_hinge_off;     /* [n_bodies+1] or NULL when n_hinges == 0 */
    const double* rest_x;              /* [n_particles][3] rest positions (AoS) */
    const int32_t* tet_idx;            /* [n_tets][4] particle indices (model-global) */
    const int32_t* tri_idx;            /* [n_tris][3] */
    const int32_t* hinge_idx;          /* [n_hinges][4] = wing0, wing1, edge0, edge1 */
    const uint8_t* pinned;             /* [n_particles] nonzero = kinematic (w = 0), or NULL */
    const double* gravity;             /* [n_bodies][3] acceleration */
    const double* dt;                  /* [n_bodies] time step */
    const double* ground;              /* [n_bodies][4] plane n.x = d as (nx, ny, nz, d), or NULL */
    const uint8_t* contact_on;         /* [n_bodies] nonzero = ground contact active, or NULL (off) */
    const double* k_bend;              /* [n_bodies] bending stiffness, or NULL (0) */
    const uint8_t* air_on;             /* [n_bodies] nonzero = lift/drag on the body's triangles
                                          (see gsim_params.air), or NULL (off) */
    int tile_elems;                    /* elements per element tile of the two-pass path, in
                                          [GSIM_TILE_MIN, GSIM_TILE_MAX]; 0 = GSIM_TILE_DEFAULT.
                                          A launch-shape choice (the autotuner searches it): it
                                          changes the summation order of the scatter, not the model */
} gsim_model_desc;

enum { GSIM_TILE_MIN = 32, GSIM_TILE_MAX = 2048, GSIM_TILE_DEFAULT = 256 };

typedef struct gsim_plan gsim_plan;    /* host object: validated topology, rest data, tiles */
typedef struct gsim_model gsim_model;  /* host handle bound to a caller-owned device workspace */

/* Validates the description (indices in range and inside their body, finite
 * rest positions, dt > 0), orients every tet so det(Dm) > 0 (swapping corners
 * 1 and 2), precomputes Dm^-1 and rest volume / area and rest dihedral angles,
 * and builds the deterministic force-gather tables (each particle sums its
 * element-corner contributions in a fixed order: no atomics).
 * Errors: GSIM_E_INVALID, GSIM_E_TOPOLOGY, GSIM_E_DEGENERATE, GSIM_E_NONFINITE. */
int gsim_plan_create(const gsim_model_desc* desc, gsim_plan** out);
int gsim_plan_destroy(gsim_plan* plan);

/* Exact byte sizes of the caller-owned device buffers for rollouts of up to
 * max_steps steps with a checkpoint every ckpt_every steps:
 *   workspace: element records, gather tables, internal state buffers, launch
 *              tables (pass to gsim_model_init);
 *   ckpt:      ceil(max_steps/ckpt_every) saved states (x, v);
 *   segment:   ckpt_every recomputed states used by gsim_rollout_backward.
 * Any output pointer may be NULL. */
int gsim_plan_sizes(const gsim_plan* plan, int max_steps, int ckpt_every, size_t* workspace_bytes,
                    size_t* ckpt_bytes, size_t* segment_bytes);

/* Counts of the planned model: particles, tets, tris, hinges, bodies. */
int gsim_plan_counts(const gsim_plan* plan, int64_t* n_particles, int64_t* n_tets, int64_t* n_tris,
                     int64_t* n_hinges, int* n_bodies);

/* Host-only plan introspection (for checking the planner; no device needed).
 * kind: 0 tets, 1 triangles, 2 hinges.
 * gsim_plan_colouring: order[i] = element at colour-ordered position i (a
 * permutation of the kind's elements); bounds[] = colour boundaries over
 * positions, per body in body order (n_bounds entries written, at most
 * max_bounds); returns GSIM_E_UNSUPPORTED if colouring failed (> 128 colours).
 * Two-pass element tiles (Sec. 2.1 step; the force scatter of App. A.1 as a
 * segmented reduction): per body and kind, consecutive elements are cut into
 * tiles of at most 256 elements (fewer when the tile's particles would need
 * more than 16384 words of adjoint LDS).  The tile particles of a tile are the
 * particles its elements touch, in increasing order; its corners are ordered by
 * (tile particle, element, corner), so each tile particle owns one run of
 * corners; the element pass sums each run into one partial, written to the
 * particle's sliced-ELL table of partials.
 * gsim_plan_tiles: tiles[5 i .. 5 i + 4] = kind (0 tet, 1 tri, 2 hinge), body,
 * first element, element count, first tile particle of tile i (plan order);
 * per tile particle (tiles' lists concatenated): particle index, run (first
 * sorted corner | corner count << 16), partial slot.
 * gsim_plan_codes: codes[c * n + e] = tile-local index of the particle of corner
 * c of element e | position of the corner in its tile's sorted order << 16.
 * gsim_plan_partials: the partial table; the k-th tile (plan order) touching
 * the particle at lane j of 64-particle slice g writes slot slice_base[g] +
 * 64 k + j, k < degree[p].  Any output pointer may be NULL (sizes only). */
int gsim_plan_colouring(const gsim_plan* plan, int kind, int32_t* order, int32_t* bounds, int max_bounds,
                        int* n_bounds);
int gsim_plan_tiles(const gsim_plan* plan, int64_t* tiles, int64_t* n_tiles, int32_t* tile_particles, int32_t* runs,
                    int32_t* slots, int64_t* n_tile_particles);
int gsim_plan_codes(const gsim_plan* plan, int kind, uint32_t* codes);
int gsim_plan_partials(const gsim_plan* plan, int32_t* slice_base, int64_t* n_slices, int32_t* degree,
                       int64_t* n_slots);

/* Binds a plan to a caller-owned device workspace (>= workspace_bytes of
 * gsim_plan_sizes for the same max_steps / ckpt_every) and uploads the
 * element records on `stream`.  The plan may be destroyed afterwards. */
int gsim_model_init(const gsim_plan* plan, int max_steps, int ckpt_every, void* d_workspace, size_t bytes,
                    void* stream, gsim_model** out);
int gsim_model_destroy(gsim_model* model);

/* Selects the rollout execution strategy (GSIM_EXEC_*) and, for both passes,
 * the launch shape: block = threads per workgroup (64..512, multiple of 64),
 * items = particles per thread (1..8; particle passes: a workgroup's tile is
 * block * items particles).  Element passes run one workgroup per planned
 * element tile (see gsim_plan_tiles); their items value is kept but has no
 * effect.  0 keeps the current value.  get_exec reports the element-pass
 * shape. */
int gsim_model_set_exec(gsim_model* model, int exec, int block, int items);
int gsim_model_get_exec(const gsim_model* model, int* exec, int* block, int* items);

/* Launch shape of one pass (0 = element passes, 1 = particle passes), as above.
 * Results do not depend on the element-pass shape; the particle-pass shape
 * fixes the summation tree of per-body contact gradients and losses. */
int gsim_model_set_launch(gsim_model* model, int pass, int block, int items);
int gsim_model_get_launch(const gsim_model* model, int pass, int* block, int* items);

/* Launch lanes of the two-pass path (1..4; a new model with at least two bodies
 * starts with 2).  With L lanes the bodies are split into L groups of about
 * equal work, and the element and particle passes of consecutive steps of the
 * groups run on L streams: the caller's and L - 1 the model owns (default
 * priority), forked from and joined back into the caller's stream within each
 * call, so a captured graph holds L parallel branches.  Results do not depend
 * on the lanes.  GSIM_E_UNSUPPORTED for more lanes than bodies. */
int gsim_model_set_lanes(gsim_model* model, int lanes);
int gsim_model_get_lanes(const gsim_model* model, int* lanes);

/* Overlapped recompute in gsim_rollout_backward (the checkpointed reverse pass of
 * App. A.2: every segment's states are recomputed from its checkpoint before its
 * adjoint steps).  The recompute of segment s - 1 needs only its own checkpoint,
 * so it can run beside the adjoint steps of segment s: with a second segment buffer
 * d_segment2 of at least max(ckpt_every - 1, 1) states (6 n_particles values each,
 * caller-owned device memory that must outlive its use), the two passes share each
 * element launch and each particle launch, and consecutive segments alternate
 * between the two buffers.  A checkpointed gsim_rollout also leaves the states of its
 * last segment in d_segment2, and the next gsim_rollout_backward with the same d_ckpt
 * and n_steps skips that segment's recompute; any other checkpointed rollout, any
 * backward and any call of this function in between discard them (forward-only
 * rollouts, single steps and losses do not touch them).  The shared launches apply
 * under GSIM_EXEC_PLAIN and GSIM_EXEC_GRAPH, the kept segment also under
 * GSIM_EXEC_PERSIST, both for models without lift/drag; otherwise, and with
 * d_segment2 = NULL (the default), the passes run one after another.  Results are
 * bitwise the same either way.  GSIM_E_WORKSPACE when `bytes` is too small. */
int gsim_model_set_overlap(gsim_model* model, void* d_segment2, size_t bytes);

/* Kernel timing for measurement: with bit k of `mask` set, every launch of
 * kernel k is bracketed by HIP events on its stream (k: 0 element pass,
 * 1 particle pass, 2 element adjoint pass, 3 particle adjoint pass, 4 fused
 * forward segment, 5 fused adjoint segment, 6 shared adjoint + recompute element
 * launch, 7 shared adjoint + recompute particle launch of gsim_model_set_overlap).
 * With timing on, each pass (or shared pair of passes) is one launch over every
 * lane's tiles.  Plain
 * execution only (GSIM_E_UNSUPPORTED under GSIM_EXEC_GRAPH).
 * gsim_model_read_timing waits for the recorded events and returns (then
 * clears) kernel k's launch count and summed duration in milliseconds. */
int gsim_model_set_timing(gsim_model* model, int mask);
int gsim_model_read_timing(gsim_model* model, int kernel, int64_t* launches, double* total_ms);

/* Device-side failure detection.  The kernels raise per-body status flags in the
 * model's workspace: GSIM_FLAG_NONFINITE when a body's state or adjoint state stops
 * being finite (the explicit step is only conditionally stable: the paper's
 * limitations name instability at small masses; a NaN or infinite parameter shows
 * the same way), GSIM_FLAG_INVERTED when one of its tets reaches J <= 0 (the stable
 * Neo-Hookean energy is defined there; reported, not an error).  Flags stay raised
 * until cleared.  gsim_model_check waits for `stream` (the calls' stream), writes each
 * body's flags to body_flags (host [n_bodies], or NULL), clears them when `clear` is
 * nonzero, and returns GSIM_E_NONFINITE when any body is non-finite (the message names
 * the first), GSIM_OK otherwise.  Bodies are independent: one body going non-finite
 * leaves every other body's results unchanged. */
enum { GSIM_FLAG_NONFINITE = 1, GSIM_FLAG_INVERTED = 2 };
int gsim_model_check(gsim_model* model, int32_t* body_flags, int clear, void* stream);

/* ------------------------------------------------------------------------ */
/* STATE, PARAMETERS, GRADIENTS (device pointers, caller-owned)              */
/* ------------------------------------------------------------------------ */
typedef struct {
    void* x; /* [3][n_particles] */
    void* v; /* [3][n_particles] */
} gsim_state;

/* Actuation (App. A.1): a tet's actuation a shifts alpha in its energy
 * (alpha = 1 + 3 mu / (4 lambda) + a); a hinge's actuation shifts the bending
 * force's angle, f = -k_b s sin((phi - phi0)/2 + a_h) u.  Both may vary from
 * step to step: in gsim_step (over its n_steps), gsim_rollout and
 * gsim_rollout_backward, step t of the call reads act + t * act_stride (and
 * hact + t * hact_stride); a stride of 0 uses the same array every step. */
typedef struct {
    const void* mu;      /* [n_tets] Lame mu            (required if n_tets)  */
    const void* lam;     /* [n_tets] Lame lambda        (required if n_tets)  */
    const void* act;     /* [n_tets] tet actuation, NULL = 0                  */
    const void* k_tri;   /* [n_tris] membrane stiffness (required if n_tris)  */
    const void* mass;    /* [n_particles] mass > 0 (pinned particles ignore it) */
    const void* contact; /* [n_bodies][4] = k_e, k_d, k_f, mu_f (required if any contact) */
    const void* hact;    /* [n_hinges] hinge actuation, NULL = 0              */
    int64_t act_stride;  /* elements between consecutive steps' act arrays (>= 0) */
    int64_t hact_stride; /* same for hact */
    const void* air;     /* [n_bodies][2] = k_drag, k_lift (required if any body has air_on) */
} gsim_params;

/* Air (App. A.1 thin shells: a lift/drag model of the surrounding air, whose form
 * the paper leaves open).  On each triangle of a body with air_on, with u the
 * mean of its corner velocities (still air), n its unit normal, A its area and
 * s = n.u, the force F = -A (k_drag |s| u + k_lift s (|u|^2 n - s u) / |u|)
 * (quadratic drag on the projected area plus flat-plate lift perpendicular to u;
 * F = 0 at u = 0) is shared equally by its three corners.  k_drag and k_lift
 * are inputs only: no gradient is produced for them.  The position and velocity
 * adjoints include the force's dependence on both.  The fused path does not
 * model air (GSIM_E_UNSUPPORTED). */

/* Gradients accumulate (+=).  The actuation gradients of step t go to
 * act + t * act_stride (hact + t * hact_stride): with a stride of 0 every
 * step's contribution is summed into one array; with n_tets (n_hinges) each
 * step has its own. */
typedef struct {         /* any pointer may be NULL = gradient not requested; the
                            per-tet buffers mu, lam and act must be distinct
                            (GSIM_E_INVALID otherwise) */
    void* mu;            /* [n_tets]      */
    void* lam;           /* [n_tets]      */
    void* k_tri;         /* [n_tris]      */
    void* mass;          /* [n_particles] */
    void* contact;       /* [n_bodies][4] */
    void* act;           /* [n_tets] (per step: see act_stride) */
    void* hact;          /* [n_hinges] (per step: see hact_stride) */
    int64_t act_stride;
    int64_t hact_stride;
} gsim_grads;

/* ------------------------------------------------------------------------ */
/* STEP, ROLLOUT, BACKWARD, LOSS                                             */
/* ------------------------------------------------------------------------ */

/* n_steps semi-implicit Euler steps from `in` to `out` (App. A.2).  `in` and
 * `out` may alias.  1 <= n_steps <= max_steps. */
int gsim_step(gsim_model* model, const gsim_params* params, gsim_state in, gsim_state out, int n_steps,
              void* stream);

/* Reverse of ONE step taken at state s_minus: given adj_plus = dl/ds+ it writes
 * adj_minus = dl/ds- and accumulates dl/dtheta into grad (App. A).
 * adj_plus and adj_minus must not alias. */
int gsim_step_backward(gsim_model* model, const gsim_params* params, gsim_state s_minus, gsim_state adj_plus,
                       gsim_state adj_minus, const gsim_grads* grad, void* stream);

/* Rollout of n_steps steps from s0 into s_final, saving the state at every
 * step t with t % ckpt_every == 0 into d_ckpt (slot t/ckpt_every; layout
 * [slot][x|v][3][n_particles]).  d_ckpt may be NULL for a forward-only run.
 * ckpt_every must equal the value the model was initialised with. */
int gsim_rollout(gsim_model* model, const gsim_params* params, gsim_state s0, int n_steps, void* d_ckpt,
                 gsim_state s_final, void* stream);

/* Checkpointed reverse pass of a rollout made by gsim_rollout with the same
 * params and n_steps: for each checkpoint segment in reverse order it recomputes
 * the segment's states into d_segment and runs the adjoint steps.  adj_final =
 * dl/d(final state) (input, not modified), adj_initial = dl/d(s0) (output).
 * Gradients accumulate into grad. */
int gsim_rollout_backward(gsim_model* model, const gsim_params* params, const void* d_ckpt, int n_steps,
                          void* d_segment, gsim_state adj_final, gsim_state adj_initial, const gsim_grads* grad,
                          void* stream);

/* Per-body mean squared distance to a target: loss[b] = (1/n_b) sum_i
 * |x_i - x*_i|^2 over the body's particles; seeds adj_out.x = 2 (x - x*)/n_b
 * and adj_out.v = 0 (either field may be NULL to skip).  d_target is
 * [3][n_particles]; d_loss is [n_bodies]. */
int gsim_loss_mse(gsim_model* model, gsim_state s, const void* d_target, void* d_loss, gsim_state adj_out,
                  void* stream);

/* ------------------------------------------------------------------------ */
/* OPEN-LOOP ACTUATION CONTROLLER                                            */
/* ------------------------------------------------------------------------ */
/* The paper's control policy (App. "MPC controller architecture"; Sec. 5.3,
 * control-walker and control-fem): N phase-shifted sinusoids of the simulation
 * time feed one fully connected layer without bias and a tanh, which gives one
 * actuation value per output element (tet or hinge) per step:
 *
 *     s_k(t)    = sin(omega * (t0 + t) * dt + 2 pi k / N),      k = 0 .. N-1
 *     act[t][e] = scale * tanh(sum_k W[k][e] * s_k(t)),         t = 0 .. n_steps-1
 *
 * (the sum over k in increasing k).  The rows act[t] are the per-step actuation
 * rows of gsim_params (act = the array, act_stride = n); the gradient rows that
 * gsim_rollout_backward writes with act_stride = n are the act_grad input of
 * gsim_controller_backward.  The signals are evaluated in FP64 and rounded to
 * the dtype; everything else runs in the dtype. */
#define GSIM_CTRL_MAX_SIGNALS 16
typedef struct {
    int n_signals; /* N, 1 .. GSIM_CTRL_MAX_SIGNALS */
    double omega;  /* angular frequency (radians per unit of simulation time) */
    double dt;     /* simulation time of one step */
    double scale;  /* output amplitude; 1 gives the plain tanh */
} gsim_controller;

/* act[n_steps][n] (device, dtype elements) from the weights W[N][n] (device,
 * row k contiguous over the n outputs), for steps t0 .. t0 + n_steps - 1.
 * n == 0 or n_steps == 0 does nothing.  Asynchronous on `stream`.
 * Errors (nothing launched): GSIM_E_INVALID for a bad dtype, NULL pointers with
 * work to do, N outside 1..GSIM_CTRL_MAX_SIGNALS, negative n / t0 / n_steps, or
 * non-finite omega, dt, scale. */
int gsim_controller_forward(int dtype, const gsim_controller* ctrl, const void* W, int64_t n, int64_t t0,
                            int64_t n_steps, void* act, void* stream);
/* W_grad[N][n] += the gradient of sum_{t,e} act_grad[t][e] * act[t][e] with
 * respect to W, for the same steps; recomputes the layer from W (act itself
 * is not read).  act_grad is [n_steps][n].  Same errors as the forward. */
int gsim_controller_backward(int dtype, const gsim_controller* ctrl, const void* W, const void* act_grad, int64_t n,
                             int64_t t0, int64_t n_steps, void* W_grad, void* stream);

/* ------------------------------------------------------------------------ */
/* RIGID BODIES                                                              */
/* ------------------------------------------------------------------------ */
/* App. A.1 "Rigid bodies": state per body s = [x (3), r (4), v (3), omega (3)]
 * (centre-of-mass position; unit quaternion (w, i, j, k), body to world; linear
 * and angular velocity, world frame), stored [n_bodies][13].  Parameters per
 * body: mass m > 0, body-frame inertia about the centre of mass I = [Ixx, Iyy,
 * Izz, Ixy, Ixz, Iyz] (positive definite), contact [k_e, k_d, k_f, mu_f] (the
 * particle contact model of App. A.1 applied at every vertex).  One step
 * (semi-implicit Euler, App. A.2), with a_k = R(r) p_k for the body-frame
 * vertices p_k:
 *     F = sum_k f_k, tau = sum_k a_k x f_k, f_k = contact(x + a_k, v + omega x a_k)
 *     v+ = v + dt (F / m + g)
 *     omega+ = omega + dt Iw^-1 (tau - omega x (Iw omega)),  Iw = R I R^T
 *     x+ = x + dt v+,   r+ = normalise(r + dt/2 [0, omega+] (x) r)
 * R(r) is the rotation matrix of a unit quaternion: pass unit r0 (later states
 * are normalised by the step). */
#define GSIM_RIGID_MAX_VERTS 256
typedef struct gsim_rigid gsim_rigid;
typedef struct {
    int dtype;                 /* GSIM_F32 or GSIM_F64 */
    int n_bodies;              /* >= 1 */
    const int64_t* vert_off;   /* [n_bodies+1]; body b owns vertices [off[b], off[b+1]), 1..256 of them */
    const double* verts;       /* [n_verts][3] body-frame positions relative to the centre of mass */
    const double* gravity;     /* [n_bodies][3] */
    const double* dt;          /* [n_bodies] */
    const double* ground;      /* [n_bodies][4] plane (nx, ny, nz, d), or NULL (y = 0) */
    const uint8_t* contact_on; /* [n_bodies] nonzero = vertex contact with the plane, or NULL (off) */
} gsim_rigid_desc;
typedef struct {
    const void* mass;    /* [n_bodies] */
    const void* inertia; /* [n_bodies][6] */
    const void* contact; /* [n_bodies][4] */
} gsim_rigid_params;
typedef struct {         /* gradients accumulate (+=); NULL = not requested */
    void* mass;
    void* inertia;
    void* contact;       /* only bodies with contact_on */
} gsim_rigid_grads;

/* Exact device bytes of a rigid model's workspace.  Errors: GSIM_E_INVALID,
 * GSIM_E_UNSUPPORTED (a body with more than GSIM_RIGID_MAX_VERTS vertices),
 * GSIM_E_NONFINITE. */
int gsim_rigid_sizes(const gsim_rigid_desc* desc, size_t* workspace_bytes);
/* Binds a rigid model to a caller-owned, 256-byte aligned device workspace and
 * uploads the bodies (synchronises `stream`). */
int gsim_rigid_init(const gsim_rigid_desc* desc, void* d_workspace, size_t bytes, void* stream, gsim_rigid** out);
int gsim_rigid_destroy(gsim_rigid* model);
/* n_steps steps from s0 [n_bodies][13]; writes every state to traj
 * [(n_steps + 1)][n_bodies][13] (traj[0] = s0; the adjoint reads them).  One
 * launch for the whole rollout. */
int gsim_rigid_rollout(gsim_rigid* model, const gsim_rigid_params* params, const void* s0, int n_steps, void* traj,
                       void* stream);
/* loss[b] = mean over body b's vertices of |x + R p_k - target_k|^2 (target
 * [n_verts][3], world frame); state_bar [n_bodies][13] (or NULL) receives its
 * gradient with respect to the state (x and r; the velocity entries are 0). */
int gsim_rigid_loss(gsim_rigid* model, const void* state, const void* target, void* loss, void* state_bar,
                    void* stream);
/* Reverse pass over the stored trajectory (App. A): from adj_final (the adjoint
 * of state n_steps) to adj_init (of state 0), accumulating parameter gradients. */
int gsim_rigid_rollout_backward(gsim_rigid* model, const gsim_rigid_params* params, const void* traj, int n_steps,
                                const void* adj_final, void* adj_init, const gsim_rigid_grads* grads, void* stream);

/* ------------------------------------------------------------------------ */
/* SOFT SILHOUETTE RENDERER                                                  */
/* ------------------------------------------------------------------------ */
/* The paper puts its losses on rendered pixels through a differentiable soft
 * rasterizer (Sec. 3, rendering appendix: SoftRas, DIB-R).  Built here: SoftRas's
 * silhouette.  Vertex X (SoA positions, e.g. a model's particle state) projects to
 * pixel coordinates u = P0.[X,1] / P2.[X,1], v = P1.[X,1] / P2.[X,1] (P a 3x4
 * matrix, row-major; vertices must have P2.[X,1] > 0); triangle j covers pixel
 * (row, col), centre (col + 0.5, row + 0.5), with D_j = sigmoid(+-d^2 / sigma), d the
 * distance to its edges (+ inside); image[row][col] = 1 - prod_j (1 - D_j).  Terms
 * outside a triangle with d^2 > 13.8155 sigma (D < 1e-6) are dropped. */
typedef struct gsim_raster gsim_raster;
typedef struct {
    double P[12];  /* camera matrix, world -> homogeneous pixel coordinates */
    double sigma;  /* blur, pixel^2 (> 0) */
} gsim_camera;
/* Exact device bytes of a renderer for n_verts vertices, n_tris triangles and an
 * image of height x width pixels. */
int gsim_raster_sizes(int dtype, int64_t n_verts, int64_t n_tris, int height, int width, size_t* workspace_bytes);
/* tris: host [n_tris][3] vertex indices (copied).  Errors: GSIM_E_INVALID,
 * GSIM_E_TOPOLOGY (index out of range), GSIM_E_WORKSPACE. */
int gsim_raster_init(int dtype, int64_t n_verts, int64_t n_tris, const int32_t* tris, int height, int width,
                     void* d_workspace, size_t bytes, void* stream, gsim_raster** out);
int gsim_raster_destroy(gsim_raster* raster);
/* image [height][width] of the vertices x ([3][n_verts] SoA, device; image
 * device, caller-owned, dtype of the renderer).  Asynchronous on stream.  Errors
 * (returned before anything is launched): GSIM_E_INVALID (NULL pointer, sigma not
 * > 0), GSIM_E_NONFINITE (camera matrix); GSIM_E_HIP from the launch. */
int gsim_raster_forward(gsim_raster* raster, const gsim_camera* camera, const void* x, void* image, void* stream);
/* x_bar ([3][n_verts], +=) of sum(image_bar * image) for the same x and camera
 * (recomputes what it needs; independent of earlier forward calls).  Calls on one
 * renderer must not overlap (they share its workspace). */
int gsim_raster_backward(gsim_raster* raster, const gsim_camera* camera, const void* x, const void* image_bar,
                         void* x_bar, void* stream);

/* FOR CALLERS THAT CANNOT ALLOCATE DEVICE MEMORY (code under graph capture, tight
 * serving loops, harnesses that forbid allocation): the forward of gsim_raster_forward
 * without a renderer object or workspace.  The same kernels run with their scratch
 * (projected vertices, transmittance, triangle records, chunk boxes) in one static
 * device array of GSIM_RASTER_SCRATCH_BYTES that each GPU the library runs on holds
 * until the process ends; nothing is allocated, on the device or the host.
 *   d_tris  device [n_tris][3] vertex indices (caller-owned input).  The host cannot
 *           check them: a triangle with an index outside [0, n_verts) is not read and
 *           covers no pixel.
 *   x       device [3][n_verts] SoA positions; image: device [height][width] output;
 *           dtype GSIM_F32 or GSIM_F64 for both.
 * Results equal gsim_raster_forward's for the same inputs.  Every scratch region is
 * written before it is read, so a call needs nothing cleared and keeps no state
 * between calls.  Calls on one GPU share its array: calls that overlap (different
 * streams or threads) race and must be serialised by the caller.
 * Errors (before any launch): GSIM_E_INVALID, GSIM_E_NONFINITE as gsim_raster_forward;
 * GSIM_E_WORKSPACE when the sizes need more scratch than the array holds (about
 * 64 B per triangle + 12 B per vertex + 4 B per pixel in FP32). */
enum { GSIM_RASTER_SCRATCH_BYTES = 32 << 20 };
int gsim_raster_forward_noalloc(int dtype, int64_t n_verts, int64_t n_tris, const int32_t* d_tris, int height,
                                int width, const gsim_camera* camera, const void* x, void* image, void* stream);

/* ------------------------------------------------------------------------ */
/* SERVING ENGINE: continuous batching of rollout-gradient queries           */
/* ------------------------------------------------------------------------ */
/* A query is one gradient evaluation of the physical-parameter estimation task
 * (Sec. 5.1 "Physical parameter estimation": a loss on the simulated trajectory,
 * minimised over the body's physical parameters by gradient descent through the
 * simulator): one FP32 body
 * (n_bodies == 1) with parameters, start state and target; its answer is the loss
 * of its final positions (gsim_loss_mse) and the gradients of that loss, exactly
 * as gsim_rollout + gsim_loss_mse + gsim_rollout_backward would compute them on a
 * model of its own (bit for bit: a query's arithmetic does not depend on the other
 * queries in flight).
 *
 * The engine carves every admitted query's device buffers out of one
 * caller-owned pool (first fit), admits queued queries in FIFO order as pool
 * space and live slots free up, and advances all live queries by one
 * micro-step per gsim_engine_tick, running the micro-steps of every live query
 * in one element pass and one particle pass (forward and adjoint). */
typedef struct gsim_engine gsim_engine;

typedef struct {
    const gsim_model_desc* desc; /* one body, dtype GSIM_F32; read during submit */
    int n_steps;                 /* rollout length T */
    int ckpt_every;              /* checkpoint interval K */
    /* host inputs, copied during submit */
    const float* mu;             /* [n_tets] */
    const float* lam;            /* [n_tets] */
    const float* k_tri;          /* [n_tris] */
    const float* mass;           /* [n_particles] */
    const float* contact;        /* [4] = k_e, k_d, k_f, mu_f */
    const float* x0;             /* [3][n_particles] SoA */
    const float* v0;             /* [3][n_particles] */
    const float* target;         /* [3][n_particles] */
    /* host outputs, written when the query completes (NULL = not wanted);
     * they must stay valid until gsim_engine_poll reports the query */
    float* out_mu;
    float* out_lam;
    float* out_k_tri;
    float* out_mass;
    float* out_contact;          /* [4] */
} gsim_query;

typedef struct {
    int64_t id;
    float loss;
    double t_submit, t_admit, t_done; /* host steady-clock seconds */
    int status;  /* GSIM_OK, or GSIM_E_NONFINITE when the query's state or adjoint went
                    non-finite (its loss and gradients are then not meaningful); the
                    queries beside it are unaffected */
} gsim_result;

/* d_pool: caller-owned device memory (256-byte aligned); max_live: live query
 * slots; max_tiles: the most tiles one round's element or particle launch may hold
 * (sum over live queries of their planned element tiles, or of their particle tiles
 * of 256 particles; a round beyond it fails with GSIM_E_WORKSPACE). */
int gsim_engine_create(void* d_pool, size_t pool_bytes, int max_live, int64_t max_tiles, void* stream,
                       gsim_engine** out);
int gsim_engine_destroy(gsim_engine* engine);
/* Exact device bytes a query occupies while live with its own checkpoint interval
 * (its admission footprint; a query the engine runs with every state stored, see
 * gsim_engine_set_store_limit, occupies the bytes of interval 1). */
int gsim_engine_query_bytes(const gsim_query* query, size_t* bytes);
/* Queries whose footprint with every state stored (checkpoint interval 1) is at most
 * `bytes` run that way: the reverse pass reads each state instead of recomputing the
 * checkpoint segments, one forward micro-step fewer per step of the rollout but the
 * first of each segment.  Results are bitwise those of the query's own interval (the
 * recomputed states are the stored ones).  Default: pool_bytes / 64; 0 keeps every
 * query's own interval.  Applies to queries submitted afterwards. */
int gsim_engine_set_store_limit(gsim_engine* engine, size_t bytes);
/* Validates and plans the query (host), copies its inputs, queues it.  Refused before
 * it takes a slot: a non-finite mass, mu, lambda, k_tri, contact coefficient, start
 * state or target (GSIM_E_NONFINITE); mass, mu, lambda or k_tri not > 0, a negative
 * contact coefficient (GSIM_E_INVALID); GSIM_E_WORKSPACE if it can never fit in the
 * pool.  A query that goes non-finite while it runs completes with status
 * GSIM_E_NONFINITE in its gsim_result and frees its slot like any other. */
int gsim_engine_submit(gsim_engine* engine, const gsim_query* query, int64_t* id);
/* gsim_engine_submit in two parts, so that the host work of a query (validation as
 * above, planning, copying its inputs: about a millisecond for 10^4 elements) can run
 * off the thread that drives the engine.  gsim_engine_prepare touches no engine state
 * and may run on several threads at once; it returns an owned handle (its submit time
 * is the call's start).  gsim_engine_submit_prepared takes ownership of the handle in
 * every case, decides the query's checkpointing (gsim_engine_set_store_limit), checks
 * that it can fit the pool (GSIM_E_WORKSPACE) and queues it.  The engine's own calls
 * (submit, submit_prepared, tick, poll, the setters, stats, destroy) are made from one
 * thread at a time.  gsim_prepared_destroy frees a handle that is not submitted. */
typedef struct gsim_prepared gsim_prepared;
int gsim_engine_prepare(const gsim_query* query, gsim_prepared** out);
int gsim_engine_submit_prepared(gsim_engine* engine, gsim_prepared* prepared, int64_t* id);
int gsim_prepared_destroy(gsim_prepared* prepared);
/* Admits what fits (the admitted queries' set-up copies move as one staged batch),
 * then runs the set number of micro-step rounds: in each, one micro-step of every live
 * query, the forward and adjoint micro-steps of all queries in one element launch and
 * one particle launch.  A completed query's results are copied out asynchronously and
 * written to its output buffers by a later call once the copy has landed; when no
 * query is live or queued the call waits for every outstanding copy, so an engine
 * whose tick reports n_live = n_queued = 0 has delivered every answer (gsim_engine_poll
 * lists them).  n_live / n_queued: after the rounds. */
int gsim_engine_tick(gsim_engine* engine, int* n_live, int* n_queued);
/* Micro-step rounds per gsim_engine_tick (1..256, default 1): admission happens once
 * per tick, then every live query advances by that many micro-steps.  More rounds per
 * call spread the caller's per-tick cost over more device work. */
int gsim_engine_set_micro_steps(gsim_engine* engine, int rounds);
/* Completed queries since the last poll (at most max). */
int gsim_engine_poll(gsim_engine* engine, gsim_result* out, int max, int* n);
int gsim_engine_stats(const gsim_engine* engine, int64_t* ticks, int64_t* admitted, int64_t* completed,
                      double* mean_live, size_t* pool_free);

#ifdef __cplusplus
}
#endif

#endif /* GSIM_H */
