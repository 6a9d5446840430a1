/*
 * map.h -- C ABI of the MI355X (gfx950) implementation of the MAP block
 * update: the EGLM-MHD two-step scheme over a list of equal-sized AMR blocks
 * (Jiang, Fang & Chen, "MAP: an MHD code with AMR and parallelization").
 *
 * Every entry point is extern "C", takes plain pointers and sizes, returns a
 * map_status (0 = MAP_OK, negative = error) and never throws or aborts; the
 * text of the last error of the calling thread is map_last_error().  The
 * library never allocates or frees device memory: the caller owns the state
 * and a workspace (sizes from map_query) and passes HIP streams as void*.
 * Work is enqueued asynchronously on the given stream; only map_query,
 * map_status_flags and map_autotune synchronise.  A context is not thread
 * safe.  All device pointers must be 256-byte aligned.
 *
 * State layout (`U`): [slot][var][z][y][x], FP64 or FP32 (per
 * map_params.precision), with 16 cells per block edge and 2 ghost layers in
 * every active dimension (a padded tile of 20^d cells; 2-D tiles have one z
 * plane).  Variables: rho, m_x, m_y, m_z, B_x, B_y, B_z, e, psi (Sec. 2,
 * eqs. MHD-1..MHD-5; 2-D runs carry m_z and B_z).  Slots are the blocks in
 * Morton order (parents before their children, Sec. 4.1); map_query returns
 * the slot of every input key.
 */
#ifndef MAP_H
#define MAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct map_ctx map_ctx;  /* opaque, host memory owned by the library */

typedef int map_status;
enum {
    MAP_OK = 0,
    MAP_EINVAL = -1,        /* bad argument (null pointer, unknown enum, bad size) */
    MAP_ETREE = -2,         /* block list: duplicate, orphan, incomplete base or
                               sibling set, or 2:1 balance violated */
    MAP_ENOMEM = -3,        /* workspace smaller than map_query's workspace_bytes */
    MAP_EHIP = -4,          /* a HIP runtime call failed */
    MAP_ENONFINITE = -5,    /* reported by map_status_flags: non-finite state */
    MAP_ENEGPRESSURE = -6,  /* reported by map_status_flags: rho or p <= 0 */
    MAP_ESTATE = -7         /* call order: workspace not bound */
};

enum { MAP_FP64 = 0, MAP_FP32_MIXED = 1 };
enum { MAP_LF = 0, MAP_MMC = 1, MAP_WENO = 2 };
enum { MAP_MINMOD = 0, MAP_VANLEER = 1, MAP_PAPER_PHI = 2 };
enum { MAP_GLM_PAPER = 0, MAP_GLM_FASTSPEED = 1 };
enum { MAP_BC_PERIODIC = 0, MAP_BC_OUTFLOW = 1 };
enum { MAP_LAUNCH_BATCHED = 0, MAP_LAUNCH_PER_BLOCK = 1 };
enum { MAP_EST_VAR = 0, MAP_EST_BMAG = 1 };
enum { MAP_RUSANOV = 0, MAP_HLLC = 1 };
enum { MAP_COND_OFF = 0, MAP_COND_ISO = 1, MAP_COND_FIELD = 2 };

/* Scheme parameters (Sec. 2 and 3).
 *   precision     MAP_FP64: state and arithmetic in FP64.  MAP_FP32_MIXED:
 *                 FP32 state and flux arithmetic; pressure recovered in FP64
 *                 inside every flux/speed evaluation; CFL speeds, dt and the
 *                 totals in FP64.
 *   scheme        MAP_LF (TVD-LF: MUSCL-Hancock predictor, Rusanov flux,
 *                 Sec. 3.2), MAP_MMC (modified MacCormack, Sec. 3.1, 2-D
 *                 and 3-D) or MAP_WENO (third-order component-wise WENO face
 *                 states, Rusanov flux, TVD Runge-Kutta 2 in time with the
 *                 boundary procedure applied to the intermediate stage,
 *                 Sec. 3.3).
 *   limiter       LF: slope limiter; MMC: flux limiter (ratio-free form);
 *                 WENO: unused.
 *   glm_mode      MAP_GLM_PAPER: c_h = cfl dx_min/dt, psi factor glm_cd per
 *                 step; MAP_GLM_FASTSPEED: c_h = alpha_g, factor
 *                 exp(-dt c_h/glm_cr).
 *   eglm_sources  1: EGLM sources -(div B)B and -B.grad(psi); 0: plain GLM.
 *   riemann       face flux of LF and WENO: MAP_RUSANOV (the Lax-Friedrichs
 *                 flux printed in Sec. 3.2) or MAP_HLLC (the HLLC solver the
 *                 paper names for MHD, Sec. 3.2 and 5.2; the GLM pair takes
 *                 its exact upwind flux and the normal field its interface
 *                 value).  MMC has no Riemann solver: MAP_HLLC is MAP_EINVAL.
 *   cond_mode     thermal conduction by a subcycle after every step (Sec. 3.4):
 *                 MAP_COND_OFF; MAP_COND_ISO, face flux
 *                 -sqrt(kappa_i kappa_i+1)(T_i+1 - T_i)/dx; MAP_COND_FIELD,
 *                 the same face kappa times b_d (b . grad T) along the field
 *                 (the form of the paper's conduction test), b = B_f/|B_f|
 *                 with B_f the mean of the two cells' fields.  T = p/rho,
 *                 kappa = kappa0 T^kappa_exp (kappa_exp a multiple of 1/2 in
 *                 [0, 5]).  Sub-step limit dt_c = cfl dx_min^2 /
 *                 (n_dim max(kappa T/p)); the step is capped at
 *                 cond_max_sub dt_c (1..64) and split into
 *                 nsub = ceil(dt/dt_c) equal sub-steps.
 *   eta           uniform resistivity (0 = off), Sec. 3.5. */
typedef struct {
    int ndim, precision, scheme, limiter, glm_mode, eglm_sources, riemann, cond_mode,
        cond_max_sub;
    double gamma, cfl, glm_cd, glm_cr, eta, kappa0, kappa_exp;
} map_params;

/* One simulation: domain box, base-level blocks per dimension, boundary kind
 * per dimension and side.  Several simulations may share one context. */
typedef struct {
    double lo[3], hi[3];
    int nbase[3];
    int bc[3][2];
} map_sim_desc;

/* A block: simulation index, level (base = 1, as in Table 1 of the paper)
 * and block coordinates at that level. */
typedef struct {
    int sim, level, ix, iy, iz;
} map_block_key;

/* Per-simulation time-step record: dt, GLM speed c_h, psi damping factor
 * and the global maximum speed alpha_g (Sec. 2 and Sec. 3.7); with
 * conduction, the sub-step dt_sub = dt / nsub and the number of sub-steps
 * (both 0 without conduction). */
typedef struct {
    double dt, ch, damp, alpha, dt_sub;
    int nsub, reserved;
} map_dt;

typedef struct {
    size_t state_bytes;      /* bytes of U */
    size_t workspace_bytes;  /* bytes of the workspace to bind (tables, face
                                fluxes and one shadow copy of the state, which
                                map_advance, map_graph_run and map_autotune use) */
    int nblocks, nleaves, nsims, max_level, tile_cells, nvar;
    int n_prolong_items, n_reflux_blocks, n_face_buffers;
} map_sizes;

/* Validate the block tree and build the neighbour, ghost-descriptor,
 * restriction and reflux tables ("neighbour statistics", Sec. 4.2) on the
 * host.  keys lists every block, leaves and parents; every non-base block's
 * parent and all its siblings must be present, the base level complete, and
 * the tree 2:1 balanced across faces, edges and corners (with periodic
 * wrap).  No device work.  On success *ctx owns host memory until
 * map_destroy.  Errors: MAP_EINVAL, MAP_ETREE. */
map_status map_init_blocks(map_ctx **ctx, const map_params *params, int nsims,
                           const map_sim_desc *sims, int nblocks,
                           const map_block_key *keys);

/* Sizes and the Morton slot of each input key (slot_of_key[nblocks], may be
 * NULL): the blocks in the space-filling-curve order of Sec. 4.1 (Morton
 * here; the paper names Morton and Hilbert orders as equivalent), the
 * numbering of the block list of Table 1.  Host only. */
map_status map_query(const map_ctx *ctx, map_sizes *sizes, int32_t *slot_of_key);

/* Ghost source of every (input key, direction) -- the paper's neighbour
 * pointers (Table 1) resolved after periodic wrap or outflow clamping:
 * the input index of the same-level block whose interior cells fill that
 * direction's ghosts, -1 where the ghosts are prolongated from the parent
 * (the same-level block does not exist), -2 for direction 0 and for the
 * unused dz != 0 directions in 2-D.  neigh[nblocks][27], direction index
 * (dz+1)*9 + (dy+1)*3 + (dx+1).  Host only. */
map_status map_neighbors(const map_ctx *ctx, int32_t *neigh);

/* The part of the parents' ghost frames that the fill inside a cycle
 * refreshes by copies: every parent whose tile the prolongation of ghosts
 * reads (Sec. 4.3 step 6), with the ghost directions its limited-linear
 * stencil reaches (bit (dz+1)*9 + (dy+1)*3 + (dx+1) of dirs[i]) and the box
 * of padded cells that holds every cell it reads (box[i][0..2] = lowest
 * x, y, z, box[i][3..5] = highest; interior cells are 0..15, ghosts -2, -1,
 * 16, 17); the copies write the ghost cells of those directions inside the
 * box.  parent[i] is an input index.  Writes min(cap, count) entries and
 * the number of such parents to *count.  Host only. */
map_status map_fill_selection(const map_ctx *ctx, int cap, int32_t *parent, uint32_t *dirs,
                              int32_t *box, int *count);

/* Bind a caller-owned device workspace of at least workspace_bytes and
 * upload the tables on `stream` (asynchronous).  The workspace must outlive
 * every later call.  Errors: MAP_EINVAL, MAP_ENOMEM, MAP_EHIP. */
map_status map_bind_workspace(map_ctx *ctx, void *workspace_dev, size_t bytes, void *stream);

/* Convert every cell of U in place from primitive (rho, v, B, p, psi) to
 * conserved variables, e = p/(gamma-1) + rho v^2/2 + B^2/2 (Sec. 2). */
map_status map_prim_to_cons(map_ctx *ctx, void *U, void *stream);

/* Ghost layers of every block (Sec. 4.3, steps 3-7): same-level copies
 * including edge and corner neighbours, periodic wrap or zero-gradient
 * outflow at the domain edge, then minmod-limited conservative prolongation
 * from the parent's padded tile for ghosts whose same-level block does not
 * exist, level by level from coarse to fine. */
map_status map_fill_ghosts(map_ctx *ctx, void *U, void *stream);

/* Parent interiors = mean of their 2^d children (Sec. 4.3 step 1), from the
 * finest level down. */
map_status map_restrict(map_ctx *ctx, void *U, void *stream);

/* Whole-block prolongation (regrid initialisation): the interiors of the
 * blocks in slots_dev[n] (device int32 slots, level >= 2) from their
 * parents' padded tiles with the interpolation of Sec. 4.3 step 6. */
map_status map_prolong(map_ctx *ctx, void *U, const int32_t *slots_dev, int n, void *stream);

/* alpha_g = max over leaf interior cells of |v_d| + c_f,d per simulation,
 * then dt = cfl dx_min/(n_dim alpha_g) (Sec. 3.7; capped by the resistive
 * limit cfl dx_min^2/(n_dim eta)), c_h and the psi factor; writes
 * dt_dev[nsims] (device memory).  Speeds are computed in FP64. */
map_status map_cfl_dt(map_ctx *ctx, const void *U, map_dt *dt_dev, void *stream);

/* One update of every leaf of every simulation (Sec. 3.1, 3.2 or 3.3, all
 * directions together, Sec. 3.7) with EGLM sources, resistivity and psi
 * damping, writing the interiors of the leaves of U_out.  Ghost cells are
 * read where map_fill_ghosts would copy them from (Sec. 4.3): the interiors
 * of same-level blocks in U_in (leaves, and parents holding the restriction
 * of their children) and the block's own prolongated ghosts, so U_in needs
 * up-to-date interiors and prolongated ghost regions only.  LF and MMC:
 * U_out must not overlap U_in (MAP_EINVAL), since blocks read their
 * neighbours' old interiors while others are written.  WENO: both
 * Runge-Kutta stages; the first writes the workspace's shadow state, which
 * then gets restriction and the ghost procedure (Sec. 4.3) before the
 * second stage reads it, and U_out may equal U_in (partial overlap is
 * MAP_EINVAL).  U_out must not overlap the workspace.  Also stores the
 * fluxes of faces shared with leaves of another level (for WENO the mean of
 * both stages' fluxes), for map_reflux. */
map_status map_step(map_ctx *ctx, const void *U_in, void *U_out, const map_dt *dt_dev,
                    void *stream);

/* Coarse leaves next to finer leaves replace their face flux by the area
 * mean of the fine fluxes (Sec. 4.3 step 2).  Run after map_step. */
map_status map_reflux(map_ctx *ctx, void *U, const map_dt *dt_dev, void *stream);

/* The thermal-conduction subcycle of one step (Sec. 3.4), with the records
 * dt_dev that map_cfl_dt wrote for the step: nsub sub-steps of length dt_sub
 * per simulation, each advancing the energy of every leaf by the conduction
 * scheme of params.cond_mode and then refluxing, restricting, exchanging and
 * prolongating the energy.  The other variables do not change.  Run after the
 * step's reflux, restriction and ghost fill (map_advance and map_graph_run
 * do so); a no-op when conduction is off.  Uses the workspace's shadow state
 * as scratch.  Errors: MAP_EINVAL (null or workspace-overlapping U). */
map_status map_conduct(map_ctx *ctx, void *U, const map_dt *dt_dev, void *stream);

/* FP64 volume-weighted totals of the conserved variables over the leaves of
 * each simulation, totals_dev[nsims][9] (device), fixed reduction order. */
map_status map_totals(map_ctx *ctx, const void *U, double *totals_dev, void *stream);

/* For callers that cannot allocate device memory or bind scratch (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the result of map_totals, with the per-leaf partial sums in a fixed
 * library-owned device array instead of the workspace.  The array holds
 * MAP_STATIC_SCRATCH_DOUBLES doubles (4 MiB) per GPU, is held by every GPU
 * the library runs on until the process ends, and is shared by all calls
 * on that GPU: calls that overlap in time on one GPU (two streams, or two
 * threads) race and give undefined totals.  Nothing is allocated or freed;
 * every scratch entry a call reads is written earlier in the same call, so
 * no clearing is needed.  Needs a bound context (the tables stay in the
 * workspace).  Errors: MAP_EINVAL when nleaves x 9 exceeds the scratch
 * (more than MAP_STATIC_SCRATCH_DOUBLES / 9 = 58254 leaves) -- checked
 * before anything else, from the host -- and as map_totals. */
#define MAP_STATIC_SCRATCH_DOUBLES 524288
map_status map_totals_static(map_ctx *ctx, const void *U, double *totals_dev, void *stream);

/* Counters latched by the kernels since the last call, then cleared (the
 * paper's check of the solution inside the main loop, Fig. 1, and the
 * positivity fall-backs of Sec. 3.2):
 * [0] LF cells whose slopes fell back to zero, [1] face states replaced by
 * the cell average, [2] non-positive rho or p seen by the CFL pass,
 * [3] non-finite values seen by the CFL pass.  Synchronises `stream`.
 * Returns MAP_ENONFINITE or MAP_ENEGPRESSURE if [3] or [2] is non-zero. */
map_status map_status_flags(map_ctx *ctx, uint64_t counters[4], void *stream);

/* nsteps full cycles of the main loop of Fig. 1 (one global time step,
 * Sec. 3.7; the boundary procedure of Sec. 4.3 after the update instead of
 * before it, which is the same cycle shifted): cfl_dt, step, reflux,
 * restrict, then the ghosts the next step reads from a block's own tile
 * (copies into the frames of the parents that feed prolongation,
 * prolongation level by level), then the conduction subcycle when
 * params.cond_mode is on (map_conduct), with dt kept on the device (the
 * record of the last step is copied to dt_dev if it is not NULL).  Without
 * conduction, every cycle after the first of a call takes its dt from the
 * cycle before: that cycle's restriction also forms the CFL maxima of the
 * leaves with a parent (their values are final after reflux), a small pass
 * those of the leaves without one; the records equal those map_cfl_dt
 * would form from the state at the start of the cycle.  LF and MMC cycles
 * alternate between U and the workspace's shadow state, and an odd nsteps
 * ends with one device copy back into U; WENO cycles update U in place (the
 * shadow holds the stage).  On return U holds the interiors of every block
 * and its prolongated ghosts; the same-level ghost regions of leaves and of
 * parents hold unspecified values (map_fill_ghosts refreshes them).  Eager
 * launches on `stream`. */
map_status map_advance(map_ctx *ctx, void *U, map_dt *dt_dev, int nsteps, void *stream);

/* Same cycles (Fig. 1) and result as map_advance: the pair of cycles
 * U -> shadow -> U (WENO: two in-place cycles) is captured once per U into a HIP graph and
 * replayed nsteps / 2 times on `stream` (without conduction, two captures:
 * the first pair of a call forms its first dt, the later ones start from
 * the dt the pair before formed); an odd nsteps adds one eager cycle (and
 * for LF and MMC the copy back). */
map_status map_graph_run(map_ctx *ctx, void *U, map_dt *dt_dev, int nsteps, void *stream);

/* MAP_LAUNCH_BATCHED: one launch per stage over the joint work list of all
 * levels and simulations (persistent workgroups); MAP_LAUNCH_PER_BLOCK: one
 * launch per block (the plain baseline).  grid_step / grid_fill: number of
 * workgroups of the batched step / fill launches (0 = one per work item). */
map_status map_set_launch(map_ctx *ctx, int mode, int grid_step, int grid_fill);

/* Launch shapes of the batched stages (map_set_launch sets the first three). */
typedef struct {
    int mode;            /* MAP_LAUNCH_BATCHED or MAP_LAUNCH_PER_BLOCK */
    int grid_step;       /* workgroups of the update launch; 0 = one per work
                            item, > 0 = a persistent grid striding over them */
    int grid_fill;       /* the same for the parent-frame copies of the fill */
    int step_shape;      /* workgroup shape of the update: 2-D LF and WENO,
                            0 = 14 blocks in 4 waves, 1 = 7 blocks in 2 waves;
                            3-D FP32 LF and WENO, 0 = compiled for two
                            workgroups per CU (256 registers per lane), 1 =
                            for one (512); 0 elsewhere */
    int restrict_split;  /* restriction levels with fewer parents than this
                            take one workgroup per child, the others one per
                            parent; -1 = the number of compute units */
    int step_blocks_per_group;  /* read only: blocks per update workgroup */
    int cfl_in_update;   /* 2-D LF: whether the update forms the next cycle's
                            CFL maxima of the leaves without parent that no
                            reflux changes, in place of the CFL pass over them
                            (the same dt records bit for bit): -1 = in batched
                            launches over at least 4 leaves per CU (a small
                            tree's update, or a single block's, is
                            latency-bound and the pass costs little), 0 =
                            never, 1 = always */
    int cfl_in_update_on;  /* read only: 1 when cfl_in_update is in effect for
                              this tree and launch mode, else 0 */
} map_launch;

map_status map_get_launch(const map_ctx *ctx, map_launch *out);
/* Errors: MAP_EINVAL (unknown mode, negative grid, a step_shape the
 * context's scheme and precision do not have, restrict_split < -1). */
map_status map_set_launch_config(map_ctx *ctx, const map_launch *in);

/* The launch autotuner: on U, with HIP events, times the update over its
 * workgroup shapes and persistent grids (multiples of the CU count below the
 * work-item count, and one workgroup per item), then the fill copies over
 * the grids, then the restriction over the per-child split, and keeps the
 * fastest of each (one untimed launch, then the best of five), a candidate
 * replacing the choice so far only when faster by more than 0.5 %
 * (map_get_launch reports them); writes grid_step and
 * grid_fill to chosen[2] if not NULL.  Synchronises `stream`.  The trial
 * updates (for WENO, first stages) write the shadow state; U's interiors are
 * not changed (the trial restrictions and copies rewrite parent interiors
 * and parent frames with the same values). */
map_status map_autotune(map_ctx *ctx, void *U, int *chosen, void *stream);

/* ---- regrid (Sec. 4.5) ------------------------------------------------ */

/* Error estimator of Sec. 4.5, per cell,
 *   (bias |D u| / (|u| + eps) + (1 - bias) |D2 u| / (|D u| + filt (|u| + eps)))
 *     * ratio^(xi (L - 1)),
 * |D u| = (sqrt 3 / 2) (sum_d (u_{+d} - u_{-d})^2)^(1/2),
 * |D2 u| = (sum_d (u_{+d} - 2 u + u_{-d})^2)^(1/2),
 * for each criterion i: u = conserved variable var[i] (MAP_EST_VAR) or |B|
 * (MAP_EST_BMAG), with its own eps[i] (the paper: 1e-12 for rho, p, T and
 * 0.1 for v, B); filt = 0.05, bias = 0.6, ratio = 2 in the paper. */
typedef struct {
    int ncrit;      /* criteria used, 1..4 */
    int mode[4];    /* MAP_EST_VAR or MAP_EST_BMAG */
    int var[4];     /* conserved variable index for MAP_EST_VAR */
    double eps[4];
    double filt, bias, ratio, xi;
} map_estimator;

/* Largest estimate of every block over its interior and the first ring of
 * ghost cells (the paper checks every cell covering the ghost region), the
 * maximum over the criteria, computed in FP64 from U (either precision):
 * err_dev[nblocks] (device, by slot).  Ghost cells are read where the ghost
 * descriptors point, so U may come straight from map_advance.  Parents are
 * evaluated on their restricted data (they are the candidates for
 * destroying their children).  Errors: MAP_EINVAL (bad criteria). */
map_status map_estimate(map_ctx *ctx, const void *U, const map_estimator *est, double *err_dev,
                        void *stream);

typedef struct {
    double tau_refine;   /* a leaf with a larger estimate is refined */
    double tau_coarsen;  /* a block whose children are all leaves, none refined,
                            loses them when its own estimate is smaller */
    int max_level;       /* finest level allowed (base = 1) */
} map_regrid_params;

/* The block tree after one regrid (Sec. 4.5), host only: flagged leaves
 * below max_level are refined, blocks whose estimate is below tau_coarsen
 * lose their children, and the result is closed under 2:1 balance across
 * faces, edges and corners (a leaf that would touch a leaf two levels finer
 * is refined instead, or its coarsening is cancelled).  err_host[nblocks]
 * by slot (as map_estimate writes it).  Writes the new keys, sorted by
 * (sim, level, ix, iy, iz), to keys_out[capacity] and their count to *nout;
 * MAP_ENOMEM (with *nout set) if capacity is too small. */
map_status map_regrid(const map_ctx *ctx, const double *err_host, const map_regrid_params *rp,
                      map_block_key *keys_out, int capacity, int *nout);

/* When to regrid next (Sec. 4.5): per simulation, the simulated time the
 * fastest wave needs to cross the 2 n_g buffer cells the estimate covers,
 * dtr = c_r 2 n_g dx_min / alpha_g (dx_min the finest leaf cell width,
 * alpha_g from the record; equal to c_r 2 n_g n_dim dt / c_cfl when dt is
 * the CFL step), written to dtr_host[nsims], and the number of whole steps
 * of the record's dt in it, at least 1, to steps_host[nsims].  dt_host:
 * host copies of the last step's records.  Host only.  Errors: MAP_EINVAL
 * (null argument, c_r <= 0, a record without a positive dt). */
map_status map_regrid_interval(const map_ctx *ctx, const map_dt *dt_host, double c_r,
                               double *dtr_host, int *steps_host);

/* Moves a state onto a new tree of the same simulations and parameters
 * (Sec. 4.5 with the boundary procedure of Sec. 4.3): blocks present in
 * both trees are copied; blocks new in dst (children of src leaves) are
 * filled by the conservative prolongation of Sec. 4.3 step 6 from their
 * parent's padded tile; then every parent is restricted from its children
 * and all ghost frames are filled.  Blocks that lose their children keep
 * their restricted data as leaf data.  Both contexts must be bound; a dst
 * block absent from src must have its parent in src (one level of
 * refinement per regrid).  Synchronises `stream`.  Errors: MAP_EINVAL,
 * MAP_ETREE, MAP_ESTATE, MAP_EHIP. */
map_status map_remap(map_ctx *dst, void *U_dst, const map_ctx *src, const void *U_src,
                     void *stream);

const char *map_last_error(void);
void map_destroy(map_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
