/*
 * lts.h -- C ABI of the MI355X (gfx950) octree local-timestepping library.
 *
 * Method: "Scalable Local Timestepping on Octree Grids" (Fernando & Sundar,
 * arXiv 2011.10570).  A method-of-lines system du/dt = F(u) (eq. evolve_eq) is
 * discretised on a periodic, balanced linear octree over [-1,1]^3 whose leaves
 * carry 5^3 octant-local nodes (Sec. 3.2, fig. dg_to_cg "octant local nodes").
 * The octree is cut into uniformly refined blocks (Sec. 3.2.5, fig. oct_to_blocks);
 * each RK stage builds ghost-padded blocks (unzip, Sec. 3.3, fig. unzip), applies
 * sixth-order finite differences with Kreiss-Oliger dissipation on the block
 * grid (rhs), scatters the result back to the octants (zip) and, after the last
 * stage, forms the RK update (eq. rk_schemes).  Global timestepping (GTS,
 * Alg. 1) steps every block with the finest dt; local timestepping (LTS,
 * Alg. 2 with the schedule of fig. blk_loop) steps level-l blocks with
 * dt_l = 0.25 h_l and converts a neighbour's stored RK stages to the receiver's
 * step with the correction operators of eqs. fc_1 / fc_2.
 *
 * Conventions
 *   Status.     Every entry point returns lts_status (0 = LTS_OK); on error
 *               lts_last_error() gives a message for the calling thread.  No C++
 *               exception and no abort crosses this boundary.
 *   Ownership.  lts_mesh / lts_sim handles (and the device tables they upload)
 *               belong to the library; free them with *_destroy.  State and
 *               stage arrays are owned by the caller and passed as raw device
 *               pointers; the library only borrows them.
 *   Streams.    Device work is enqueued asynchronously on the hipStream_t given
 *               (passed as void*, NULL = default stream); only calls that return
 *               host results synchronise that stream.  A kernel fault surfaces as
 *               LTS_EDEVICE from the next call that synchronises.
 *   Layouts.    All device arrays are contiguous.  n = nodes per octant side
 *               (5 by default, or 7; lts_mesh_spec.nodes), ni = n - 1.
 *               U  : double [2][F][N][n^3]       two state buffers ("parities")
 *               K  : double|float [p][F][N][n^3] RK stages (float in FP32-RHS mode)
 *               node index within an octant: i + n j + n^2 k (i fastest, along x);
 *               octants in Morton order (child index x + 2y + 4z), the order of
 *               lts_mesh_export(LTS_EXPORT_LEAVES).
 *               Padded blocks (lts_unzip output / lts_rhs input): per field, the
 *               blocks of the call in call order, block b holding S^3 doubles,
 *               S = ni m_b + 7, point (i,j,k) in [-3, ni m + 3]^3 at
 *               ((k+3) S + (j+3)) S + (i+3).
 *               Block grids (lts_rhs output / lts_zip input): per field, blocks
 *               in call order, G^3 values each, G = ni m_b + 1, (k G + j) G + i.
 *   Buffers.    A block's step writes its new state into the U buffer its step
 *               record does not read.  Which buffer a block reads follows from the
 *               step counters: a level-l block's step index at substep j of
 *               coarse step n is s = n 2^(l - lmin) + (j >> (lmax - l)) in LTS and
 *               s = n 2^(lmax - lmin) + j in GTS; its record reads U[s & 1] and
 *               its update writes U[(s + 1) & 1].
 */
#ifndef LTS_H_
#define LTS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LTS_OK = 0,
  LTS_EINVAL = 1,        /* bad argument, size or layout                       */
  LTS_ENOMEM = 2,        /* host or device allocation failed                   */
  LTS_EDEVICE = 3,       /* HIP runtime error (launch, copy, kernel fault)     */
  LTS_EUNBALANCED = 4,   /* a ghost source is not within one level             */
  LTS_ENONFINITE = 5,    /* a NaN/Inf was found in the state                   */
  LTS_EUNSUPPORTED = 6   /* combination not built (equation/precision/tile)    */
} lts_status;

enum { LTS_MAX_LEVEL = 16 };

enum { LTS_CRIT_BALL = 0, LTS_CRIT_ANNULUS = 1 };
enum { LTS_MODE_LTS = 0, LTS_MODE_GTS = 1 };
/* Equations: the linear wave system (u, v); vacuum Maxwell (E, B); the
 * non-linear wave of Sec. 4.2 (eqs. lsm, chi, phi: fields chi, phi, source
 * -c sin(2 chi) / r^2) with, on a bounded mesh, the radiative outer boundary. */
enum { LTS_EQ_WAVE = 0, LTS_EQ_MAXWELL = 1, LTS_EQ_NLWAVE = 2 };
/* Domain: periodic [-1, 1]^3, or [-1, 1]^3 bounded by its outer faces. */
enum { LTS_BOUNDARY_PERIODIC = 0, LTS_BOUNDARY_OUTER = 1 };
enum { LTS_FP64 = 0, LTS_FP32_RHS = 1 };
enum { LTS_RK4 = 0, LTS_SSPRK3 = 1 };

/* Export kinds for lts_mesh_export (all int32 rows unless stated). */
enum {
  LTS_EXPORT_LEAVES = 0,     /* [N][4]  anchor x, y, z (level-L octant units), level          */
  LTS_EXPORT_BLOCKS = 1,     /* [B][6]  first leaf, m, level, anchor x, y, z                  */
  LTS_EXPORT_UNZIP_MAP = 2,  /* [sum_b S_b^3][5] source leaf, kind, 2*px, 2*py, 2*pz            */
  LTS_EXPORT_SCHEDULE = 3,   /* for j = 0..2^dL-1: count, then that many block indices         */
  LTS_EXPORT_TILES = 4,      /* [T][8] tiles of the fused kernel (see lts_mesh_set_tile)       */
  LTS_EXPORT_GHOSTS = 5      /* [E][2] ghost table: coarser source leaf, then its receivers'
                              * level (bits 0-4) | the half-node box they read, 4 bits per
                              * bound from bit 5: x lo, x hi, y lo, y hi, z lo, z hi
                              * (0..2(n-1) for n nodes per side); finest receivers first   */
};

/* Unzip-map source kinds (Sec. 3.3): own octant, same-level neighbour, finer
 * neighbour (f->c injection), coarser neighbour (c->f interpolation), and on a
 * bounded mesh a point beyond the outer faces (no source, leaf -1). */
enum { LTS_SRC_OWN = 0, LTS_SRC_SAME = 1, LTS_SRC_FINE = 2, LTS_SRC_COARSE = 3, LTS_SRC_NONE = 4 };

/* Refinement criterion around an integer centre (node units at level l_max:
 * ni * 2^l_max per side, x = -1 + 2 X / (ni * 2^l_max), ni = nodes - 1 the
 * node intervals per octant side).  A level-l leaf is split
 * if, with dmin / dmax the smallest / largest periodic distance from the centre
 * to the leaf's closed box,
 *   LTS_CRIT_BALL:    dmin^2 < r2[l]
 *   LTS_CRIT_ANNULUS: rlo2[l] < dmax^2 and dmin^2 < rhi2[l]
 * Negative entries never refine.  (Integer stand-in for the wavelet criterion
 * of Sec. 3.2.2 so that meshes are reproducible bit for bit.) */
typedef struct {
  int32_t kind;
  int32_t center[3];
  int64_t r2[LTS_MAX_LEVEL];
  int64_t rlo2[LTS_MAX_LEVEL];
  int64_t rhi2[LTS_MAX_LEVEL];
} lts_criterion;

/* Mesh specification.  Either criteria (refine from the uniform level l_min) or an
 * explicit leaf list (int32 [n_leaves][4] = anchor x, y, z in level-l_max octant
 * units, level; must tile the domain) is used.  Octants carry nodes^3 DG nodes.
 * The result is always closed under the balance the three ghost layers of a block
 * need to reach only leaves one level apart:
 *   nodes = 5: ghost-reach balance, a level-l leaf is split while a leaf of level
 *              >= l+2 lies within 3 h_l of it (2:1 balance of Sec. 3.2.3
 *              extended: the layers reach 3/4 into a neighbouring octant);
 *   nodes = 7: the paper's 2:1 balance (face, edge and corner contact; the
 *              layers reach half-way into a neighbouring octant). */
typedef struct {
  int32_t l_min, l_max;      /* 0 <= l_min <= l_max < LTS_MAX_LEVEL, l_max <= 10 */
  int32_t block_cap;         /* max octants per block side: 1, 2 or 4              */
  int32_t n_criteria;
  const lts_criterion* criteria;   /* host */
  int64_t n_leaves;          /* > 0: use the explicit leaf list                    */
  const int32_t* leaves;     /* host */
  int32_t boundary;          /* LTS_BOUNDARY_PERIODIC (0) or LTS_BOUNDARY_OUTER: on a */
                             /* bounded mesh distances, balance and neighbours stop */
                             /* at the outer faces                                   */
  int32_t nodes;             /* nodes per octant side: 5 (0 means 5) or 7 (the      */
                             /* paper's 7^3 points per octant, Sec. 4.5)            */
} lts_mesh_spec;

typedef struct {
  int64_t n_oct, n_blocks, n_tiles;
  int32_t L;                 /* coordinate resolution (spec l_max)                  */
  int32_t lmin, lmax;        /* levels present                                      */
  int32_t n_substeps;        /* 2^(lmax - lmin)                                     */
  int32_t tile;              /* current fused-kernel tile side (1, 2 or 4)          */
  int64_t level_count[LTS_MAX_LEVEL];   /* leaves per level                          */
  int64_t unzip_points;      /* sum over blocks of (ni m + 7)^3, ni = nodes - 1      */
  int64_t grid_points;       /* sum over blocks of (ni m + 1)^3                     */
  int64_t node_updates_lts;  /* DG node-updates per coarse step, LTS (eq. w_nuts)   */
  int64_t node_updates_gts;  /* same for GTS (eq. w_uts)                             */
  double s_est;              /* speedup model 1/S of eq. invS, inverted             */
  double s_max;              /* |W| / alpha_0                                        */
  int64_t table_bytes;       /* device memory of the mesh's tables (all tile sides) */
  int64_t ghost_entries;     /* coarser ghost sources of the fused tiles: a sim's   */
                             /* ghost-table scratch is ghost_entries x F x 729 doubles */
  int32_t boundary;          /* the spec's boundary                                  */
  int32_t nodes;             /* nodes per octant side (5 or 7)                       */
} lts_mesh_info;

typedef struct lts_mesh lts_mesh;
typedef struct lts_sim lts_sim;
typedef struct lts_batch lts_batch;

/* Device arrays of one state (see Layouts).  nfields: 2 (wave) or 6 (Maxwell). */
typedef struct {
  void* U;                   /* double [2][F][N][n^3], n = nodes per octant side    */
  void* K;                   /* [p][F][N][n^3], double (LTS_FP64) / float (FP32_RHS) */
  int32_t nfields;
  int32_t precision;         /* LTS_FP64 / LTS_FP32_RHS                             */
  int32_t tableau;           /* LTS_RK4 / LTS_SSPRK3                                */
} lts_stage_view;

/* Schedule position: substep j in [0, 2^dL) of coarse step n, and the mode.
 * The time case of every ghost relation and the U buffer of every step record
 * follow from it (see Buffers). */
typedef struct {
  int32_t substep;
  int32_t mode;              /* LTS_MODE_LTS / LTS_MODE_GTS                          */
  int64_t coarse_step;
} lts_position;

typedef struct {
  double ko_sigma;           /* Kreiss-Oliger strength (0.1 default)                */
  double nl_coeff;           /* LTS_EQ_NLWAVE: coefficient c of the source (1 in   */
                             /* the paper's runs, 0 gives the linear wave)          */
} lts_rhs_params;

/* ---- errors ---------------------------------------------------------------- */
const char* lts_last_error(void);
const char* lts_version(void);

/* ---- mesh (host; Sec. 3.2) ----------------------------------------------- */
/* Build leaves (refinement + balance), blocks, tiles, unzip source tables and the
 * level schedule on the host.  No device call is made; tables are uploaded on
 * first device use.  Errors: LTS_EINVAL (bad spec / leaves do not tile),
 * LTS_EUNBALANCED (internal check), LTS_ENOMEM. */
lts_status lts_build_mesh(const lts_mesh_spec* spec, lts_mesh** out);
void lts_mesh_destroy(lts_mesh* mesh);
lts_status lts_mesh_query(const lts_mesh* mesh, lts_mesh_info* info);
/* Copy a table to host memory `buf` of `cap` bytes; `*needed` receives the size
 * in bytes (call with buf = NULL to ask).  LTS_EINVAL if cap is too small. */
lts_status lts_mesh_export(const lts_mesh* mesh, int32_t kind, void* buf, size_t cap, size_t* needed);
/* Fused-kernel tile side t (1, 2 or 4): a block of side m is cut into tiles of
 * side min(m, t).  Tiles of side 1 and 2 sit whole in LDS; side-4 tiles (whole
 * 4^3-octant blocks, wave equation only) are streamed plane by plane after a
 * pre-pass that prolongates their coarser ghosts.  FP64 results do not depend on
 * t (bitwise); in FP32-RHS mode the FP32 stencils run on Y minus one FP64
 * reference value per tile, so results differ between tile sides at FP32
 * rounding.  Maxwell needs t = 1 or 2 (side-2 Maxwell tiles hold 153 KB of LDS:
 * one workgroup per CU); batches (lts_batch_*) need t = 1 or 2.
 * LTS_EINVAL for other t or while a sim of the mesh is attached to a batch. */
lts_status lts_mesh_set_tile(lts_mesh* mesh, int32_t tile);
/* Exact-rational stage conversion weights w^[case][stage][i] as float64 (eqs.
 * rk_crrection, fc_1, fc_2 with K = C P D), cases (delta, rho) = (0,1), (0,1/2),
 * (0,2), (1,2); plus a[p][p] and b[p].  out: double[4*p*p + p*p + p] (host). */
lts_status lts_coefficients(int32_t tableau, double* out, size_t cap);

/* ---- unfused hot path (one call per phase; Sec. 3.3, Alg. 1/2) --------------- */
/* `blocks` is a HOST array of nb block indices (NULL = every block of B_j at
 * `pos`, in block order).  All other pointers are device pointers. */

/* a2: padded stage state Y_s = U0 + dt_r sum_i w^_{s,i}(case) K_i of every padded
 * point of the listed blocks, with f->c injection and tensor degree-4 Lagrange
 * c->f interpolation (Sec. 3.3; eqs. fc_1/fc_2).  stage is 0-based. */
lts_status lts_unzip(lts_mesh* mesh, const lts_stage_view* view, int32_t stage,
                     const lts_position* pos, const int32_t* blocks, int32_t nb,
                     double* padded, void* stream);
/* a3: block RHS on the (ni m+1)^3 block grid: wave du = v + KO(u), dv = Lap6 u +
 * KO(v); Maxwell dE = curl6 B + KO(E), dB = -curl6 E + KO(B); KO(f) =
 * sigma/(64h) sum_axes (1,-6,15,-20,15,-6,1) f.  precision LTS_FP32_RHS evaluates
 * the stencils in float (output float), else double. */
lts_status lts_rhs(lts_mesh* mesh, int32_t equation, const lts_rhs_params* params,
                   const double* padded, int32_t precision, const int32_t* blocks,
                   int32_t nb, void* k_block, void* stream);
/* a5: block grid -> every DG node of the blocks' octants (intra-block duplicates
 * get the block grid value).  k_octant: [F][N][n^3] (a K_s slice), element type
 * from precision. */
lts_status lts_zip(lts_mesh* mesh, int32_t nfields, int32_t precision, const void* k_block,
                   const int32_t* blocks, int32_t nb, void* k_octant, void* stream);
/* a4: out = U0 + dt_l sum_i coef_i K_i on the listed blocks' octants, dt_l the
 * block's step (finest step in GTS).  out = NULL writes the block's other U buffer
 * (the RK update of eq. rk_schemes when coef = b). */
lts_status lts_rk_stage(lts_mesh* mesh, const lts_stage_view* view, const double* coef,
                        int32_t ncoef, const lts_position* pos, const int32_t* blocks,
                        int32_t nb, double* out, void* stream);

/* a6: the fused stage (unzip + rhs + zip [+ RK update at the last stage]) for
 * every block of B_j, one launch over LDS-resident tiles. */
lts_status lts_fused_stage(lts_mesh* mesh, const lts_stage_view* view, int32_t equation,
                           const lts_rhs_params* params, int32_t stage,
                           const lts_position* pos, void* stream);

/* The same fused stage for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): it
 * calls no hipMalloc / hipFree and no allocating library routine.  Its scratch
 * (the coarse-step counter and the stage's ghost table) is a fixed 64 MiB device
 * array of the library, one per GPU, held until the process ends; its address is
 * looked up on the first call on each device.  The caller still owns U and K.
 * Requirements and errors:
 *   - the mesh's tables must already be on the current device (any earlier
 *     device call on the mesh uploads them: lts_sim_create, lts_fused_stage,
 *     lts_unzip, ...), else LTS_EINVAL;
 *   - the stage's ghost table (entries with receiver level >= the substep's
 *     lowest active level, F x 729 doubles each) must fit in 64 MiB - 256 B,
 *     else LTS_EINVAL before any device work;
 *   - all calls on one GPU share that GPU's scratch, which keeps the last call's
 *     contents: calls that overlap on one GPU (different streams or host threads
 *     without ordering) race.  Calls ordered on one stream are safe.
 * Results are bitwise those of lts_fused_stage with the same arguments. */
lts_status lts_fused_stage_noalloc(lts_mesh* mesh, const lts_stage_view* view, int32_t equation,
                                   const lts_rhs_params* params, int32_t stage, const lts_position* pos,
                                   void* stream);

/* Launch shape of the fused stage kernels (process-wide; used by every later
 * fused launch and graph capture): threads per workgroup of the side-2 LDS tile
 * kernels (256 or 512, default 512; side-1 tiles always run 256) and of the
 * streaming kernel of side-4 tiles (256 or 512, default 512), and the cap on the
 * grid in workgroups (default 65536: one
 * workgroup per tile up to that many tiles; below the tile count, workgroups
 * walk several tiles each; batched launches use at most 4096).  Results do not
 * depend on it.  LTS_EINVAL for other values. */
lts_status lts_set_launch(int32_t threads, int32_t max_workgroups, int32_t stream_threads);
lts_status lts_get_launch(int32_t* threads, int32_t* max_workgroups, int32_t* stream_threads);
/* Launch shape of batched launches (lts_batch_*): threads per workgroup of their
 * side-2 tile kernels (256 or 512, default 512; side-1 tiles always run 256)
 * and the cap on their grids (default
 * 4096; workgroups walk several tiles of the union).  Results do not depend on
 * it; a captured round is redone when it changes. */
lts_status lts_set_batch_launch(int32_t threads, int32_t max_workgroups);
lts_status lts_get_batch_launch(int32_t* threads, int32_t* max_workgroups);

/* ---- simulation driver (a7; Alg. 1 / Alg. 2) ---------------------------------- */
lts_status lts_sim_create(lts_mesh* mesh, int32_t equation, int32_t precision, int32_t tableau,
                          const lts_rhs_params* params, lts_sim** out);
/* Bind caller-owned device arrays (see lts_stage_view).  U[0] must hold the
 * initial state; the sim's coarse-step counter is reset to 0. */
lts_status lts_sim_bind(lts_sim* sim, void* U, void* K);
/* Flags of lts_advance. */
enum {
  LTS_ADVANCE_GRAPH = 1,         /* capture one coarse step in a hipGraph on first use, replay it */
  LTS_ADVANCE_CHECK_FINITE = 2,  /* count non-finite values written by the RK updates of these
                                    steps (inside the last stage's kernels), synchronise the
                                    stream at the end and return LTS_ENONFINITE if any */
  LTS_ADVANCE_POISON = 4         /* race check (debug): before every stage, set the stage's K
                                    entries of the stage's active octants to NaN.  A stage that
                                    read its own K before writing it (or any K that no stage of
                                    the step has written yet) would carry NaN into the state,
                                    which LTS_ADVANCE_CHECK_FINITE reports.  Results are
                                    otherwise unchanged; GTS leaves the unstored last K NaN */
};
/* Advance n coarse steps (T += n dt_lmin) with the fused kernels (Alg. 1 / Alg. 2);
 * a mesh of 7-node octants runs the same schedule on the phase kernels (unzip,
 * rhs, zip, RK update; its first call allocates their block lists and scratch).
 * flags: LTS_ADVANCE_* (1 alone = graph, the former use_graph != 0).  Without
 * LTS_ADVANCE_CHECK_FINITE the call is asynchronous. */
lts_status lts_advance(lts_sim* sim, int64_t n_coarse_steps, int32_t mode, int32_t flags,
                       void* stream);
/* Same with the unfused phase kernels (unzip, rhs, zip, rk_stage). */
lts_status lts_advance_unfused(lts_sim* sim, int64_t n_coarse_steps, int32_t mode, void* stream);
/* Gather the current state of every octant into out ([F][N][n^3] doubles). */
lts_status lts_sim_current(lts_sim* sim, double* out, void* stream);
/* Restart from a checkpoint taken at a coarse-step boundary: `state` (device,
 * [F][N][n^3] doubles, as lts_sim_current returns it) becomes the state of every
 * octant after `coarse_step` coarse steps in `mode`; the sim's counter is set to
 * it.  Continuing from here gives bitwise the results of the uninterrupted run
 * (nothing of an earlier coarse step is read after its end: every level starts
 * a step at substep 0).  LTS_EINVAL for a sim attached to a batch. */
lts_status lts_sim_restore(lts_sim* sim, const double* state, int64_t coarse_step, int32_t mode, void* stream);
int64_t lts_sim_coarse_step(const lts_sim* sim);
void lts_sim_destroy(lts_sim* sim);

/* ---- batches: several simulations per launch (continuous batching) ---------------
 * A batch advances up to `capacity` (<= 256) independent simulations of one
 * equation, precision, tableau and mode together, by rounds.  In round r a sim
 * that joined at round r0 runs its own substep j = (r - r0) mod 2^(lmax-lmin)
 * (Alg. 2 schedule, fig. blk_loop, of its own mesh) of coarse step
 * n0 + (r - r0) div 2^(lmax-lmin); every stage of a round is one launch per tile
 * side over the union of the active tiles of all attached sims (the
 * sims' meshes, level ranges and sizes may differ).  Each sim's arithmetic is the
 * one lts_advance performs: its results are bitwise those of running it alone.
 * A batch is used from one host thread and one stream. */
typedef struct {
  int64_t round;             /* next round to run                                   */
  int64_t rounds_to_drain;   /* rounds until every attached sim is done             */
  int32_t attached, capacity;
} lts_batch_info;

lts_status lts_batch_create(int32_t equation, int32_t precision, int32_t tableau, int32_t mode,
                            int32_t capacity, lts_batch** out);
/* Attach a bound sim for n coarse steps (n 2^(lmax-lmin) rounds) starting at the
 * next round.  While attached, the sim is driven only by the batch (lts_advance,
 * lts_sim_bind and lts_mesh_set_tile of its mesh return LTS_EINVAL).  When its
 * rounds are done it is released by itself and its coarse-step counter advanced.
 * n = 0 attaches nothing.  LTS_EINVAL: batch full, mismatched equation /
 * precision / tableau / device, or a mode that differs from the sim's history. */
lts_status lts_batch_attach(lts_batch* batch, lts_sim* sim, int64_t n_coarse_steps);
/* Release an attached sim early, at one of its coarse-step boundaries (else
 * LTS_EINVAL); its counter advances by the coarse steps it completed. */
lts_status lts_batch_detach(lts_batch* batch, lts_sim* sim, void* stream);
/* Enqueue n rounds on `stream` (asynchronous; a table upload after attach or
 * early release goes through pinned memory and waits only for the previous
 * upload).  use_graph != 0 captures one round (p stages x 2 tile sides + the
 * device round counter) as a hipGraph and replays it; the capture is redone when
 * a sim joins or leaves early or the launch shape changes (sims that reach T
 * keep it valid: they are inactive in later rounds). */
lts_status lts_batch_run(lts_batch* batch, int64_t n_rounds, int32_t use_graph, void* stream);
lts_status lts_batch_query(const lts_batch* batch, lts_batch_info* info);
/* Rounds the sim still takes part in (0 when it is not attached). */
int64_t lts_sim_rounds_left(const lts_sim* sim);
/* Waits for the batch's enqueued work, releases sims still attached (their
 * counters are not advanced) and frees the batch. */
void lts_batch_destroy(lts_batch* batch);

/* All of sims[0..n) (n <= 256) advanced n_coarse_steps coarse steps in one batch
 * (create, attach, run graph-captured rounds until drained, destroy). */
lts_status lts_batch_advance(lts_sim* const* sims, int32_t n, int64_t n_coarse_steps,
                             int32_t mode, void* stream);

/* ---- remeshing at a coarse-step boundary (Sec. 3.2.2, Sec. 5) -------------------------
 * The octree follows the wavelet criterion: the wavelet indicator of an octant
 * is the largest |v - I2 v| over fields and over its nodes off the every-second-
 * node grid, I2 the tensor degree-2 Lagrange interpolant of its 27 nodes at
 * positions 0, 2, 4 (the failure to be interpolated from one level coarser).
 * `state` is a device array [F][N][125] (lts_sim_current's layout). */
/* Host arrays of N doubles: the indicator of every leaf, and at the first leaf of
 * every complete family of 8 same-level siblings the indicator of their parent
 * (whose nodes are nodes of the children), -1 at the other leaves.  Synchronises. */
lts_status lts_remesh_indicators(lts_mesh* mesh, int32_t nfields, const double* state, double* leaf_ind,
                                 double* family_ind, void* stream);
/* The new octree: a leaf of level < l_max splits where its indicator exceeds eps,
 * a family of level > l_min none of whose leaves splits merges where its parent's
 * indicator is below eps / 4; then the ghost-reach balance.  Same coordinates (L),
 * domain and block cap as `mesh`; free *out with lts_mesh_destroy.  Synchronises. */
lts_status lts_remesh(lts_mesh* mesh, int32_t nfields, const double* state, double eps, int32_t l_min,
                      int32_t l_max, lts_mesh** out, void* stream);
/* Intergrid transfer of a state between meshes of one domain whose leaves nest:
 * a leaf of `to` inside a leaf of `from` takes the tensor degree-4 Lagrange
 * interpolant of that leaf at its nodes (a copy at equal levels); a leaf of `to`
 * that is the union of 8 leaves of `from` one level finer takes their coincident
 * nodes.  state_to: device [F][N_to][125].  LTS_EINVAL if the meshes do not nest
 * that way.  Synchronises. */
lts_status lts_transfer(lts_mesh* from, lts_mesh* to, int32_t nfields, const double* state_from, double* state_to,
                        void* stream);

/* ---- reductions ----------------------------------------------------------------- */
/* Per field volume-weighted l2 and max norm of (a - b) over all DG nodes (b may
 * be NULL) and the number of non-finite values in a.  out (host):
 * double[2F + 1] = l2[F], linf[F], nonfinite.  Synchronises the stream. */
lts_status lts_norms(lts_mesh* mesh, int32_t nfields, const double* a, const double* b,
                     double* out, void* stream);
/* Device copy of nbytes (bandwidth probe used as the measured HBM reference). */
lts_status lts_copy_probe(const void* src, void* dst, size_t nbytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LTS_H_ */
