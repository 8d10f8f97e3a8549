// Kernel launch interface between the C ABI layer and the HIP kernels (k_*.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lts {

// Arguments of one stage launch.  w holds the stage's conversion weights per
// time case (w[case][i], eqs. fc_1/fc_2); b the RK weights.
struct StageParams {
  const double* U;      // [2][F][N][n^3], n = ni + 1 nodes per octant side
  double* Uw;           // same array, written by the last stage
  const void* K;        // [p][F][N][n^3] double or float
  void* Kw;             // same array, K_stage written
  int64_t N;
  int F, p, stage, mode, j, lmin, lmax;
  const int64_t* step;  // device coarse-step counter (read by every launch)
  double w[4][4];
  double b[4];
  double sigma;
  int kmask[4];         // per case: bit i set if w[case][i] != 0 (uniform branches)
  // non-linear wave (positions and the outer boundary): leaf anchors [N][4]
  // (x, y, z in level-L octant units, level), L, periodic flag, source coefficient
  const int32_t* leafxyz;
  int L, periodic;
  double nl_coeff;
  // counter of non-finite values written by the RK update (nullptr: not counted)
  unsigned int* nonfinite;
  // node intervals per octant side (4 or 6) and, for ni = 6, the mesh's table
  // of 8 finer leaves per finer ghost cell
  int ni;
  const int32_t* fine8;
};

// Geometry the non-linear wave's stencils need at one block: its grid origin in
// node units, the grid step, and the domain (side Nu node units; periodic or
// bounded by the outer faces).
struct Geom {
  int X0[3];
  int w, Nu, periodic;
  double c_nl;
};

// Launch shape of the fused kernels: threads per workgroup of the tile kernels
// and of the streaming kernel (256 or 512 each) and the cap on the grid
// (workgroups, rounded to a multiple of 8 XCDs): at or above the tile count one
// workgroup per tile, below it workgroups walk several tiles.
struct LaunchShape {
  int threads = 512;
  int max_wg = 65536;
  int stream_threads = 512;
  // batched launches (lts_batch_*): threads of the tile kernels and grid cap
  int batch_threads = 512;
  int batch_max_wg = 4096;
};

// Tiles of one launch cut into 8 contiguous ranges, one per XCD: XCD x walks
// tiles [b[x], b[x+1]); b[8] is the launch's tile count.
struct XcdRanges {
  int b[9];
};

// One simulation of a batched launch (continuous batching).  It joined at round
// r0 from coarse step n0 and takes part in `rounds` rounds; round r is its
// substep (r - r0) mod 2^(lmax-lmin) of coarse step n0 + (r - r0) div 2^(lmax-lmin).
constexpr int kMaxBatch = 256;
// Default grid cap of batched launches (lts_set_batch_launch changes it).
constexpr int kBatchMaxWg = 4096;
struct BatchSim {
  double* U;                     // [2][F][N][125]
  void* K;                       // [p][F][N][125]
  const int32_t* tiles[2];       // tile records of side 1 and 2 (finest level first)
  const int32_t* slots[2];
  const int32_t* ghosts;         // ghost table [E][2] (leaf, receiver level)
  int64_t N;
  int64_t r0, rounds, n0;
  int64_t gbase;                 // first entry of this simulation in the batch's ghost scratch
  double sigma;
  int32_t lmin, lmax;
  int32_t n_ge[2][LTS_MAX_LEVEL + 1];  // tiles of side t+1 with level >= l
  int32_t ghost_ge[LTS_MAX_LEVEL + 1]; // ghost entries with receiver level >= l
};

// One stage over tiles of side tt (1 or 2) in LDS; coarser ghosts are read from
// the ghost table scr, which launch_ghost_pre has filled for this stage.
hipError_t launch_fused(int tt, int eq, bool kf32, const StageParams& sp, const int32_t* tiles,
                        const int32_t* slots, const double* scr, const XcdRanges& xr, const LaunchShape& ls,
                        hipStream_t s);
// Ghost-table pre-pass of one stage: entries [0, n) (leaf, receiver level) of
// ghosts, prolongated to scr[g][F][GW^3].
hipError_t launch_ghost_pre(int F, bool kf32, const StageParams& sp, const int32_t* ghosts, int64_t n, double* scr,
                            hipStream_t s);
// Weights and stage masks of every stage of a substep (the multi-stage pre-pass).
struct GhostStages {
  double w[4][4][4];   // [stage][time case][i]
  int kmask[4];        // [stage]: the 4 time cases' masks, 4 bits each
  int p;
};
// Ghost-table pre-pass of all p stages of a substep at once, for entries
// [g0, g0 + n) whose coarser sources do not advance during the substep (their
// level is below the lowest active one): entry g's stage-s values to
// scr + s * slot + g * F * GW^3.  Each stage's values are those launch_ghost_pre
// gives for that stage (the same operations, in the same order).
hipError_t launch_ghost_multi(int F, bool kf32, const StageParams& sp, const GhostStages& gs, const int32_t* ghosts,
                              int64_t g0, int64_t n, double* scr, int64_t slot, hipStream_t s);
// One stage of the round *round (device counter) for the simulations
// sims[0..nsims) (device table); `total` bounds the union of their active side-tt
// tiles and sizes the grid (host-computed; any larger value is correct too).
hipError_t launch_fused_batch(int tt, int eq, bool kf32, const StageParams& sp0, const BatchSim* sims, int nsims,
                              const int64_t* round, int64_t total, const double* scr, const int32_t* cum_tab,
                              const LaunchShape& ls, hipStream_t s);
// The round table of a batch: the exclusive prefix sums of the active side-1
// tiles, side-2 tiles and ghost entries of every simulation in round *round, into
// tab[3][kMaxBatch + 1] (read by the round's batched launches).
hipError_t launch_batch_table(const BatchSim* sims, int nsims, int mode, const int64_t* round, int32_t* tab,
                              hipStream_t s);
// The batch's ghost pre-pass of one stage: the union (at most `total` entries)
// of the active ghost entries of every simulation, into scr at each gbase.
hipError_t launch_ghost_pre_batch(int F, bool kf32, const StageParams& sp0, const BatchSim* sims, int nsims,
                                  const int64_t* round, int64_t total, double* scr, const int32_t* cum_tab,
                                  int max_wg, hipStream_t s);
// Streamed whole 4^3 blocks (side-4 tiles, wave equation) over the launch's
// tiles (XCD ranges as for launch_fused), ghosts from the ghost table scr.
hipError_t launch_stream(int eq, bool kf32, const StageParams& sp, const int32_t* tiles, const int32_t* slots,
                         const double* scr, const XcdRanges& xr, const LaunchShape& ls, hipStream_t s);
hipError_t launch_set_i64(int64_t* ptr, int64_t value, hipStream_t s);
// The phase unzip; coarser ghosts come from the ghost table that the launch
// first fills (ghosts[0..nghost) into scr, entry of a leaf: gid[leaf]).
hipError_t launch_unzip(bool kf32, const StageParams& sp, const int32_t* tiles, const int32_t* slots,
                        const int32_t* list, const int64_t* off, int nb, int64_t total, double* out,
                        const int32_t* ghosts, int64_t nghost, double* scr, const int32_t* gid, hipStream_t s);
hipError_t launch_rhs(int eq, bool f32, const int32_t* tiles, const int32_t* list, const int64_t* poff,
                      int64_t ptotal, const int64_t* goff, int64_t gtotal, int nb, const double* padded, void* kout,
                      double sigma, const StageParams& geo, hipStream_t s);
hipError_t launch_zip(bool f32, int ni, const int32_t* tiles, const int32_t* list, const int64_t* goff, int64_t gtotal,
                      int nb, int F, int64_t N, const void* kblock, void* kout, hipStream_t s);
hipError_t launch_rk(bool kf32, const StageParams& sp, const int32_t* tiles, const int32_t* list, int nb,
                     const double* coef, double* out, hipStream_t s);
hipError_t launch_current(const StageParams& sp, const int32_t* tiles, int nblocks, double* out, hipStream_t s);
// Inverse of launch_current: the state of every octant into the U buffer each
// block reads at the coarse step *sp.step.
hipError_t launch_restore(const StageParams& sp, const int32_t* tiles, int nblocks, const double* in, hipStream_t s);
// Race check (debug): NaN into the K slice Ks ([F][N][nn]) over the octants of
// tiles list[0..n) (or tiles 0..n-1 when list is null).
hipError_t launch_poison(const int32_t* tiles, const int32_t* list, int n, void* Ks, bool kf32, int F, int64_t N,
                         int nn, hipStream_t s);
hipError_t launch_set_u32(unsigned int* ptr, unsigned int value, hipStream_t s);
// Remeshing: wavelet indicators of every leaf and of the parents of the families
// fam[0..nfam) (first leaf of 8 siblings); intergrid transfer by records
// rec[N_new][6] = {old leaf, kind (0 interpolate, 1 inject), offset x, y, z, shift}.
hipError_t launch_wavelet(const double* st, int F, int64_t N, const int64_t* fam, int64_t nfam, double* leaf_out,
                          double* fam_out, hipStream_t s);
hipError_t launch_transfer(const double* st_old, int64_t N_old, double* st_new, int64_t N_new, int F,
                           const int32_t* rec, hipStream_t s);
hipError_t launch_increment(int64_t* ctr, hipStream_t s);
hipError_t launch_norm_partials(const double* a, const double* b, int F, int64_t N, int nn, double* sq, double* mx,
                                unsigned long long* bad, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t nbytes, hipStream_t s);

}  // namespace lts
