// Batched fused stage launch (continuous batching): the union of the active
// tiles of several meshes in one launch per tile side.
#include "dev_fused.h"

namespace lts {

// Several independent meshes advanced together (continuous batching): in round r
// every simulation of the table is at its own substep (BatchSim); one launch per
// stage covers the union of the active tiles of side TT of all of them, in table
// order.  Union tile t belongs to the simulation whose cumulative-count range
// holds it; the union is cut into 8 contiguous ranges, one per XCD.  The
// arithmetic of every tile is that of the one-mesh kernel; coarser ghosts come
// from the batch's ghost pre-pass (scr, simulation s at entry gbase_s).
template <int TT, int F, int EQ, bool KF32, int NT, int KS, int ZM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(fused_waves_per_eu<TT, F, KF32, NT, EQ>())))
void k_fused_batch(StageParams sp0, const BatchSim* __restrict__ sims, int nsims, const int64_t* __restrict__ round,
                   const double* __restrict__ scr, const int32_t* __restrict__ cum_tab) {
  __shared__ FusedLds<TT, F, KF32> L;
  __shared__ int cum[kMaxBatch + 1];
  fused_init(L, sp0);
  const int64_t r = *round;
  // cumulative active tile counts of this round (the round table, side TT)
  for (int s = threadIdx.x; s <= nsims; s += NT) cum[s] = cum_tab[(TT - 1) * (kMaxBatch + 1) + s];
  __syncthreads();
  const int total = cum[nsims];
  const int nslot = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7;
  const int sid = blockIdx.x >> 3;
  const int lo = (int)((int64_t)total * xcd / 8), hi = (int)((int64_t)total * (xcd + 1) / 8);
  fused_walk<TT, F, EQ, KF32, NT, KS, 4, ZM>(L, sp0, lo + sid, nslot, hi, [&](int ti) {
    int a = 0, z = nsims - 1;   // the simulation s with cum[s] <= ti < cum[s+1]
    while (a < z) {
      const int mid = (a + z + 1) >> 1;
      if (cum[mid] <= ti) a = mid;
      else z = mid - 1;
    }
    const int s = __builtin_amdgcn_readfirstlane(a);
    const BatchSim& b = sims[s];
    const int64_t rr = r - b.r0;
    const int dl = b.lmax - b.lmin;
    return TileRef{SimView{b.U, b.U, b.K, b.K, b.N, b.lmin, b.lmax, (int)(rr & ((1 << dl) - 1)), b.sigma},
                   (int)((b.n0 + (rr >> dl)) & 3), b.tiles[TT - 1] + 8 * (int64_t)(ti - cum[s]), b.slots[TT - 1],
                   scr + (int64_t)b.gbase * F * 729};
  });
}


namespace {
struct BatchArgs {
  static constexpr bool kNonLinear = false;   // whether the non-linear wave kernels are built for these launches
  static constexpr bool kNodes7 = false;      // whether the 7-node-octant kernels are built for these launches
  static constexpr bool kMaxwell2 = true;     // whether side-2 Maxwell tiles are built for these launches
  const BatchSim* sims;
  int nsims;
  const int64_t* round;
  int64_t total;
  const double* scr;
  const int32_t* cum_tab;
  template <int TT, int F, int EQ, bool KF32, int NT, int KS, int NI, int ZM>
  static hipError_t go(const StageParams& sp, const BatchArgs& a, int max_wg, hipStream_t s) {
    static_assert(NI == 4, "batched launches are built for 5-node octants");
    const int grid = fused_grid((int)std::min<int64_t>(a.total, 1 << 30), max_wg);
    hipLaunchKernelGGL((k_fused_batch<TT, F, EQ, KF32, NT, KS, ZM>), dim3(grid), dim3(NT), 0, s, sp, a.sims, a.nsims,
                       a.round, a.scr, a.cum_tab);
    return hipGetLastError();
  }
};
}  // namespace

hipError_t launch_fused_batch(int tt, int eq, bool kf32, const StageParams& sp0, const BatchSim* sims, int nsims,
                              const int64_t* round, int64_t total, const double* scr, const int32_t* cum_tab,
                              const LaunchShape& ls, hipStream_t s) {
  if (total <= 0 || nsims <= 0) return hipSuccess;
  if (nsims > kMaxBatch) return hipErrorInvalidValue;
  return dispatch_fused(tt, eq, kf32, sp0, BatchArgs{sims, nsims, round, total, scr, cum_tab}, ls, s);
}

// The round table: per simulation the active side-1 tiles, side-2 tiles and ghost
// entries of round *round, as exclusive prefix sums over the table (Hillis-Steele
// in LDS), into tab[3][kMaxBatch + 1].  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_batch_table(const BatchSim* __restrict__ sims, int nsims, int mode,
                                                     const int64_t* __restrict__ round, int32_t* __restrict__ tab) {
  __shared__ int buf[2][3][kMaxBatch + 1];
  const int64_t r = *round;
  const int s = threadIdx.x;
  int c[3] = {0, 0, 0};
  if (s < nsims) {
    const BatchSim& b = sims[s];
    const int64_t rr = r - b.r0;
    if (rr >= 0 && rr < b.rounds) {
      const int j = (int)(rr & ((1 << (b.lmax - b.lmin)) - 1));
      const int lo = (mode == LTS_MODE_GTS || j == 0) ? b.lmin : b.lmax - __builtin_ctz(j);
      c[0] = b.n_ge[0][lo];
      c[1] = b.n_ge[1][lo];
      c[2] = b.ghost_ge[lo];
    }
  }
  for (int k = 0; k < 3; ++k) {
    buf[0][k][s + 1] = s < nsims ? c[k] : 0;
    if (s == 0) buf[0][k][0] = 0;
  }
  __syncthreads();
  int src = 0;
  for (int d = 1; d <= kMaxBatch; d <<= 1) {
    for (int k = 0; k < 3; ++k) {
      const int v = buf[src][k][s + 1] + (s + 1 - d >= 0 ? buf[src][k][s + 1 - d] : 0);
      buf[src ^ 1][k][s + 1] = v;
      if (s == 0) buf[src ^ 1][k][0] = 0;
    }
    __syncthreads();
    src ^= 1;
  }
  for (int k = 0; k < 3; ++k) {
    tab[k * (kMaxBatch + 1) + s + 1] = buf[src][k][s + 1];
    if (s == 0) tab[k * (kMaxBatch + 1)] = 0;
  }
}

hipError_t launch_batch_table(const BatchSim* sims, int nsims, int mode, const int64_t* round, int32_t* tab,
                              hipStream_t s) {
  if (nsims > kMaxBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_batch_table, dim3(1), dim3(kMaxBatch), 0, s, sims, nsims, mode, round, tab);
  return hipGetLastError();
}

}  // namespace lts
