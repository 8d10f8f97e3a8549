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
template <int TT, int F, int EQ, bool KF32, int NT, int KS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(fused_waves_per_eu<TT, F, KF32, NT, EQ>())))
void k_fused_batch(StageParams sp0, const BatchSim* __restrict__ sims, int nsims, const int64_t* __restrict__ round,
                   const double* __restrict__ scr) {
  __shared__ FusedLds<TT, F, KF32> L;
  __shared__ int cum[kMaxBatch + 1];
  fused_init(L, sp0);
  const int64_t r = *round;
  for (int s = threadIdx.x; s < nsims; s += NT) {
    const BatchSim& b = sims[s];
    const int64_t rr = r - b.r0;
    int cnt = 0;
    if (rr >= 0 && rr < b.rounds) {
      const int j = (int)(rr & ((1 << (b.lmax - b.lmin)) - 1));
      const int lo = (sp0.mode == LTS_MODE_GTS || j == 0) ? b.lmin : b.lmax - __builtin_ctz(j);
      cnt = b.n_ge[TT - 1][lo];
    }
    cum[s + 1] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cum[0] = 0;
    for (int s = 0; s < nsims; ++s) cum[s + 1] += cum[s];
  }
  __syncthreads();
  const int total = cum[nsims];
  const int nslot = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7;
  const int sid = blockIdx.x >> 3;
  const int lo = (int)((int64_t)total * xcd / 8), hi = (int)((int64_t)total * (xcd + 1) / 8);
  fused_walk<TT, F, EQ, KF32, NT, KS>(L, sp0, lo + sid, nslot, hi, [&](int ti) {
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
  const BatchSim* sims;
  int nsims;
  const int64_t* round;
  int64_t total;
  const double* scr;
  template <int TT, int F, int EQ, bool KF32, int NT, int KS>
  static hipError_t go(const StageParams& sp, const BatchArgs& a, int max_wg, hipStream_t s) {
    const int grid = fused_grid((int)std::min<int64_t>(a.total, 1 << 30), std::min(max_wg, kBatchMaxWg));
    hipLaunchKernelGGL((k_fused_batch<TT, F, EQ, KF32, NT, KS>), dim3(grid), dim3(NT), 0, s, sp, a.sims, a.nsims,
                       a.round, a.scr);
    return hipGetLastError();
  }
};
}  // namespace

hipError_t launch_fused_batch(int tt, int eq, bool kf32, const StageParams& sp0, const BatchSim* sims, int nsims,
                              const int64_t* round, int64_t total, const double* scr, const LaunchShape& ls,
                              hipStream_t s) {
  if (total <= 0 || nsims <= 0) return hipSuccess;
  if (nsims > kMaxBatch) return hipErrorInvalidValue;
  return dispatch_fused(tt, eq, kf32, sp0, BatchArgs{sims, nsims, round, total, scr}, ls, s);
}

}  // namespace lts
