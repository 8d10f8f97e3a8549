// Ghost-table pre-pass of a stage (one mesh and batched).
#include "dev_common.h"

namespace lts {

// Ghost-table pre-pass, before the fused launches of a stage: entry g (a leaf
// that is a coarser source of receivers one level finer) gets its stage state
// for those receivers (time case, buffer and dt of the receiver level, eqs.
// fc_1/fc_2) prolongated to its 9^3 half-node grid, scr[g][f][z2][y2][x2].  The
// prolongation is separable, x, then y, then z, each a degree-4 Lagrange sum in
// node order; the one-mesh and batched pre-passes share it, so a ghost has one
// value whichever launch forms it.
template <int F>
struct GhostLds {
  double wsh[16];
  double lag[45];
  double Yc[F * 125];
  double T1[F * 225];
  double T2[F * 405];
};

// One ghost-table entry of simulation v: leaf (coarser source), receivers of
// level rlev; the 9^3 grid of each field to out[f][729].
template <bool KF32, int F>
__device__ __forceinline__ void ghost_entry(GhostLds<F>& L, const StageParams& sp, const SimView& v, int n4,
                                            int leaf, int rlev, double* __restrict__ out) {
  using KT = typename std::conditional<KF32, float, double>::type;
  // a receiver tile of the entry's receiver level (only its level matters here)
  int32_t trec[8] = {0, 0, 0, 1, 1, 0, 0, 0};
  trec[TI_LEVEL] = rlev;
  const TileCtx c = tile_ctx(trec, sp.mode, v.j, v.lmin, v.lmax, n4);
  const int fsz = (int)(v.N * 125);
  const double* __restrict__ Uc = v.U + (int64_t)c.par_coarse * F * fsz;
  const KT* __restrict__ Kr = (const KT*)v.K;
  const int kmc = stage_mask(sp, c.case_coarse);
  const double* wc = L.wsh + 4 * c.case_coarse;
  __syncthreads();   // weights loaded; previous entry done with Yc / T1 / T2
  for (int e = threadIdx.x; e < F * 125; e += blockDim.x) {
    const int f = e / 125, n = e - 125 * f;
    const uint32_t off = (uint32_t)(leaf * 125 + n);
    double acc = 0.0;
    #pragma unroll
    for (int i = 0; i < 4; ++i)
      if ((kmc >> i) & 1) acc = fma(wc[i], (double)ld32(Kr + (uint32_t)((i * F + f) * fsz), off), acc);
    L.Yc[e] = ld32(Uc + (uint32_t)(f * fsz), off) + c.dt * acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < F * 225; e += blockDim.x) {
    const int kf = e / 225, r = e - 225 * kf;
    const int x2 = r / 25, yz = r - 25 * x2;
    const double* yc = L.Yc + kf * 125 + 5 * yz;
    double tx;
    if (x2 & 1) {
      tx = 0.0;
      #pragma unroll
      for (int kx = 0; kx < 5; ++kx) tx = fma(L.lag[5 * x2 + kx], yc[kx], tx);
    } else {
      tx = fma(1.0, yc[x2 >> 1], 0.0);
    }
    L.T1[e] = tx;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < F * 405; e += blockDim.x) {
    const int kf = e / 405, r = e - 405 * kf;
    const int x2 = r / 45, r2 = r - 45 * x2;
    const int y2 = r2 / 5, kz = r2 - 5 * y2;
    const double* t1 = L.T1 + kf * 225 + 25 * x2 + 5 * kz;
    double ty;
    if (y2 & 1) {
      ty = 0.0;
      #pragma unroll
      for (int ky = 0; ky < 5; ++ky) ty = fma(L.lag[5 * y2 + ky], t1[ky], ty);
    } else {
      ty = fma(1.0, t1[y2 >> 1], 0.0);
    }
    L.T2[e] = ty;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < F * 729; e += blockDim.x) {
    const int f = e / 729, r = e - 729 * f;
    const int z2 = r / 81, y2 = (r / 9) % 9, x2 = r % 9;
    const double* t2 = L.T2 + f * 405 + 45 * x2 + 5 * y2;
    double v2;
    if (z2 & 1) {
      v2 = 0.0;
      #pragma unroll
      for (int kz = 0; kz < 5; ++kz) v2 = fma(L.lag[5 * z2 + kz], t2[kz], v2);
    } else {
      v2 = fma(1.0, t2[z2 >> 1], 0.0);
    }
    out[e] = v2;
  }
}

template <int F>
__device__ __forceinline__ void ghost_init(GhostLds<F>& L, const StageParams& sp) {
  if (threadIdx.x < 16) L.wsh[threadIdx.x] = stage_weight(sp, threadIdx.x);
  if (threadIdx.x < 45) L.lag[threadIdx.x] = c_lag[threadIdx.x / 5][threadIdx.x % 5];
}

// Ghost-table pre-pass, before the fused launches of a stage: entry g (a leaf
// that is a coarser source of receivers one level finer) gets its stage state
// for those receivers (time case, buffer and dt of the receiver level, eqs.
// fc_1/fc_2) prolongated to its 9^3 half-node grid, scr[g][f][z2][y2][x2].  The
// prolongation is separable, x, then y, then z, each a degree-4 Lagrange sum in
// node order.
template <bool KF32, int F>
__global__ __launch_bounds__(256) void k_ghost_pre(StageParams sp, const int32_t* __restrict__ ghosts,
                                                   double* __restrict__ scr) {
  __shared__ GhostLds<F> L;
  ghost_init(L, sp);
  const int g = blockIdx.x;
  const SimView v{sp.U, sp.Uw, sp.K, sp.Kw, sp.N, sp.lmin, sp.lmax, sp.j, sp.sigma};
  ghost_entry<KF32, F>(L, sp, v, (int)(*sp.step & 3), __builtin_amdgcn_readfirstlane(ghosts[2 * g]),
                       __builtin_amdgcn_readfirstlane(ghosts[2 * g + 1]), scr + (int64_t)g * F * 729);
}

// The same for every simulation of a batch in round *round: the union of their
// active entries (receivers of levels >= each one's lowest active level), in
// table order; simulation s writes its entries at gbase_s.  Each workgroup walks
// several entries (the grid is capped for batches).
template <bool KF32, int F>
__global__ __launch_bounds__(256) void k_ghost_pre_batch(StageParams sp0, const BatchSim* __restrict__ sims,
                                                         int nsims, const int64_t* __restrict__ round,
                                                         double* __restrict__ scr, const int32_t* __restrict__ cum_tab) {
  __shared__ GhostLds<F> L;
  __shared__ int cum[kMaxBatch + 1];
  ghost_init(L, sp0);
  const int64_t r = *round;
  // cumulative active ghost entries of this round (the round table)
  for (int s = threadIdx.x; s <= nsims; s += blockDim.x) cum[s] = cum_tab[2 * (kMaxBatch + 1) + s];
  __syncthreads();
  const int total = cum[nsims];
  for (int q = blockIdx.x; q < total; q += gridDim.x) {
    int a = 0, z = nsims - 1;   // the simulation s with cum[s] <= q < cum[s+1]
    while (a < z) {
      const int mid = (a + z + 1) >> 1;
      if (cum[mid] <= q) a = mid;
      else z = mid - 1;
    }
    const int s = __builtin_amdgcn_readfirstlane(a);
    const BatchSim& b = sims[s];
    const int64_t rr = r - b.r0;
    const int dl = b.lmax - b.lmin;
    const SimView v{b.U, b.U, b.K, b.K, b.N, b.lmin, b.lmax, (int)(rr & ((1 << dl) - 1)), b.sigma};
    const int n4 = (int)((b.n0 + (rr >> dl)) & 3);
    const int g = q - cum[s];
    ghost_entry<KF32, F>(L, sp0, v, n4, __builtin_amdgcn_readfirstlane(b.ghosts[2 * g]),
                         __builtin_amdgcn_readfirstlane(b.ghosts[2 * g + 1]),
                         scr + ((int64_t)b.gbase + g) * F * 729);
  }
}

hipError_t launch_ghost_pre(int F, bool kf32, const StageParams& sp, const int32_t* ghosts, int64_t n, double* scr,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)n);
  if (F == 2) {
    if (kf32) hipLaunchKernelGGL((k_ghost_pre<true, 2>), grid, dim3(256), 0, s, sp, ghosts, scr);
    else hipLaunchKernelGGL((k_ghost_pre<false, 2>), grid, dim3(256), 0, s, sp, ghosts, scr);
  } else if (F == 6) {
    if (kf32) hipLaunchKernelGGL((k_ghost_pre<true, 6>), grid, dim3(256), 0, s, sp, ghosts, scr);
    else hipLaunchKernelGGL((k_ghost_pre<false, 6>), grid, dim3(256), 0, s, sp, ghosts, scr);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ghost_pre_batch(int F, bool kf32, const StageParams& sp0, const BatchSim* sims, int nsims,
                                  const int64_t* round, int64_t total, double* scr, const int32_t* cum_tab,
                                  int max_wg, hipStream_t s) {
  if (total <= 0 || nsims <= 0) return hipSuccess;
  if (nsims > kMaxBatch) return hipErrorInvalidValue;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(total, max_wg)));
  if (F == 2) {
    if (kf32) hipLaunchKernelGGL((k_ghost_pre_batch<true, 2>), grid, dim3(256), 0, s, sp0, sims, nsims, round, scr, cum_tab);
    else hipLaunchKernelGGL((k_ghost_pre_batch<false, 2>), grid, dim3(256), 0, s, sp0, sims, nsims, round, scr, cum_tab);
  } else if (F == 6) {
    if (kf32) hipLaunchKernelGGL((k_ghost_pre_batch<true, 6>), grid, dim3(256), 0, s, sp0, sims, nsims, round, scr, cum_tab);
    else hipLaunchKernelGGL((k_ghost_pre_batch<false, 6>), grid, dim3(256), 0, s, sp0, sims, nsims, round, scr, cum_tab);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lts
