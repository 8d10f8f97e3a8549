// Ghost-table pre-pass of a stage (one mesh and batched).
#include "dev_common.h"

namespace lts {

// Ghost-table pre-pass, before the fused launches of a stage: entry g (a leaf
// that is a coarser source of receivers one level finer) gets its stage state
// for those receivers (time case, buffer and dt of the receiver level, eqs.
// fc_1/fc_2) prolongated to its GW^3 half-node grid (GW = 2 NI + 1: 9 for
// 5-node octants, 13 for 7-node octants), scr[g][f][z2][y2][x2].  The
// prolongation is separable, x, then y, then z, each a degree-NI Lagrange sum in
// node order; the one-mesh and batched pre-passes share it, so a ghost has one
// value whichever launch forms it.
template <int F, int NI = 4>
struct GhostLds {
  static constexpr int NP = NI + 1, GW = 2 * NI + 1;
  double wsh[16];
  double lag[GW * NP];
  double Yc[F * NP * NP * NP];
  double T1[F * GW * NP * NP];
  double T2[F * GW * GW * NP];
};

// e / d for 0 <= e < 2^20 and d >= 1, from a float estimate (off by at most one
// at these sizes) and one correction each way; r = 1 / d.
__device__ __forceinline__ int small_div(int e, int d, float r) {
  int q = (int)((float)e * r);
  q += (q + 1) * d <= e ? 1 : 0;
  q -= q * d > e ? 1 : 0;
  return q;
}

// The 4 time cases' stage masks of sp, 4 bits each.
__device__ __forceinline__ int packed_masks(const StageParams& sp) {
  return (sp.kmask[0] & 15) | (sp.kmask[1] & 15) << 4 | (sp.kmask[2] & 15) << 8 | (sp.kmask[3] & 15) << 12;
}

// One ghost-table entry of simulation v: leaf (coarser source), rec = receiver
// level (bits 0-4) and the half-node box that the receivers read (4 bits per
// bound from bit 5: x lo, x hi, y lo, y hi, z lo, z hi); the box of the GW^3
// grid of each field to out[f][GW^3].  Points outside the box are not written
// (no tile reads them); inside it every value is the full prolongation's.  The
// stage: weights wsh[case][i] (LDS) and masks km (packed_masks).
template <bool KF32, int F, int NI = 4>
__device__ __forceinline__ void ghost_entry(GhostLds<F, NI>& L, const StageParams& sp, const SimView& v, int n4,
                                            int leaf, int rec, double* __restrict__ out, const double* wsh, int km) {
  using KT = typename std::conditional<KF32, float, double>::type;
  constexpr int NP = NI + 1, NN = NP * NP * NP, GW = 2 * NI + 1;
  const int rlev = rec & 31;
  const int xlo = (rec >> 5) & 15, ylo = (rec >> 13) & 15, zlo = (rec >> 21) & 15;
  const int bx = ((rec >> 9) & 15) - xlo + 1, by = ((rec >> 17) & 15) - ylo + 1, bz = ((rec >> 25) & 15) - zlo + 1;
  // a receiver tile of the entry's receiver level (only its level matters here)
  int32_t trec[8] = {0, 0, 0, 1, 1, 0, 0, 0};
  trec[TI_LEVEL] = rlev;
  const TileCtx c = tile_ctx<NI>(trec, sp.mode, v.j, v.lmin, v.lmax, n4);
  const int fsz = (int)(v.N * NN);
  const double* __restrict__ Uc = v.U + (int64_t)c.par_coarse * F * fsz;
  const KT* __restrict__ Kr = (const KT*)v.K;
  const int kmc = (km >> (4 * c.case_coarse)) & 15;
  const double* wc = wsh + 4 * c.case_coarse;
  __syncthreads();   // weights loaded; previous entry done with Yc / T1 / T2
  for (int e = threadIdx.x; e < F * NN; e += blockDim.x) {
    const int f = e / NN, n = e - NN * f;
    const uint32_t off = (uint32_t)(leaf * NN + n);
    double acc = 0.0;
    #pragma unroll
    for (int i = 0; i < 4; ++i)
      if ((kmc >> i) & 1) acc = fma(wc[i], (double)ld32(Kr + (uint32_t)((i * F + f) * fsz), off), acc);
    L.Yc[e] = ld32(Uc + (uint32_t)(f * fsz), off) + c.dt * acc;
  }
  __syncthreads();
  // x: T1[f][x2][z][y], x2 in the box
  const int n1 = bx * NP * NP;
  const float r1 = 1.0f / (float)n1;
  for (int e = threadIdx.x; e < F * n1; e += blockDim.x) {
    const int kf = small_div(e, n1, r1), r = e - n1 * kf;
    const int x2 = xlo + r / (NP * NP), yz = r % (NP * NP);
    const double* yc = L.Yc + kf * NN + NP * yz;
    double tx;
    if (x2 & 1) {
      tx = 0.0;
      #pragma unroll
      for (int kx = 0; kx < NP; ++kx) tx = fma(L.lag[NP * x2 + kx], yc[kx], tx);
    } else {
      tx = fma(1.0, yc[x2 >> 1], 0.0);
    }
    L.T1[kf * (GW * NP * NP) + (NP * NP) * x2 + yz] = tx;
  }
  __syncthreads();
  // y: T2[f][x2][y2][z], (x2, y2) in the box
  const int n2 = by * NP, n2f = bx * n2;
  const float r2 = 1.0f / (float)n2, r2f = 1.0f / (float)n2f;
  for (int e = threadIdx.x; e < F * n2f; e += blockDim.x) {
    const int kf = small_div(e, n2f, r2f), ra = e - n2f * kf;
    const int xi = small_div(ra, n2, r2), rb = ra - n2 * xi;
    const int x2 = xlo + xi, y2 = ylo + rb / NP, kz = rb % NP;
    const double* t1 = L.T1 + kf * (GW * NP * NP) + (NP * NP) * x2 + NP * kz;
    double ty;
    if (y2 & 1) {
      ty = 0.0;
      #pragma unroll
      for (int ky = 0; ky < NP; ++ky) ty = fma(L.lag[NP * y2 + ky], t1[ky], ty);
    } else {
      ty = fma(1.0, t1[y2 >> 1], 0.0);
    }
    L.T2[kf * (GW * GW * NP) + (GW * NP) * x2 + NP * y2 + kz] = ty;
  }
  __syncthreads();
  // z: out[f][z2][y2][x2], the box
  constexpr int GE = GW * GW * GW;
  const int nxy = bx * by, n3 = nxy * bz;
  const float rx = 1.0f / (float)bx, rxy = 1.0f / (float)nxy, r3 = 1.0f / (float)n3;
  for (int e = threadIdx.x; e < F * n3; e += blockDim.x) {
    const int f = small_div(e, n3, r3), ra = e - n3 * f;
    const int zi = small_div(ra, nxy, rxy), rb = ra - nxy * zi;
    const int yi = small_div(rb, bx, rx), xi = rb - bx * yi;
    const int x2 = xlo + xi, y2 = ylo + yi, z2 = zlo + zi;
    const double* t2 = L.T2 + f * (GW * GW * NP) + (GW * NP) * x2 + NP * y2;
    double v2;
    if (z2 & 1) {
      v2 = 0.0;
      #pragma unroll
      for (int kz = 0; kz < NP; ++kz) v2 = fma(L.lag[NP * z2 + kz], t2[kz], v2);
    } else {
      v2 = fma(1.0, t2[z2 >> 1], 0.0);
    }
    out[f * GE + (z2 * GW + y2) * GW + x2] = v2;
  }
}

template <int F, int NI = 4>
__device__ __forceinline__ void ghost_init(GhostLds<F, NI>& L, const StageParams& sp) {
  constexpr int NP = NI + 1, GW = 2 * NI + 1;
  if (threadIdx.x < 16) L.wsh[threadIdx.x] = stage_weight(sp, threadIdx.x);
  for (int i = threadIdx.x; i < GW * NP; i += blockDim.x)
    L.lag[i] = NI == 4 ? c_lag[i / NP][i % NP] : c_lag7[i / NP][i % NP];
}

// One workgroup per ghost-table entry (see ghost_entry).
template <bool KF32, int F, int NI>
__global__ __launch_bounds__(NI == 6 ? 512 : 256) void k_ghost_pre(StageParams sp, const int32_t* __restrict__ ghosts,
                                                   double* __restrict__ scr) {
  constexpr int GW = 2 * NI + 1;
  __shared__ GhostLds<F, NI> L;
  ghost_init(L, sp);
  const int g = blockIdx.x;
  const SimView v{sp.U, sp.Uw, sp.K, sp.Kw, sp.N, sp.lmin, sp.lmax, sp.j, sp.sigma};
  ghost_entry<KF32, F, NI>(L, sp, v, (int)(*sp.step & 3), __builtin_amdgcn_readfirstlane(ghosts[2 * g]),
                           __builtin_amdgcn_readfirstlane(ghosts[2 * g + 1]),
                           scr + (int64_t)g * F * (GW * GW * GW), L.wsh, packed_masks(sp));
}

// All p stages of a substep for entry g0 + blockIdx.x, whose coarser source is
// idle during the substep: the stage values differ only in their weights, and
// the source's U and K's, read from HBM for the first stage, come from L2 for
// the others.
template <bool KF32, int F, int NI>
__global__ __launch_bounds__(NI == 6 ? 512 : 256) void k_ghost_multi(StageParams sp, GhostStages gs,
                                                     const int32_t* __restrict__ ghosts, int64_t g0,
                                                     double* __restrict__ scr, int64_t slot) {
  constexpr int GW = 2 * NI + 1;
  __shared__ GhostLds<F, NI> L;
  __shared__ double wall[4][16];
  ghost_init(L, sp);
  if (threadIdx.x < 64) wall[threadIdx.x >> 4][threadIdx.x & 15] = gs.w[threadIdx.x >> 4][(threadIdx.x >> 2) & 3][threadIdx.x & 3];
  const int64_t g = g0 + blockIdx.x;
  const SimView v{sp.U, sp.Uw, sp.K, sp.Kw, sp.N, sp.lmin, sp.lmax, sp.j, sp.sigma};
  const int n4 = (int)(*sp.step & 3);
  const int leaf = __builtin_amdgcn_readfirstlane(ghosts[2 * g]);
  const int rec = __builtin_amdgcn_readfirstlane(ghosts[2 * g + 1]);
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if (s < gs.p)
      ghost_entry<KF32, F, NI>(L, sp, v, n4, leaf, rec, scr + s * slot + g * F * (GW * GW * GW), wall[s],
                               gs.kmask[s]);
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
                         scr + ((int64_t)b.gbase + g) * F * 729, L.wsh, packed_masks(sp0));
  }
}

hipError_t launch_ghost_pre(int F, bool kf32, const StageParams& sp, const int32_t* ghosts, int64_t n, double* scr,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)n);
  if (sp.ni == 6) {   // 7-node octants: the wave equation
    if (F != 2) return hipErrorInvalidValue;
    // 512 threads for the 13^3-point entries (measured 4.5 % faster on the
    // 7-node step than 256)
    if (kf32) hipLaunchKernelGGL((k_ghost_pre<true, 2, 6>), grid, dim3(512), 0, s, sp, ghosts, scr);
    else hipLaunchKernelGGL((k_ghost_pre<false, 2, 6>), grid, dim3(512), 0, s, sp, ghosts, scr);
    return hipGetLastError();
  }
  if (sp.ni != 4) return hipErrorInvalidValue;
  if (F == 2) {
    if (kf32) hipLaunchKernelGGL((k_ghost_pre<true, 2, 4>), grid, dim3(256), 0, s, sp, ghosts, scr);
    else hipLaunchKernelGGL((k_ghost_pre<false, 2, 4>), grid, dim3(256), 0, s, sp, ghosts, scr);
  } else if (F == 6) {
    if (kf32) hipLaunchKernelGGL((k_ghost_pre<true, 6, 4>), grid, dim3(256), 0, s, sp, ghosts, scr);
    else hipLaunchKernelGGL((k_ghost_pre<false, 6, 4>), grid, dim3(256), 0, s, sp, ghosts, scr);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ghost_multi(int F, bool kf32, const StageParams& sp, const GhostStages& gs, const int32_t* ghosts,
                              int64_t g0, int64_t n, double* scr, int64_t slot, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (gs.p < 1 || gs.p > 4) return hipErrorInvalidValue;
  const dim3 grid((unsigned)n);
  if (sp.ni == 6) {
    if (F != 2) return hipErrorInvalidValue;
    if (kf32) hipLaunchKernelGGL((k_ghost_multi<true, 2, 6>), grid, dim3(512), 0, s, sp, gs, ghosts, g0, scr, slot);
    else hipLaunchKernelGGL((k_ghost_multi<false, 2, 6>), grid, dim3(512), 0, s, sp, gs, ghosts, g0, scr, slot);
    return hipGetLastError();
  }
  if (sp.ni != 4) return hipErrorInvalidValue;
  if (F == 2) {
    if (kf32) hipLaunchKernelGGL((k_ghost_multi<true, 2, 4>), grid, dim3(256), 0, s, sp, gs, ghosts, g0, scr, slot);
    else hipLaunchKernelGGL((k_ghost_multi<false, 2, 4>), grid, dim3(256), 0, s, sp, gs, ghosts, g0, scr, slot);
  } else if (F == 6) {
    if (kf32) hipLaunchKernelGGL((k_ghost_multi<true, 6, 4>), grid, dim3(256), 0, s, sp, gs, ghosts, g0, scr, slot);
    else hipLaunchKernelGGL((k_ghost_multi<false, 6, 4>), grid, dim3(256), 0, s, sp, gs, ghosts, g0, scr, slot);
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
