// One-mesh fused stage launch (tile sides 1 and 2): one workgroup per tile of
// tt^3 octants, the padded points its stencils read resident in LDS (Sec. 3.3,
// eqs. fc_1/fc_2, eq. rk_schemes).
#include "dev_fused.h"

namespace lts {

// One mesh: workgroups are dealt to the 8 XCDs round robin; XCD x walks its own
// contiguous (Morton-ordered, cost-balanced) range of tiles.  Coarser ghosts come
// prolongated from the ghost-table pre-pass (scr).  NI: node intervals per octant
// side (4, or 6 for 7-node octants).
template <int TT, int F, int EQ, bool KF32, int NT, int KS, int NI, int ZM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(fused_waves_per_eu<TT, F, KF32, NT, EQ, NI>())))
void k_fused(StageParams sp, const int32_t* __restrict__ tiles, const int32_t* __restrict__ slots,
             const double* __restrict__ scr, XcdRanges xr) {
  __shared__ FusedLds<TT, F, KF32, NI> L;
  fused_init(L, sp);
  const int n4 = (int)(*sp.step & 3);
  const int nslot = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7;
  const int sid = blockIdx.x >> 3;
  const SimView v{sp.U, sp.Uw, sp.K, sp.Kw, sp.N, sp.lmin, sp.lmax, sp.j, sp.sigma};
  int lo, hi;
  xcd_range(xr, xcd, lo, hi);
  fused_walk<TT, F, EQ, KF32, NT, KS, NI, ZM>(L, sp, lo + sid, nslot, hi, [&](int ti) {
    return TileRef{v, n4, tiles + 8 * (int64_t)ti, slots, scr};
  });
}

namespace {
struct OneArgs {
  static constexpr bool kNonLinear = true;   // whether the non-linear wave kernels are built for these launches
  static constexpr bool kNodes7 = true;      // whether the 7-node-octant kernels are built for these launches
  static constexpr bool kMaxwell2 = true;    // whether side-2 Maxwell tiles are built for these launches
  const int32_t* tiles;
  const int32_t* slots;
  const double* scr;
  XcdRanges xr;
  template <int TT, int F, int EQ, bool KF32, int NT, int KS, int NI, int ZM>
  static hipError_t go(const StageParams& sp, const OneArgs& a, int max_wg, hipStream_t s) {
    hipLaunchKernelGGL((k_fused<TT, F, EQ, KF32, NT, KS, NI, ZM>), dim3(fused_grid(a.xr.b[8], max_wg)), dim3(NT), 0, s, sp,
                       a.tiles, a.slots, a.scr, a.xr);
    return hipGetLastError();
  }
};
}  // namespace

hipError_t launch_fused(int tt, int eq, bool kf32, const StageParams& sp, const int32_t* tiles,
                        const int32_t* slots, const double* scr, const XcdRanges& xr, const LaunchShape& ls,
                        hipStream_t s) {
  if (xr.b[8] <= 0) return hipSuccess;
  return dispatch_fused(tt, eq, kf32, sp, OneArgs{tiles, slots, scr, xr}, ls, s);
}

}  // namespace lts
