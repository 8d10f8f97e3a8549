// Streamed whole 4^3-octant blocks (side-4 tiles, wave equation).
#include "dev_common.h"

namespace lts {

// ------------------------------------------------------------------ streamed blocks
// Whole 4^3-octant blocks (side-4 tiles) are streamed along z: the padded block
// (23^3 points per field) never sits in LDS at once.  A ring of 8 padded planes
// holds the 7 planes one output plane of the 17^3 block grid needs plus the plane
// being loaded, so the loads of padded plane z+7 are in flight while the stencils
// of output plane z run.  Of each plane only the points a stencil reads are
// gathered: 1.26 points per DG node, against 2.19 for side-2 tiles.


template <int F, bool KF32>
struct StreamLds {
  static constexpr int P = 23, PL = P * P, G = 17, GL = G * G, RING = 8, NS = 216;
  using LT = typename std::conditional<KF32, float, double>::type;
  LT Y[F * RING * PL];       // ring of padded planes: [f][slot][y][x]
  double R[2][F * GL];       // stencil results of an output plane (double buffered)
  int32_t sl[2 * NS];        // slot table
  uint8_t axl[2][P];         // x / y: slot position | node offset << 3
  double wsh[16];
  double ref[F];
};

// Accessor of the ring: x, y inside a plane, z across the ring slots zb[0..6].
template <typename T>
struct RingAt {
  const T* Y;
  int fs, cxy;
  const int* zb;
  __device__ __forceinline__ T operator()(int f, int ax, int k) const {
    if (ax == 2) return Y[f * fs + zb[3 + k] + cxy];
    return Y[f * fs + zb[3] + cxy + k * (ax == 0 ? 1 : 23)];
  }
};

// Raw loads of one padded plane (per thread: KP points), issued one step before
// they are combined into stage values, so that their latency spans a whole step:
// U (or the prolongated ghost) and the same-level stages K_i, i in the mask KS.
// Points of finer sources load theirs when they are combined (they are few).
template <int KP, int F, int KS>
struct PlaneLoads {
  static constexpr int NK = (KS & 1) + ((KS >> 1) & 1) + ((KS >> 2) & 1);
  int kind[KP];
  double uu[KP][F];
  double kk[KP][F][NK > 0 ? NK : 1];
};

// The k-th set bit of the mask KS (compile-time).
template <int KS>
constexpr int ks_bit(int k) {
  for (int i = 0; i < 3; ++i)
    if ((KS >> i) & 1) {
      if (k == 0) return i;
      --k;
    }
  return 0;
}

// Per-block constants of the streaming kernel.
template <bool KF32>
struct StreamCtx {
  using KT = typename std::conditional<KF32, float, double>::type;
  const double* Us;      // U buffer of the block's step (same-level sources, U0)
  const double* Uf;      // U buffer of finer sources
  double* Uw1;           // the other U buffer (RK update)
  const KT* Kr;          // stages
  KT* Kw;                // K_s
  const double* cs;      // ghost table (prolongated coarser ghosts)
  const double* wf;      // weights of finer sources (LDS)
  double dt, h, sigma;
  int fsz, first, kmf;
};

// loads of padded plane pz into Q.  Every lane loads (lanes that need no value
// read a valid dummy element), so the loads form one straight-line batch.  Only
// points that a stencil reads are loaded: no corner of a plane of the block's z
// range, and only the block's x-y core in the planes above and below it.
template <int F, bool KF32, int NT, int KS, int KP>
__device__ __forceinline__ void stream_issue(const StreamLds<F, KF32>& L, const StreamCtx<KF32>& x, int pz,
                                             PlaneLoads<KP, F, KS>& Q) {
  constexpr int P = StreamLds<F, KF32>::P, PL = StreamLds<F, KF32>::PL;
  constexpr int NK = PlaneLoads<KP, F, KS>::NK;
  if (pz >= P) return;
  const int Qz = pz - 3;
  const int cz = cell_of(Qz, 4);
  const int nuz = Qz - 4 * cz, szz = cz + 1;
  const bool zcore = pz >= 3 && pz < P - 3;
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    const int p = threadIdx.x + u * NT;
    const int pp = p < PL ? p : 0;
    const int qy = pp / P, qx = pp - P * qy;
    const bool xc = qx >= 3 && qx < P - 3, yc = qy >= 3 && qy < P - 3;
    const bool on = p < PL && (zcore ? (xc || yc) : (xc && yc));
    const int ax = L.axl[0][qx], ay = L.axl[1][qy];
    const int si = (ax & 7) + 6 * ((ay & 7) + 6 * szz);
    const int kb = L.sl[2 * si + 1];
    const int leaf = L.sl[2 * si];
    const int nux = ax >> 3, nuy = ay >> 3;
    const int kind = on ? (kb & 15) : -1;
    const bool same = kind == SRC_SAME, coarse = kind == SRC_COARSE;
    const uint32_t off = same ? (uint32_t)(leaf * 125 + nux + 5 * nuy + 25 * nuz) : 0u;
    // coarser: the prolongated ghost in scr (leaf = the ghost-table entry)
    const int beta = (kb >> 4) & 7;
    const int x2 = 4 * (beta & 1) + nux, y2 = 4 * ((beta >> 1) & 1) + nuy, z2 = 4 * ((beta >> 2) & 1) + nuz;
    const double* pa = coarse ? x.cs + ((int64_t)leaf * F * 729 + (z2 * 9 + y2) * 9 + x2) : x.Us + off;
    const int fst = coarse ? 729 : x.fsz;
    Q.kind[u] = kind;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      Q.uu[u][f] = pa[(int64_t)f * fst];
#pragma unroll
      for (int k = 0; k < NK; ++k)
        Q.kk[u][f][k] = (double)ld32(x.Kr + (uint32_t)((ks_bit<KS>(k) * F + f) * x.fsz), off);
    }
  }
}

// stage values of plane pz (loads in Q) into its ring slot: Y = U + dt sum w K
// (same-level: case (0,1) weights; finer: case (0,1/2), loaded here), coarser
// ghosts as they are
template <int F, bool KF32, int NT, int KS, int KP>
__device__ __forceinline__ void stream_store(StreamLds<F, KF32>& L, const StreamCtx<KF32>& x, int pz,
                                             const PlaneLoads<KP, F, KS>& Q) {
  using LS = StreamLds<F, KF32>;
  constexpr int P = LS::P, PL = LS::PL;
  constexpr int NK = PlaneLoads<KP, F, KS>::NK;
  using LT = typename LS::LT;
  if (pz >= P) return;
  LT* Yp = L.Y + (pz & 7) * PL;
  const int Qz = pz - 3;
  const int cz = cell_of(Qz, 4);
  const int nuz = Qz - 4 * cz, szz = cz + 1;
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    const int kind = Q.kind[u];
    const int p = threadIdx.x + u * NT;
    if (kind == SRC_FINE) {
      // the coincident node of child c of the finer source
      const int qy = p / P, qx = p - P * qy;
      const int ax = L.axl[0][qx], ay = L.axl[1][qy];
      const int si = (ax & 7) + 6 * ((ay & 7) + 6 * szz);
      const int leaf = L.sl[2 * si];
      const int nux = ax >> 3, nuy = ay >> 3;
      const int cx = min(nux >> 1, 1), cy = min(nuy >> 1, 1), czz = min(nuz >> 1, 1);
      const uint32_t off = (uint32_t)((leaf + cx + 2 * cy + 4 * czz) * 125 + 2 * (nux - 2 * cx) +
                                      10 * (nuy - 2 * cy) + 50 * (nuz - 2 * czz));
#pragma unroll
      for (int f = 0; f < F; ++f) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          if ((x.kmf >> i) & 1) acc = fma(x.wf[i], (double)ld32(x.Kr + (uint32_t)((i * F + f) * x.fsz), off), acc);
        Yp[f * 8 * PL + p] = (LT)(ld32(x.Uf + (uint32_t)(f * x.fsz), off) + x.dt * acc - L.ref[f]);
      }
    } else if (kind == SRC_SAME) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NK; ++k) acc = fma(L.wsh[ks_bit<KS>(k)], Q.kk[u][f][k], acc);
        Yp[f * 8 * PL + p] = (LT)(Q.uu[u][f] + x.dt * acc - L.ref[f]);
      }
    } else if (kind == SRC_COARSE) {
#pragma unroll
      for (int f = 0; f < F; ++f) Yp[f * 8 * PL + p] = (LT)(Q.uu[u][f] - L.ref[f]);
    }
  }
}

// stencils of output plane gz from the ring into R
template <int F, int EQ, bool KF32, int NT>
__device__ __forceinline__ void stream_stencil(const StreamLds<F, KF32>& L, const StreamCtx<KF32>& x, int gz,
                                               double* R) {
  using LS = StreamLds<F, KF32>;
  constexpr int P = LS::P, PL = LS::PL, G = LS::G, GL = LS::GL;
  using LT = typename LS::LT;
  if (gz < 0 || gz >= G) return;
  int zb[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) zb[k] = ((gz + k) & 7) * PL;
  for (int gp = threadIdx.x; gp < GL; gp += NT) {
    const int gy = gp / G, gx = gp - G * gy;
    double kv[F];
    rhs_at<LT, EQ, F, true>(RingAt<LT>{L.Y, 8 * PL, (gy + 3) * P + (gx + 3), zb}, (LT)x.h, (LT)x.sigma, L.ref, kv);
#pragma unroll
    for (int f = 0; f < F; ++f) R[f * GL + gp] = kv[f];
  }
}

// DG node e (0 .. 400 nl) of output plane gz: its element offset and its point
// of the block grid plane.  The plane's node layers: octant layer oz1, node layer
// c1, and where octant layers meet (gz = 4, 8, 12) also layer oz1-1, node 4.
__device__ __forceinline__ void plane_node(int first, int gz, int e, uint32_t& off, int& gp) {
  const int oz1 = min(gz >> 2, 3), c1 = gz - 4 * oz1;
  const int layer = e / 400, r = e - 400 * layer;
  const int qo = r / 25, n = r - 25 * qo;
  const int ox = qo & 3, oy = qo >> 2;
  const int oz = layer ? oz1 - 1 : oz1, cz = layer ? 4 : c1;
  off = (uint32_t)((first + (int)morton3(ox, oy, oz)) * 125 + cz * 25 + n);
  const int b = n / 5, a = n - 5 * b;
  gp = (4 * oy + b) * 17 + (4 * ox + a);
}

__device__ __forceinline__ int plane_nodes(int gz) { return ((gz & 3) == 0 && gz > 0 && gz < 16) ? 800 : 400; }

// zip (+ RK update at the last stage, its operands loaded here) of output
// plane gz from R
template <int F, bool KF32, int NT, bool LAST>
__device__ __forceinline__ void stream_zip(const StageParams& sp, const StreamCtx<KF32>& x, int gz, const double* R) {
  constexpr int GL = StreamLds<F, KF32>::GL;
  if (gz < 0 || gz >= 17) return;
  const int nn = plane_nodes(gz);
  double bs = sp.b[0];   // b_s without a dynamic index into the kernel arguments
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i == sp.stage) bs = sp.b[i];
#pragma unroll 1
  for (int e = threadIdx.x; e < nn; e += NT) {
    uint32_t off;
    int gp;
    plane_node(x.first, gz, e, off, gp);
    double u0[F], kp[F][3];
    if constexpr (LAST) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        u0[f] = ld32(x.Us + (uint32_t)(f * x.fsz), off);
#pragma unroll
        for (int i = 0; i < 3; ++i)
          kp[f][i] = i < sp.stage ? (double)ld32(x.Kr + (uint32_t)((i * F + f) * x.fsz), off) : 0.0;
      }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) {
      double kv = R[f * GL + gp];
      // GTS: the last stage's K is read by no ghost relation and not stored
      const bool storek = !(LAST && sp.mode == LTS_MODE_GTS);
      if constexpr (KF32) {
        const float kf = (float)kv;
        if (storek) st32(x.Kw + (uint32_t)(f * x.fsz), off, kf);
        kv = (double)kf;
      } else {
        if (storek) st32(x.Kw + (uint32_t)(f * x.fsz), off, kv);
      }
      if constexpr (LAST) {
        // U0 + dt (b_0 K_0 + ... + b_s K_s), s = p - 1, accumulated in stage order
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          if (i < sp.stage) acc = fma(sp.b[i], kp[f][i], acc);
        acc = fma(bs, kv, acc);
        const double un = u0[f] + x.dt * acc;
        st32(x.Uw1 + (uint32_t)(f * x.fsz), off, un);
        if (sp.nonfinite && !isfinite(un)) atomicAdd(sp.nonfinite, 1u);
      }
    }
  }
}

// One streamed block, a software pipeline over the 23 padded planes.  Step `it`
// (0..24): issue the loads of padded plane it+1 (stage values of same-level /
// finer sources, prolongated coarser ghosts from scr) and, at the last stage,
// of the RK operands of output plane it-7; zip (and RK-update) output plane it-8
// from the LDS result of the previous step; run the stencils of output plane
// it-7 from the ring; combine the loads of plane it (issued in the previous
// step) into its ring slot; barrier.
template <int F, int EQ, bool KF32, int NT, int KS, bool LAST>
__device__ __forceinline__ void stream_tile(StreamLds<F, KF32>& L, const StageParams& sp, const SimView& v, int n4,
                                            const int32_t* __restrict__ tile, const int32_t* __restrict__ slots,
                                            const double* __restrict__ cs) {
  using LS = StreamLds<F, KF32>;
  constexpr int P = LS::P, PL = LS::PL, NS = LS::NS;
  constexpr int KP = (PL + NT - 1) / NT;          // padded points per thread and plane
  using KT = typename std::conditional<KF32, float, double>::type;
  int32_t trec[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) trec[e] = __builtin_amdgcn_readfirstlane(tile[e]);
  const int32_t* t = trec;
  const TileCtx c = tile_ctx(t, sp.mode, v.j, v.lmin, v.lmax, n4);
  StreamCtx<KF32> x;
  x.fsz = (int)(v.N * 125);
  x.first = t[TI_FIRST];
  x.Us = v.U + (int64_t)c.par_same * F * x.fsz;
  x.Uf = v.U + (int64_t)c.par_fine * F * x.fsz;
  x.Uw1 = v.Uw + (int64_t)(c.par_same ^ 1) * F * x.fsz;
  x.Kr = (const KT*)v.K;
  x.Kw = (KT*)v.Kw + (int64_t)sp.stage * F * x.fsz;
  x.cs = cs;
  x.kmf = stage_mask(sp, c.case_fine);
  x.wf = L.wsh + 4 * c.case_fine;
  x.dt = c.dt;
  x.h = c.h;
  x.sigma = v.sigma;
  __syncthreads();  // previous block done with LDS
  for (int e = threadIdx.x; e < 2 * NS; e += NT) L.sl[e] = slots[2 * (int64_t)t[TI_SLOT] + e];
  if (threadIdx.x < 2 * P) {
    const int q = threadIdx.x % P;
    const int Q = q - 3;
    const int cell = cell_of(Q, 4);
    L.axl[threadIdx.x / P][q] = (uint8_t)((cell + 1) | ((Q - 4 * cell) << 3));
  }
  if (threadIdx.x < F) L.ref[threadIdx.x] = KF32 ? x.Us[threadIdx.x * x.fsz + x.first * 125] : 0.0;
  __syncthreads();
  // Two sets of plane loads alternate: step `it` issues plane it+1 into one set
  // while the other, issued in step it-1, is consumed.
  PlaneLoads<KP, F, KS> A, B;
  stream_issue<F, KF32, NT, KS>(L, x, 0, A);
  for (int it = 0; it <= P + 1; it += 2) {
    stream_issue<F, KF32, NT, KS>(L, x, it + 1, B);
    stream_stencil<F, EQ, KF32, NT>(L, x, it - 7, L.R[it & 1]);
    stream_zip<F, KF32, NT, LAST>(sp, x, it - 8, L.R[(it + 1) & 1]);
    stream_store<F, KF32, NT, KS>(L, x, it, A);
    __syncthreads();
    if (it + 1 > P + 1) break;
    stream_issue<F, KF32, NT, KS>(L, x, it + 2, A);
    stream_stencil<F, EQ, KF32, NT>(L, x, it - 6, L.R[(it + 1) & 1]);
    stream_zip<F, KF32, NT, LAST>(sp, x, it - 7, L.R[it & 1]);
    stream_store<F, KF32, NT, KS>(L, x, it + 1, B);
    __syncthreads();
  }
}

template <int F, int EQ, bool KF32, int NT, int KS, bool LAST>
__global__ __launch_bounds__(NT) void k_stream(StageParams sp, const int32_t* __restrict__ tiles,
                                               const int32_t* __restrict__ slots, const double* __restrict__ scr,
                                               XcdRanges xr) {
  __shared__ StreamLds<F, KF32> L;
  if (threadIdx.x < 16) L.wsh[threadIdx.x] = stage_weight(sp, threadIdx.x);
  const int n4 = (int)(*sp.step & 3);
  const int nslot = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7;
  const int sid = blockIdx.x >> 3;
  const SimView v{sp.U, sp.Uw, sp.K, sp.Kw, sp.N, sp.lmin, sp.lmax, sp.j, sp.sigma};
  int lo, hi;
  xcd_range(xr, xcd, lo, hi);
  for (int ti = lo + sid; ti < hi; ti += nslot)
    stream_tile<F, EQ, KF32, NT, KS, LAST>(L, sp, v, n4, tiles + 8 * (int64_t)ti, slots, scr);
}

// Streamed side-4 tiles (wave equation), after the ghost pre-pass.
template <bool KF32, int NT, int KS>
static hipError_t go_stream(const StageParams& sp, const int32_t* tiles, const int32_t* slots, const double* scr,
                            const XcdRanges& xr, int max_wg, hipStream_t s) {
  const dim3 grid(fused_grid(xr.b[8], max_wg));
  if (sp.stage == sp.p - 1)
    hipLaunchKernelGGL((k_stream<2, LTS_EQ_WAVE, KF32, NT, KS, true>), grid, dim3(NT), 0, s, sp, tiles, slots, scr, xr);
  else
    hipLaunchKernelGGL((k_stream<2, LTS_EQ_WAVE, KF32, NT, KS, false>), grid, dim3(NT), 0, s, sp, tiles, slots, scr,
                       xr);
  return hipGetLastError();
}

template <bool KF32, int NT>
static hipError_t stream_ks(const StageParams& sp, const int32_t* tiles, const int32_t* slots, const double* scr,
                            const XcdRanges& xr, int max_wg, hipStream_t s) {
  switch (sp.kmask[0]) {
    case 0: return go_stream<KF32, NT, 0>(sp, tiles, slots, scr, xr, max_wg, s);
    case 1: return go_stream<KF32, NT, 1>(sp, tiles, slots, scr, xr, max_wg, s);
    case 2: return go_stream<KF32, NT, 2>(sp, tiles, slots, scr, xr, max_wg, s);
    case 3: return go_stream<KF32, NT, 3>(sp, tiles, slots, scr, xr, max_wg, s);
    case 4: return go_stream<KF32, NT, 4>(sp, tiles, slots, scr, xr, max_wg, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stream(int eq, bool kf32, const StageParams& sp, const int32_t* tiles, const int32_t* slots,
                         const double* scr, const XcdRanges& xr, const LaunchShape& ls, hipStream_t s) {
  if (xr.b[8] <= 0) return hipSuccess;
  if (eq != LTS_EQ_WAVE) return hipErrorInvalidValue;   // 6 fields do not fit the plane ring
  switch (ls.stream_threads) {
    case 256: return kf32 ? stream_ks<true, 256>(sp, tiles, slots, scr, xr, ls.max_wg, s)
                          : stream_ks<false, 256>(sp, tiles, slots, scr, xr, ls.max_wg, s);
    case 512: return kf32 ? stream_ks<true, 512>(sp, tiles, slots, scr, xr, ls.max_wg, s)
                          : stream_ks<false, 512>(sp, tiles, slots, scr, xr, ls.max_wg, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lts
