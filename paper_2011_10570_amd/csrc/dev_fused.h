// The fused stage of LDS-resident tiles: layout, one tile, a workgroup's walk
// over tiles and the dispatch over template arguments.
#pragma once
#include "dev_common.h"

namespace lts {

// ------------------------------------------------------------------ fused stage
// The block RHS reads only along the axes (centred first and second differences
// and Kreiss-Oliger terms, no mixed derivatives), so of the (NI tt+7)^3 padded
// points of a tile (NI node intervals per octant side: 4, or 6 for 7-node
// octants) it uses those with at most one coordinate in the 3-point halo.
// They are kept plane by plane: core plane z = 3 + gz (gz < G) as a P x P square
// at gz P^2 (its four 3 x 3 corners unused), then the six halo planes (z = h for
// h < 3, z = G + h for h >= 3) as G x G squares of the core x and y.
template <int TT, int NI = 4>
struct Cross {
  static constexpr int P = NI * TT + 7;    // padded points per axis
  static constexpr int G = NI * TT + 1;    // grid points per axis
  static constexpr int PP = P * P, GG = G * G;
  static constexpr int HB = G * PP;        // element of the first halo plane
  static constexpr int LS = HB + 6 * GG;   // elements per field
  static constexpr int NA = P * GG;        // core planes, y in the core: whole x rows
  static constexpr int NB = 6 * GG;        // core planes, y in the halo: x in the core
  static constexpr int NC = NA + NB + 6 * GG;
  // used point i (x rows, then y-halo rows, then halo planes) -> padded
  // coordinates and element
  __device__ static __forceinline__ void point(int i, int& qx, int& qy, int& qz, int& li) {
    if (i < NA) {
      qx = i % P;
      const int r = i / P;
      qy = 3 + r % G;
      qz = 3 + r / G;
    } else if (i < NA + NB) {
      const int j = i - NA, r = j / G, h = r % 6;
      qx = 3 + j % G;
      qy = h < 3 ? h : G + h;
      qz = 3 + r / 6;
    } else {
      const int j = i - NA - NB, r = j / G, h = r / G;
      qx = 3 + j % G;
      qy = 3 + r % G;
      qz = h < 3 ? h : G + h;
    }
    li = (qz >= 3 && qz < 3 + G) ? ((qz - 3) * P + qy) * P + qx : HB + ((qz < 3 ? qz : qz - G) * G + qy - 3) * G + qx - 3;
  }
};

// Accessor of the plane-wise padded tile at grid point (gx, gy, gz): c is its
// element in the core planes, hb the element of (gx, gy) in the first halo plane.
template <typename T, int TT, int NI = 4>
struct CrossAt {
  const T* Y;
  int c, hb, gz;
  __device__ __forceinline__ T operator()(int f, int ax, int k) const {
    using X = Cross<TT, NI>;
    int e;
    if (ax == 0) {
      e = c + k;
    } else if (ax == 1) {
      e = c + k * X::P;
    } else {
      const int z = gz + k;
      e = (z >= 0 && z < X::G) ? c + k * X::PP : hb + (z < 0 ? z + 3 : z - X::G + 3) * X::GG;
    }
    return Y[f * X::LS + e];
  }
};

// LDS of one workgroup of the fused stage kernels.
template <int TT, int F, bool KF32, int NI = 4>
struct FusedLds {
  static constexpr int W = TT + 2;
  static constexpr int NS = W * W * W;
  using LT = typename std::conditional<KF32, float, double>::type;
  // side-2 tiles run their stencils once per grid point and stage the results
  // for the zip (octants of a tile share face nodes); side-1 tiles of two
  // fields need no stage (six fields do, for registers: see fused_tile)
  static constexpr bool kStaged = TT > 1 || F > 2;
  static constexpr int G3 = (NI * TT + 1) * (NI * TT + 1) * (NI * TT + 1);
  double R[kStaged ? F * G3 : 1]; // stencil results (staged tiles)
  double wsh[16];                 // stage weights of the 4 time cases
  double ref[2][F];               // FP32 stencils: reference value of each field (this and the next tile)
  LT Y[F * Cross<TT, NI>::LS];    // stage values of the used padded points
  // per-tile tables, read only by the gather: the next tile's are stored once
  // this one's gather is done
  int32_t sl[2 * NS];             // slot records
  uint8_t axl[3][NI * TT + 7];    // per axis: slot position | node offset << 3
};

// A tile and what it needs of its simulation and mesh.
struct TileRef {
  SimView v;
  int n4;                   // coarse-step index mod 4
  const int32_t* tile;      // its 8-int record
  const int32_t* slots;     // slot table of its mesh
  const double* cs;         // ghost table of its mesh
};

// The tile record is uniform: keep it in scalar registers.
__device__ __forceinline__ void load_trec(const int32_t* tile, int32_t t[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) t[k] = __builtin_amdgcn_readfirstlane(tile[k]);
}

// One thread's share of a tile's LDS tables: slot record element, location-table
// element (from the location rule) and, for FP32 stencils, a field's reference
// value.  Loads are issued here and consumed by tables_store, so that their
// latency can be covered by other work.
struct TileTables {
  int32_t slv;
  int32_t axv;
  double refv;
};

template <int TT, int F, bool KF32, int NT, int NI = 4>
__device__ __forceinline__ TileTables tables_issue(const StageParams& sp, const TileRef& r, const int32_t* t) {
  constexpr int P = NI * TT + 7;
  constexpr int NN = (NI + 1) * (NI + 1) * (NI + 1);
  constexpr int NS2 = 2 * (TT + 2) * (TT + 2) * (TT + 2);
  static_assert(NT >= NS2 && NT >= 3 * P, "one table element per thread");
  TileTables tb{0, 0, 0.0};
  if (threadIdx.x < NS2) tb.slv = r.slots[2 * (int64_t)t[TI_SLOT] + threadIdx.x];
  if (threadIdx.x < 3 * P) {
    const int d = threadIdx.x / P, q = threadIdx.x - P * d;
    const int off = t[TI_OFF];
    const int o = (off >> (8 * d)) & 255;
    const int Q = NI * o + q - 3;
    const int cell = cell_of(Q, t[TI_M], NI);
    tb.axv = (cell - o + 1) | ((Q - NI * cell) << 3);
  }
  if (KF32 && threadIdx.x < F) {
    // FP32 stencils work on Y - ref (the Laplacian and KO ignore constants)
    const TileCtx c = tile_ctx<NI>(t, sp.mode, r.v.j, r.v.lmin, r.v.lmax, r.n4);
    const int64_t fsz = r.v.N * NN;
    tb.refv = r.v.U[((int64_t)c.par_same * F + threadIdx.x) * fsz + (int64_t)t[TI_FIRST] * NN];
  }
  return tb;
}

template <int TT, int F, bool KF32, int NI>
__device__ __forceinline__ void tables_store(FusedLds<TT, F, KF32, NI>& L, int b, const TileTables& tb) {
  constexpr int P = NI * TT + 7;
  constexpr int NS2 = 2 * (TT + 2) * (TT + 2) * (TT + 2);
  if (threadIdx.x < NS2) L.sl[threadIdx.x] = tb.slv;
  if (threadIdx.x < 3 * P) L.axl[threadIdx.x / P][threadIdx.x % P] = (uint8_t)tb.axv;
  if (threadIdx.x < F) L.ref[b][threadIdx.x] = KF32 ? tb.refv : 0.0;
}

// One tile of the fused stage (Sec. 3.3, eqs. fc_1/fc_2, eq. rk_schemes).  Its
// slot records and per-axis location tables (slot position and node offset of
// every padded coordinate, from the location rule) are in LDS, its FP32
// reference values in buffer b.
//   (1) every used padded point takes its stage value: a same-level leaf (the
//       tile's own octants included) or 8 finer leaves give Y = U0 + dt sum w_i
//       K_i, read directly (uniform base pointers, 32-bit offsets, UB points per
//       thread loaded before use); a coarser leaf gives its prolongated value
//       from the ghost table;
//   (2) the stencils run once per tile grid point; K_s (and the RK update at
//       the last stage) are written to every DG node of the tile's contiguous
//       octants.  Side-2 tiles stage the results in LDS (octants share face
//       nodes); a side-1 tile's nodes are its grid points, each written
//       directly for two fields.  Six fields (Maxwell) stage them as well: six
//       stencil results held while the last stage's 24 RK operands arrive
//       would exceed the register file.
// With a next tile, its record is loaded at the start and its tables are
// stored, once this tile's gather is done, just before the second barrier
// (reference values into buffer b ^ 1).  Two barriers per tile: after the
// gather, and after the stencils (staged) or the zip (side 1, two fields).
// sp holds the stage (weights, masks).  ZM, the zip mode, is fixed per launch:
// bit 0 = the last stage (RK update), bit 1 = store K_s (all but the last stage
// of GTS), bit 2 = count non-finite updates; as template bits the zip carries no
// run-time branch for them.
template <int ZM>
struct ZipMode {
  static constexpr bool last = (ZM & 1) != 0, storek = (ZM & 2) != 0, check = (ZM & 4) != 0;
};

template <int TT, int F, int EQ, bool KF32, int NT, int KS, int NI = 4, int ZM = 2>
__device__ __forceinline__ void fused_tile(FusedLds<TT, F, KF32, NI>& L, const StageParams& sp, const TileRef& cur,
                                           const int32_t* t, int b, const TileRef& nxt, bool more,
                                           int32_t (&ntrec)[8]) {
  using X = Cross<TT, NI>;
  constexpr int NP = NI + 1, NN = NP * NP * NP;   // nodes per octant side, per octant
  constexpr int GW = 2 * NI + 1, GE = GW * GW * GW;  // ghost-table half-node grid of an entry
  constexpr int P = X::P;
  constexpr int LS = X::LS;
  constexpr int W = TT + 2;
  constexpr int UB = 2;                      // points per thread loaded together
  using LT = typename std::conditional<KF32, float, double>::type;
  using KT = typename std::conditional<KF32, float, double>::type;
  const SimView& v = cur.v;
  const double* __restrict__ cs = cur.cs;
  auto& Y = L.Y;
  const int32_t* sl = L.sl;
  const auto& axl = L.axl;
  auto& wsh = L.wsh;
  const double* ref = L.ref[b];
  if (more) load_trec(nxt.tile, ntrec);
  const int fsz = (int)(v.N * NN);           // elements per field (< 2^31)
  constexpr bool last = ZipMode<ZM>::last;
  // GTS reads no stored stage of the last one (every ghost relation is the
  // same-level case, whose first stage reads U0 only): it is not stored
  constexpr bool storek = ZipMode<ZM>::storek;
  const KT* __restrict__ Kr = (const KT*)v.K;
  KT* __restrict__ Kw = (KT*)v.Kw + (int64_t)sp.stage * F * fsz;
  // KS: stages read by same-level sources (the tableau row's non-zero pattern),
  // a compile-time mask so the hot gather has no branches around its loads
  const TileCtx c = tile_ctx<NI>(t, sp.mode, v.j, v.lmin, v.lmax, cur.n4);
  const int first = t[TI_FIRST];
  const double* __restrict__ Us = v.U + (int64_t)c.par_same * F * fsz;
  const double* __restrict__ Uf = v.U + (int64_t)c.par_fine * F * fsz;
  double* __restrict__ Uw1 = v.Uw + (int64_t)(c.par_same ^ 1) * F * fsz;
  const int kmf = stage_mask(sp, c.case_fine);
  const double* wf = wsh + 4 * c.case_fine;

  // (1) stage values of the used padded points
  for (int p0 = threadIdx.x; p0 < X::NC; p0 += UB * NT) {
    int li[UB], kind[UB], leaf[UB], kbv[UB], nuv[UB][3], below[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int pi = p0 + u * NT;
      kind[u] = -1;
      li[u] = 0;
      leaf[u] = 0;
      kbv[u] = 0;
      below[u] = 0;
      nuv[u][0] = nuv[u][1] = nuv[u][2] = 0;
      if (pi >= X::NC) continue;
      int qx, qy, qz;
      X::point(pi, qx, qy, qz, li[u]);
      const int ax = axl[0][qx], ay = axl[1][qy], az = axl[2][qz];
      const int si = (ax & 7) + W * ((ay & 7) + W * (az & 7));
      nuv[u][0] = ax >> 3;
      nuv[u][1] = ay >> 3;
      nuv[u][2] = az >> 3;
      // a finer slot at slot position 0 along an axis lies below the block there
      if constexpr (NI == 6) below[u] = ((ax & 7) == 0 ? 1 : 0) | ((ay & 7) == 0 ? 2 : 0) | ((az & 7) == 0 ? 4 : 0);
      kbv[u] = sl[2 * si + 1];
      kind[u] = kbv[u] & 15;
      leaf[u] = sl[2 * si];
    }
    // one straight-line batch of loads for every lane: a same-level point reads
    // U0 and the K's of its node, a coarser one its ghost-table value (and,
    // like every other lane, K's at a valid dummy element); loads under
    // per-kind branches would wait for each other's registers
    double uu[UB][F], kk[UB][F][4];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const bool same = kind[u] == SRC_SAME, coarse = kind[u] == SRC_COARSE;
      const uint32_t off = same ? (uint32_t)(leaf[u] * NN + nuv[u][0] + NP * nuv[u][1] + NP * NP * nuv[u][2]) : 0u;
      // ghost-table entry (in the slot's first int), octant beta of the leaf
      const int beta = (kbv[u] >> 4) & 7;
      const int x2 = NI * (beta & 1) + nuv[u][0], y2 = NI * ((beta >> 1) & 1) + nuv[u][1],
                z2 = NI * ((beta >> 2) & 1) + nuv[u][2];
      const double* pa = coarse ? cs + ((int64_t)leaf[u] * F * GE + (z2 * GW + y2) * GW + x2) : Us + off;
      const int fst = coarse ? GE : fsz;
#pragma unroll
      for (int f = 0; f < F; ++f) {
        uu[u][f] = pa[(int64_t)f * fst];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if ((KS >> i) & 1) kk[u][f][i] = (double)ld32(Kr + (uint32_t)((i * F + f) * fsz), off);
      }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      if (kind[u] == SRC_FINE) {
        uint32_t off;
        if constexpr (NI == 4) {
          const int cx = min(nuv[u][0] >> 1, 1), cy = min(nuv[u][1] >> 1, 1), cz = min(nuv[u][2] >> 1, 1);
          off = (uint32_t)((leaf[u] + cx + 2 * cy + 4 * cz) * 125 + 2 * (nuv[u][0] - 2 * cx) +
                           10 * (nuv[u][1] - 2 * cy) + 50 * (nuv[u][2] - 2 * cz));
        } else {
          // 2:1 balance: the slot names a row of the fine table
          const int cx = fine_child6(nuv[u][0], below[u] & 1), cy = fine_child6(nuv[u][1], (below[u] >> 1) & 1),
                    cz = fine_child6(nuv[u][2], (below[u] >> 2) & 1);
          const int lf = sp.fine8[8 * leaf[u] + cx + 2 * cy + 4 * cz];
          off = (uint32_t)(lf * NN + (2 * nuv[u][0] - NI * cx) + NP * (2 * nuv[u][1] - NI * cy) +
                           NP * NP * (2 * nuv[u][2] - NI * cz));
        }
#pragma unroll
        for (int f = 0; f < F; ++f) {
          double acc = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if ((kmf >> i) & 1) acc = fma(wf[i], (double)ld32(Kr + (uint32_t)((i * F + f) * fsz), off), acc);
          Y[f * LS + li[u]] = (LT)(ld32(Uf + (uint32_t)(f * fsz), off) + c.dt * acc - ref[f]);
        }
      } else if (kind[u] == SRC_SAME) {
#pragma unroll
        for (int f = 0; f < F; ++f) {
          double acc = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if ((KS >> i) & 1) acc = fma(wsh[i], kk[u][f][i], acc);
          Y[f * LS + li[u]] = (LT)(uu[u][f] + c.dt * acc - ref[f]);
        }
      } else if (kind[u] == SRC_COARSE) {
#pragma unroll
        for (int f = 0; f < F; ++f) Y[f * LS + li[u]] = (LT)(uu[u][f] - ref[f]);
      } else if (EQ == LTS_EQ_NLWAVE && kind[u] == SRC_NONE) {   // only bounded meshes have them
        // beyond the outer faces: never read by the bounded-domain stencils
#pragma unroll
        for (int f = 0; f < F; ++f) Y[f * LS + li[u]] = (LT)0;
      }
    }
  }
  TileTables tb{0, 0, 0.0};
  if (more) tb = tables_issue<TT, F, KF32, NT, NI>(sp, nxt, ntrec);
  __syncthreads();
  // from here on the gather is done with this tile's tables: the next tile's
  // replace them before the second barrier (their loads have had the stencils'
  // time to arrive)
  constexpr int NT3 = TT * TT * TT * NN;     // DG nodes of the tile
  constexpr int G = X::G;
  Geom geo{};
  if constexpr (EQ == LTS_EQ_NLWAVE) geo = geom_of(sp, first, c.lev);
  // the stencils at grid point (gx, gy, gz) of the tile
  auto stencil = [&](int gx, int gy, int gz, double (&k)[F]) {
    const int ce = (gz * P + gy + 3) * P + gx + 3;
    if constexpr (EQ == LTS_EQ_NLWAVE) {
      const int Xp[3] = {geo.X0[0] + geo.w * gx, geo.X0[1] + geo.w * gy, geo.X0[2] + geo.w * gz};
      rhs_nl_at(CrossAt<LT, TT, NI>{Y, ce, X::HB + gy * G + gx, gz}, c.h, v.sigma, geo, Xp, k);
    } else {
      // one axis at a time: fewer live registers (same operations, same order)
      rhs_at<LT, EQ, F, true>(CrossAt<LT, TT, NI>{Y, ce, X::HB + gy * G + gx, gz}, (LT)c.h, (LT)v.sigma, ref, k);
    }
  };
  double bs = sp.b[0];   // b_s without a dynamic index into the kernel arguments
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i == sp.stage) bs = sp.b[i];
  // the last stage's RK operands of node element off
  auto rk_operands = [&](uint32_t off, double (&zu)[F], double (&zk)[F][3]) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      zu[f] = ld32(Us + (uint32_t)(f * fsz), off);
#pragma unroll
      for (int i = 0; i < 3; ++i)
        zk[f][i] = (i < sp.stage) ? (double)ld32(Kr + (uint32_t)((i * F + f) * fsz), off) : 0.0;
    }
  };
  // K_s of node element off (and at the last stage the RK update)
  auto emit = [&](uint32_t off, const double (&k)[F], const double (&zu)[F], const double (&zk)[F][3]) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      double kv = k[f];
      if constexpr (KF32) {
        const float kf = (float)kv;
        if constexpr (storek) st32(Kw + (uint32_t)(f * fsz), off, kf);
        kv = (double)kf;
      } else {
        if constexpr (storek) st32(Kw + (uint32_t)(f * fsz), off, kv);
      }
      if constexpr (last) {
        // compute_step_partial: U_new = U0 + dt (b_0 K_0 + ... + b_s K_s),
        // s = p - 1, accumulated in stage order, into the other buffer
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          if (i < sp.stage) acc = fma(sp.b[i], zk[f][i], acc);
        acc = fma(bs, kv, acc);
        const double un = zu[f] + c.dt * acc;
        st32(Uw1 + (uint32_t)(f * fsz), off, un);
        if constexpr (ZipMode<ZM>::check) {
          if (!isfinite(un)) atomicAdd(sp.nonfinite, 1u);
        }
      }
    }
  };
  if constexpr (FusedLds<TT, F, KF32, NI>::kStaged) {
    // (2a) stencils once per tile grid point (NI tt+1)^3, results staged in LDS
    constexpr int G3 = G * G * G;
    auto& R = L.R;
    for (int gi = threadIdx.x; gi < G3; gi += NT) {
      double k[F];
      stencil(gi % G, (gi / G) % G, gi / (G * G), k);
#pragma unroll
      for (int f = 0; f < F; ++f) R[f * G3 + gi] = k[f];
    }
    if (more) tables_store(L, b ^ 1, tb);
    __syncthreads();
    // (2b) zip: node e of the tile is element first*NN + e of every field array
    // and takes its grid point's results; its RK operands are issued first
    constexpr int KZ = (NT3 + NT - 1) / NT;
#pragma unroll
    for (int u = 0; u < KZ; ++u) {
      const int e = threadIdx.x + u * NT;
      if (e >= NT3) continue;
      const uint32_t off = (uint32_t)(first * NN + e);
      double zu[F], zk[F][3];
      if constexpr (last) rk_operands(off, zu, zk);
      const int o = e / NN, node = e - NN * o;
      const int gi = ((NI * ((o >> 2) & 1) + node / (NP * NP)) * G + (NI * ((o >> 1) & 1) + (node / NP) % NP)) * G +
                     (NI * (o & 1) + node % NP);
      double k[F];
#pragma unroll
      for (int f = 0; f < F; ++f) k[f] = R[f * G3 + gi];
      emit(off, k, zu, zk);
    }
    // the next tile's gather writes Y only, its stencils R after its first barrier
  } else {
    // (2) side-1 tiles of two fields: the octant's nodes are the tile's grid
    // points; each runs its stencils and writes its results directly
    static_assert(TT == 1 && F == 2, "unstaged stencils are for side-1 tiles of two fields");
    for (int e = threadIdx.x; e < NT3; e += NT) {
      const uint32_t off = (uint32_t)(first * NN + e);
      double k[F];
      stencil(e % NP, (e / NP) % NP, e / (NP * NP), k);
      // RK operands after the stencils: held across them they would cost
      // registers beyond the budget
      double zu[F], zk[F][3];
      if constexpr (last) rk_operands(off, zu, zk);
      emit(off, k, zu, zk);
    }
    if (more) tables_store(L, b ^ 1, tb);
    // the next tile's gather overwrites Y and reads the tables stored above
    __syncthreads();
  }
}

template <int TT, int F, bool KF32, int NI>
__device__ __forceinline__ void fused_init(FusedLds<TT, F, KF32, NI>& L, const StageParams& sp) {
  if (threadIdx.x < 16) L.wsh[threadIdx.x] = stage_weight(sp, threadIdx.x);
}

// Waves per SIMD that the LDS of one workgroup allows: the register budget the
// compiler is asked to keep so that registers do not cost occupancy.  Capped
// where a tighter budget spills: 6 (80 registers) for FP64 side-2 tiles, 8 (64)
// with FP32 stencils, 5 for side-1 tiles, 4 for the non-linear wave; left free
// for 6 fields.
template <int TT, int F, bool KF32, int NT, int EQ = LTS_EQ_WAVE, int NI = 4>
constexpr int fused_waves_per_eu() {
  const int wg = (160 * 1024) / (int)sizeof(FusedLds<TT, F, KF32, NI>);
  const int w = wg * (NT / 64) / 4;
  // the non-linear wave's boundary-aware stencils need more registers
  const int cap = EQ == LTS_EQ_NLWAVE ? 4 : (TT == 1 ? 5 : (KF32 ? 8 : 6));
  return (F > 2 || w < 1) ? 1 : (w > cap ? cap : w);
}

// A workgroup's walk over tiles lo, lo + step, ... < hi; ref_of(i) gives tile i.
// The first tile's tables are loaded here, every later one's by the tile before.
template <int TT, int F, int EQ, bool KF32, int NT, int KS, int NI, int ZM, typename RefOf>
__device__ __forceinline__ void fused_walk(FusedLds<TT, F, KF32, NI>& L, const StageParams& sp, int lo, int step,
                                           int hi, const RefOf& ref_of) {
  if (lo >= hi) return;
  TileRef cur = ref_of(lo);
  int32_t trec[8];
  load_trec(cur.tile, trec);
  tables_store(L, 0, tables_issue<TT, F, KF32, NT, NI>(sp, cur, trec));
  __syncthreads();
  int b = 0;
  for (int ti = lo;; ti += step) {
    const bool more = ti + step < hi;
    TileRef nxt = more ? ref_of(ti + step) : cur;
    int32_t ntrec[8];
    fused_tile<TT, F, EQ, KF32, NT, KS, NI, ZM>(L, sp, cur, trec, b, nxt, more, ntrec);
    if (!more) break;
    cur = nxt;
#pragma unroll
    for (int k = 0; k < 8; ++k) trec[k] = ntrec[k];
    b ^= 1;
  }
}


// The same-level stage mask, the zip mode and the workgroup size are template
// arguments: the masks that occur for the built tableaus are RK4: none, {0},
// {1} for the first three stages and {2} for the last, SSP-RK3: none, {0} and
// {0,1} for the last; only the last stages (masks {2} and {0,1}) take the RK
// update, and only they have zip modes other than "store K".  A::go<...>
// launches the kernel of one combination.
template <int TT, int F, int EQ, bool KF32, int NT, int KS, int NI, typename A>
hipError_t dispatch_zm(int zm, const StageParams& sp, const A& a, int max_wg, hipStream_t s) {
  switch (zm) {
    case 1: return A::template go<TT, F, EQ, KF32, NT, KS, NI, 1>(sp, a, max_wg, s);
    case 3: return A::template go<TT, F, EQ, KF32, NT, KS, NI, 3>(sp, a, max_wg, s);
    case 5: return A::template go<TT, F, EQ, KF32, NT, KS, NI, 5>(sp, a, max_wg, s);
    case 7: return A::template go<TT, F, EQ, KF32, NT, KS, NI, 7>(sp, a, max_wg, s);
    default: return hipErrorInvalidValue;
  }
}

template <int TT, int F, int EQ, bool KF32, int NT, int NI, typename A>
hipError_t dispatch_ks(const StageParams& sp, const A& a, int max_wg, hipStream_t s) {
  const bool last = sp.stage == sp.p - 1;
  const int zm = last ? (1 | (sp.mode == LTS_MODE_GTS ? 0 : 2) | (sp.nonfinite ? 4 : 0)) : 2;
  const int ks = sp.kmask[0];
  if (last != (ks == 3 || ks == 4)) return hipErrorInvalidValue;
  switch (ks) {
    case 0: return A::template go<TT, F, EQ, KF32, NT, 0, NI, 2>(sp, a, max_wg, s);
    case 1: return A::template go<TT, F, EQ, KF32, NT, 1, NI, 2>(sp, a, max_wg, s);
    case 2: return A::template go<TT, F, EQ, KF32, NT, 2, NI, 2>(sp, a, max_wg, s);
    case 3: return dispatch_zm<TT, F, EQ, KF32, NT, 3, NI>(zm, sp, a, max_wg, s);
    case 4: return dispatch_zm<TT, F, EQ, KF32, NT, 4, NI>(zm, sp, a, max_wg, s);
    default: return hipErrorInvalidValue;
  }
}

template <int TT, int F, int EQ, bool KF32, typename A, int NI = 4>
hipError_t dispatch_nt(const StageParams& sp, const A& a, const LaunchShape& ls, hipStream_t s) {
  switch (ls.threads) {
    case 256: return dispatch_ks<TT, F, EQ, KF32, 256, NI>(sp, a, ls.max_wg, s);
    case 512: return dispatch_ks<TT, F, EQ, KF32, 512, NI>(sp, a, ls.max_wg, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename A>
hipError_t dispatch_fused(int tt, int eq, bool kf32, const StageParams& sp, const A& a, const LaunchShape& ls,
                          hipStream_t s) {
  // side-1 tiles run 256-thread workgroups whatever the launch shape's thread
  // count (more workgroups in flight per CU): 7-node wave 7 %, 5-node wave 28 %,
  // Maxwell 10-20 % faster than 512
  if (sp.ni == 6) {   // 7-node octants: the wave equation on side-1 tiles, launches that allow it
    if constexpr (A::kNodes7) {
      if (eq == LTS_EQ_WAVE && tt == 1)
        return kf32 ? dispatch_ks<1, 2, LTS_EQ_WAVE, true, 256, 6>(sp, a, ls.max_wg, s)
                    : dispatch_ks<1, 2, LTS_EQ_WAVE, false, 256, 6>(sp, a, ls.max_wg, s);
    }
    return hipErrorInvalidValue;
  }
  if (sp.ni != 4) return hipErrorInvalidValue;
  if (eq == LTS_EQ_NLWAVE) {   // FP64, tile sides 1 and 2, launches that allow it
    if constexpr (A::kNonLinear) {
      if (kf32) return hipErrorInvalidValue;
      if (tt == 1) return dispatch_ks<1, 2, LTS_EQ_NLWAVE, false, 256, 4>(sp, a, ls.max_wg, s);
      if (tt == 2) return dispatch_nt<2, 2, LTS_EQ_NLWAVE, false>(sp, a, ls, s);
    }
    return hipErrorInvalidValue;
  }
  if (eq == LTS_EQ_WAVE) {
    if (tt == 1) return kf32 ? dispatch_ks<1, 2, LTS_EQ_WAVE, true, 256, 4>(sp, a, ls.max_wg, s)
                             : dispatch_ks<1, 2, LTS_EQ_WAVE, false, 256, 4>(sp, a, ls.max_wg, s);
    if (tt == 2) return kf32 ? dispatch_nt<2, 2, LTS_EQ_WAVE, true>(sp, a, ls, s)
                             : dispatch_nt<2, 2, LTS_EQ_WAVE, false>(sp, a, ls, s);
    return hipErrorInvalidValue;
  }
  if (tt == 2) {   // one workgroup per CU (153 KB of LDS for six FP64 fields), one-mesh launches
    if constexpr (A::kMaxwell2)
      return kf32 ? dispatch_nt<2, 6, LTS_EQ_MAXWELL, true, A>(sp, a, ls, s)
                  : dispatch_nt<2, 6, LTS_EQ_MAXWELL, false, A>(sp, a, ls, s);
    return hipErrorInvalidValue;
  }
  if (tt != 1) return hipErrorInvalidValue;
  return kf32 ? dispatch_ks<1, 6, LTS_EQ_MAXWELL, true, 256, 4>(sp, a, ls.max_wg, s)
              : dispatch_ks<1, 6, LTS_EQ_MAXWELL, false, 256, 4>(sp, a, ls.max_wg, s);
}

}  // namespace lts
