// HIP kernels of the LTS hot path for gfx950 (MI355X).
//
// One RK stage (Sec. 3.3 + Alg. 1/2): unzip (ghost-padded block state with
// f->c injection, degree-4 c->f interpolation and the LTS stage conversion of
// eqs. fc_1/fc_2), block RHS (sixth-order FD + Kreiss-Oliger), zip back to the
// octant-local nodes and, after the last stage, the RK update (eq. rk_schemes).
//
// Two forms:
//   * fused: k_ghost_pre prolongates the coarser ghosts of the stage into a
//               table; k_fused then runs one workgroup per tile of tt^3 octants
//               (tt = 1, 2) with the padded points its stencils read resident
//               in LDS, and k_stream streams whole 4^3-octant blocks along z.
//               Tiles are dealt to the 8 XCDs in contiguous, Morton-ordered
//               ranges, so neighbour tiles run on one XCD and share its L2.
//   * k_unzip / k_rhs / k_zip / k_rk: the same steps as separate launches over
//               whole blocks through HBM (phase-by-phase path and parity checks).
// Stencils are not dense contractions: no MFMA; the work is bound by HBM traffic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lts_impl.h"
#include "lts_kernels.h"

namespace lts {

// Degree-4 Lagrange weights L_k(xi) = prod_{m != k} (xi - m)/(k - m) on nodes
// 0..4 at xi = x2/2 (x2 = 0..8).  Exact binary fractions (denominator 128).
__constant__ double c_lag[9][5] = {
    {1, 0, 0, 0, 0},
    {35.0 / 128, 140.0 / 128, -70.0 / 128, 28.0 / 128, -5.0 / 128},
    {0, 1, 0, 0, 0},
    {-5.0 / 128, 60.0 / 128, 90.0 / 128, -20.0 / 128, 3.0 / 128},
    {0, 0, 1, 0, 0},
    {3.0 / 128, -20.0 / 128, 90.0 / 128, 60.0 / 128, -5.0 / 128},
    {0, 0, 0, 1, 0},
    {-5.0 / 128, 28.0 / 128, -70.0 / 128, 140.0 / 128, 35.0 / 128},
    {0, 0, 0, 0, 1}};

// sixth-order central second derivative, first derivative, KO sixth difference
#define D2C0 (-49.0 / 18.0)
#define D2C1 (3.0 / 2.0)
#define D2C2 (-3.0 / 20.0)
#define D2C3 (1.0 / 90.0)
#define D1C1 (3.0 / 4.0)
#define D1C2 (-3.0 / 20.0)
#define D1C3 (1.0 / 60.0)

// ------------------------------------------------------------------ schedule
// Step index (mod 4) of a level-lev block at substep j of coarse step n:
// LTS s = n 2^(lev-lmin) + (j >> (lmax-lev)), GTS s = n 2^(lmax-lmin) + j.
__device__ __forceinline__ int step_mod4(int n4, int lev, int mode, int j, int lmin, int lmax) {
  if (mode == LTS_MODE_GTS) return ((n4 << (lmax - lmin)) + j) & 3;
  return ((n4 << (lev - lmin)) + (j >> (lmax - lev))) & 3;
}

// Kernel-argument arrays indexed without a dynamic index (a per-lane or computed
// index into a by-value argument makes the compiler copy the whole argument to
// scratch memory): stage weight e = 4 case + i, and the stage mask of a case.
__device__ __forceinline__ double stage_weight(const StageParams& sp, int e) {
  double w = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (e == k) w = sp.w[k >> 2][k & 3];
  return w;
}

__device__ __forceinline__ int stage_mask(const StageParams& sp, int cs) {
  // the 4 masks packed 4 bits each and shifted out: a select chain over the
  // array can be turned back into an indexed copy in scratch
  const int packed = (sp.kmask[0] & 15) | (sp.kmask[1] & 15) << 4 | (sp.kmask[2] & 15) << 8 | (sp.kmask[3] & 15) << 12;
  return (packed >> (4 * cs)) & 15;
}

struct TileCtx {
  int lev, m, tt, ox, oy, oz;
  int par_same, par_fine, par_coarse;   // U buffer of the source records
  int case_fine, case_coarse;           // time case of finer / coarser sources
  double dt, h;
};

__device__ __forceinline__ TileCtx tile_ctx(const int32_t* t, int mode, int j, int lmin, int lmax, int n4) {
  TileCtx c;
  c.lev = t[TI_LEVEL];
  c.m = t[TI_M];
  c.tt = t[TI_TT];
  const int off = t[TI_OFF];
  c.ox = off & 255;
  c.oy = (off >> 8) & 255;
  c.oz = (off >> 16) & 255;
  const int s = step_mod4(n4, c.lev, mode, j, lmin, lmax);
  c.par_same = s & 1;
  if (mode == LTS_MODE_GTS) {
    c.par_fine = c.par_coarse = s & 1;
    c.case_fine = c.case_coarse = 0;
    c.dt = ldexp(1.0, -lmax - 3);
  } else {
    // a finer neighbour steps twice per receiver step: its step index is 2 s;
    // a coarser one once per two: its index is floor(s / 2) (Sec. 3.6.3).
    c.par_fine = 0;
    c.par_coarse = (s >> 1) & 1;
    c.case_fine = 1;                                   // (delta, rho) = (0, 1/2)
    c.case_coarse = 2 + ((j >> (lmax - c.lev)) & 1);  // (0, 2) or (1, 2)
    c.dt = ldexp(1.0, -c.lev - 3);
  }
  c.h = ldexp(1.0, -c.lev - 1);
  return c;
}

__device__ __forceinline__ TileCtx tile_ctx(const int32_t* t, const StageParams& sp, int n4) {
  return tile_ctx(t, sp.mode, sp.j, sp.lmin, sp.lmax, n4);
}

// ------------------------------------------------------------------ gather
// Element `idx` of a field array given by a uniform base pointer, addressed with a
// 32-bit byte offset (lets the compiler use scalar-base + 32-bit-offset loads;
// the host limits arrays to < 2^32 bytes per field).
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t idx) {
  return *(const T*)((const char*)base + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, uint32_t idx, T v) {
  *(T*)((char*)base + idx * (uint32_t)sizeof(T)) = v;
}

template <bool KF32>
__device__ __forceinline__ double kload(const void* K, int64_t idx) {
  if constexpr (KF32) return (double)((const float*)K)[idx];
  else return ((const double*)K)[idx];
}

// Y = U0 + dt sum_i w_i K_i at one DG node (field stride fs = N*125); only the
// stages with a non-zero weight (bit mask km, uniform per case) are read.
template <bool KF32>
__device__ __forceinline__ double yval(const StageParams& sp, const double* w, int km, int par, int64_t idx,
                                       double dt) {
  const int64_t fs = sp.N * 125;
  const int64_t ps = fs * sp.F;
  double acc = 0.0;
  #pragma unroll
  for (int i = 0; i < 4; ++i) {
    if ((km >> i) & 1) acc = fma(w[i], kload<KF32>(sp.K, i * ps + idx), acc);
  }
  return sp.U[par * ps + idx] + dt * acc;
}

// The same value split in a load step and a combine step, so that a thread can
// keep the loads of several nodes in flight before using any of them.
template <bool KF32, int F>
struct YLoad {
  double u[F];
  double k[F][4];
};

template <bool KF32, int F>
__device__ __forceinline__ void yload(const StageParams& sp, int km, int par, int64_t base, YLoad<KF32, F>& r) {
  const int64_t fs = sp.N * 125;
  const int64_t ps = fs * sp.F;
  #pragma unroll
  for (int f = 0; f < F; ++f) {
    r.u[f] = sp.U[par * ps + f * fs + base];
    #pragma unroll
    for (int i = 0; i < 4; ++i) r.k[f][i] = ((km >> i) & 1) ? kload<KF32>(sp.K, i * ps + f * fs + base) : 0.0;
  }
}

template <bool KF32, int F>
__device__ __forceinline__ double ycombine(const YLoad<KF32, F>& r, int f, const double* w, int km, double dt) {
  double acc = 0.0;
  #pragma unroll
  for (int i = 0; i < 4; ++i)
    if ((km >> i) & 1) acc = fma(w[i], r.k[f][i], acc);
  return r.u[f] + dt * acc;
}

// Value of every field at padded tile point (qx, qy, qz).  slots: the tile's
// slot table; wsh: stage-s weights per case [4][4].
template <bool KF32, int F>
__device__ __forceinline__ void point_values(const StageParams& sp, const TileCtx& c, const int32_t* slots,
                                             const double* wsh, int qx, int qy, int qz, double out[F]) {
  const Loc L = locate(qx, qy, qz, c.ox, c.oy, c.oz, c.tt, c.m);
  const int leaf = slots[2 * L.slot];
  const int kb = slots[2 * L.slot + 1];
  const int kind = kb & 15;
  const int64_t fs = sp.N * 125;
  if (kind != SRC_COARSE) {
    int node, lf, par, km;
    const double* w;
    if (kind == SRC_FINE) {
      const int cx = min(L.nu[0] >> 1, 1), cy = min(L.nu[1] >> 1, 1), cz = min(L.nu[2] >> 1, 1);
      lf = leaf + cx + 2 * cy + 4 * cz;
      node = 2 * (L.nu[0] - 2 * cx) + 5 * 2 * (L.nu[1] - 2 * cy) + 25 * 2 * (L.nu[2] - 2 * cz);
      par = c.par_fine;
      w = wsh + 4 * c.case_fine;
      km = stage_mask(sp, c.case_fine);
    } else {
      lf = leaf;
      node = L.nu[0] + 5 * L.nu[1] + 25 * L.nu[2];
      par = c.par_same;
      w = wsh;
      km = sp.kmask[0];
    }
    const int64_t base = (int64_t)lf * 125 + node;
    #pragma unroll
    for (int f = 0; f < F; ++f) out[f] = yval<KF32>(sp, w, km, par, f * fs + base, c.dt);
    return;
  }
  // coarser source: tensor degree-4 Lagrange interpolation of its Y values
  const int beta = (kb >> 4) & 7;
  int x2[3];
  for (int d = 0; d < 3; ++d) x2[d] = 4 * ((beta >> d) & 1) + L.nu[d];
  const double* w = wsh + 4 * c.case_coarse;
  const int km = stage_mask(sp, c.case_coarse);
  const int par = c.par_coarse;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    if (x2[d] & 1) { lo[d] = 0; hi[d] = 4; }
    else { lo[d] = hi[d] = x2[d] >> 1; }
  }
  #pragma unroll
  for (int f = 0; f < F; ++f) out[f] = 0.0;
  for (int kz = lo[2]; kz <= hi[2]; ++kz) {
    double ty[F];
    #pragma unroll
    for (int f = 0; f < F; ++f) ty[f] = 0.0;
    for (int ky = lo[1]; ky <= hi[1]; ++ky) {
      double tx[F];
      #pragma unroll
      for (int f = 0; f < F; ++f) tx[f] = 0.0;
      for (int kx = lo[0]; kx <= hi[0]; ++kx) {
        const double wx = c_lag[x2[0]][kx];
        const int64_t base = (int64_t)leaf * 125 + kx + 5 * ky + 25 * kz;
        #pragma unroll
        for (int f = 0; f < F; ++f) tx[f] = fma(wx, yval<KF32>(sp, w, km, par, f * fs + base, c.dt), tx[f]);
      }
      const double wy = c_lag[x2[1]][ky];
      #pragma unroll
      for (int f = 0; f < F; ++f) ty[f] = fma(wy, tx[f], ty[f]);
    }
    const double wz = c_lag[x2[2]][kz];
    #pragma unroll
    for (int f = 0; f < F; ++f) out[f] = fma(wz, ty[f], out[f]);
  }
}

// ------------------------------------------------------------------ stencils
// One grid point of the block RHS.  at(f, axis, k) is field f at offset k (-3..3)
// from the point along axis (0 = x, 1 = y, 2 = z); k = 0 is the point itself.
// Returns du/dt of each field.  Every caller goes through this one body, so the
// floating-point operations and their order do not depend on the data layout.
template <typename T, int EQ, int F, bool SEQ = false, typename At>
__device__ __forceinline__ void rhs_at(const At& at, T h, T sigma, const double ref[F], double out[F]) {
  const T kos = sigma / (T(64) * h);
  if constexpr (EQ == LTS_EQ_WAVE) {
    T lap = T(0), ku = T(0), kv = T(0);
    auto axis = [&](int ax) {
      const T u0 = at(0, ax, 0), v0 = at(1, ax, 0);
      const T up1 = at(0, ax, 1), um1 = at(0, ax, -1), up2 = at(0, ax, 2), um2 = at(0, ax, -2), up3 = at(0, ax, 3),
              um3 = at(0, ax, -3);
      const T vp1 = at(1, ax, 1), vm1 = at(1, ax, -1), vp2 = at(1, ax, 2), vm2 = at(1, ax, -2), vp3 = at(1, ax, 3),
              vm3 = at(1, ax, -3);
      lap += T(D2C3) * (um3 + up3) + T(D2C2) * (um2 + up2) + T(D2C1) * (um1 + up1) + T(D2C0) * u0;
      ku += (um3 + up3) - T(6) * (um2 + up2) + T(15) * (um1 + up1) - T(20) * u0;
      kv += (vm3 + vp3) - T(6) * (vm2 + vp2) + T(15) * (vm1 + vp1) - T(20) * v0;
    };
    // SEQ: one axis at a time (fewer live registers); same operations, same order
    if constexpr (SEQ) {
#pragma unroll 1
      for (int ax = 0; ax < 3; ++ax) axis(ax);
    } else {
      axis(0);
      axis(1);
      axis(2);
    }
    out[0] = ((double)at(1, 0, 0) + ref[1]) + (double)(kos * ku);
    out[1] = (double)(lap / (h * h) + kos * kv);
  } else {
    // Maxwell: fields Ex Ey Ez Bx By Bz
    T d[F][3];
    T ko[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      ko[f] = T(0);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const T p1 = at(f, ax, 1), m1 = at(f, ax, -1), p2 = at(f, ax, 2), m2 = at(f, ax, -2), p3 = at(f, ax, 3),
                m3 = at(f, ax, -3);
        d[f][ax] = (T(D1C1) * (p1 - m1) + T(D1C2) * (p2 - m2) + T(D1C3) * (p3 - m3)) / h;
        ko[f] += (m3 + p3) - T(6) * (m2 + p2) + T(15) * (m1 + p1) - T(20) * at(f, ax, 0);
      }
    }
    // curl B, curl E (axis 0 = x, 1 = y, 2 = z)
    out[0] = (double)((d[5][1] - d[4][2]) + kos * ko[0]);
    out[1] = (double)((d[3][2] - d[5][0]) + kos * ko[1]);
    out[2] = (double)((d[4][0] - d[3][1]) + kos * ko[2]);
    out[3] = (double)(-(d[2][1] - d[1][2]) + kos * ko[3]);
    out[4] = (double)(-(d[0][2] - d[2][0]) + kos * ko[4]);
    out[5] = (double)(-(d[1][0] - d[0][1]) + kos * ko[5]);
  }
}

// Accessor of a padded array with point strides (1, sy, sz) and field stride fs.
template <typename T>
struct StridedAt {
  const T* Y;
  int64_t fs;
  int c, sy, sz;
  __device__ __forceinline__ T operator()(int f, int ax, int k) const {
    const int s = ax == 0 ? 1 : (ax == 1 ? sy : sz);
    return Y[f * fs + c + k * s];
  }
};

template <typename T, int EQ, int F>
__device__ __forceinline__ void rhs_point(const T* Y, int64_t fstride, int c, int sy, int sz, T h, T sigma,
                                          const double ref[F], double out[F]) {
  rhs_at<T, EQ, F>(StridedAt<T>{Y, fstride, c, sy, sz}, h, sigma, ref, out);
}

// ------------------------------------------------------------------ fused stage
// The block RHS reads only along the axes (centred first and second differences
// and Kreiss-Oliger terms, no mixed derivatives), so of the (4tt+7)^3 padded
// points of a tile it uses those with at most one coordinate in the 3-point halo.
// They are kept plane by plane: core plane z = 3 + gz (gz < G) as a P x P square
// at gz P^2 (its four 3 x 3 corners unused), then the six halo planes (z = h for
// h < 3, z = G + h for h >= 3) as G x G squares of the core x and y.
template <int TT>
struct Cross {
  static constexpr int P = 4 * TT + 7;     // padded points per axis
  static constexpr int G = 4 * TT + 1;     // grid points per axis
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
template <typename T, int TT>
struct CrossAt {
  const T* Y;
  int c, hb, gz;
  __device__ __forceinline__ T operator()(int f, int ax, int k) const {
    using X = Cross<TT>;
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
template <int TT, int F, bool KF32>
struct FusedLds {
  static constexpr int W = TT + 2;
  static constexpr int NS = W * W * W;
  static constexpr int G3 = (4 * TT + 1) * (4 * TT + 1) * (4 * TT + 1);
  using LT = typename std::conditional<KF32, float, double>::type;
  double R[F * G3];               // stencil results
  double wsh[16];                 // stage weights of the 4 time cases
  LT Y[F * Cross<TT>::LS];        // stage values of the used padded points
  // per-tile tables, two buffers: the next tile's are filled while this one runs
  double ref[2][F];               // FP32 stencils: reference value of each field
  int32_t sl[2][2 * NS];          // slot records
  uint8_t axl[2][3][4 * TT + 7];  // per axis: slot position | node offset << 3
};

// The arrays and schedule position of the simulation a tile belongs to.
struct SimView {
  const double* U;
  double* Uw;
  const void* K;
  void* Kw;
  int64_t N;
  int lmin, lmax, j;
  double sigma;
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

template <int TT, int F, bool KF32, int NT>
__device__ __forceinline__ TileTables tables_issue(const StageParams& sp, const TileRef& r, const int32_t* t) {
  constexpr int P = 4 * TT + 7;
  constexpr int NS2 = 2 * (TT + 2) * (TT + 2) * (TT + 2);
  static_assert(NT >= NS2 && NT >= 3 * P, "one table element per thread");
  TileTables tb{0, 0, 0.0};
  if (threadIdx.x < NS2) tb.slv = r.slots[2 * (int64_t)t[TI_SLOT] + threadIdx.x];
  if (threadIdx.x < 3 * P) {
    const int d = threadIdx.x / P, q = threadIdx.x - P * d;
    const int off = t[TI_OFF];
    const int o = (off >> (8 * d)) & 255;
    const int Q = 4 * o + q - 3;
    const int cell = cell_of(Q, t[TI_M]);
    tb.axv = (cell - o + 1) | ((Q - 4 * cell) << 3);
  }
  if (KF32 && threadIdx.x < F) {
    // FP32 stencils work on Y - ref (the Laplacian and KO ignore constants)
    const TileCtx c = tile_ctx(t, sp.mode, r.v.j, r.v.lmin, r.v.lmax, r.n4);
    const int64_t fsz = r.v.N * 125;
    tb.refv = r.v.U[((int64_t)c.par_same * F + threadIdx.x) * fsz + (int64_t)t[TI_FIRST] * 125];
  }
  return tb;
}

template <int TT, int F, bool KF32>
__device__ __forceinline__ void tables_store(FusedLds<TT, F, KF32>& L, int b, const TileTables& tb) {
  constexpr int P = 4 * TT + 7;
  constexpr int NS2 = 2 * (TT + 2) * (TT + 2) * (TT + 2);
  if (threadIdx.x < NS2) L.sl[b][threadIdx.x] = tb.slv;
  if (threadIdx.x < 3 * P) L.axl[b][threadIdx.x / P][threadIdx.x % P] = (uint8_t)tb.axv;
  if (threadIdx.x < F) L.ref[b][threadIdx.x] = KF32 ? tb.refv : 0.0;
}

// One tile of the fused stage (Sec. 3.3, eqs. fc_1/fc_2, eq. rk_schemes).  Its
// slot records and per-axis location tables (slot position and node offset of
// every padded coordinate, from the location rule) are in LDS buffer b.
//   (1) every used padded point takes its stage value: a same-level leaf (the
//       tile's own octants included) or 8 finer leaves give Y = U0 + dt sum w_i
//       K_i, read directly (uniform base pointers, 32-bit offsets, UB points per
//       thread loaded before use); a coarser leaf gives its prolongated value
//       from the ghost table;
//   (2) the stencils run once per tile grid point; K_s (and the RK update at the
//       last stage) are written to every DG node of the tile's contiguous octants.
// With a next tile, its record is loaded at the start and its tables during the
// stencils, into buffer b ^ 1.  Two barriers per tile: after the gather (the
// previous tile's zip has read the stencil results) and after the stencils.
// sp holds the stage (weights, masks).
template <int TT, int F, int EQ, bool KF32, int NT, int KS>
__device__ __forceinline__ void fused_tile(FusedLds<TT, F, KF32>& L, const StageParams& sp, const TileRef& cur,
                                           const int32_t* t, int b, const TileRef& nxt, bool more,
                                           int32_t (&ntrec)[8]) {
  using X = Cross<TT>;
  constexpr int P = X::P;
  constexpr int LS = X::LS;
  constexpr int W = TT + 2;
  constexpr int UB = 2;                      // points per thread loaded together
  using LT = typename std::conditional<KF32, float, double>::type;
  using KT = typename std::conditional<KF32, float, double>::type;
  const SimView& v = cur.v;
  const double* __restrict__ cs = cur.cs;
  auto& Y = L.Y;
  const int32_t* sl = L.sl[b];
  const auto& axl = L.axl[b];
  auto& wsh = L.wsh;
  const double* ref = L.ref[b];
  auto& R = L.R;
  if (more) load_trec(nxt.tile, ntrec);
  const int fsz = (int)(v.N * 125);          // elements per field (< 2^31)
  const bool last = sp.stage == sp.p - 1;
  const KT* __restrict__ Kr = (const KT*)v.K;
  KT* __restrict__ Kw = (KT*)v.Kw + (int64_t)sp.stage * F * fsz;
  // KS: stages read by same-level sources (the tableau row's non-zero pattern),
  // a compile-time mask so the hot gather has no branches around its loads
  const TileCtx c = tile_ctx(t, sp.mode, v.j, v.lmin, v.lmax, cur.n4);
  const int first = t[TI_FIRST];
  const double* __restrict__ Us = v.U + (int64_t)c.par_same * F * fsz;
  const double* __restrict__ Uf = v.U + (int64_t)c.par_fine * F * fsz;
  double* __restrict__ Uw1 = v.Uw + (int64_t)(c.par_same ^ 1) * F * fsz;
  const int kmf = stage_mask(sp, c.case_fine);
  const double* wf = wsh + 4 * c.case_fine;

  // (1) stage values of the used padded points
  for (int p0 = threadIdx.x; p0 < X::NC; p0 += UB * NT) {
    int li[UB], kind[UB], leaf[UB], kbv[UB], nuv[UB][3];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int pi = p0 + u * NT;
      kind[u] = -1;
      li[u] = 0;
      leaf[u] = 0;
      kbv[u] = 0;
      nuv[u][0] = nuv[u][1] = nuv[u][2] = 0;
      if (pi >= X::NC) continue;
      int qx, qy, qz;
      X::point(pi, qx, qy, qz, li[u]);
      const int ax = axl[0][qx], ay = axl[1][qy], az = axl[2][qz];
      const int si = (ax & 7) + W * ((ay & 7) + W * (az & 7));
      nuv[u][0] = ax >> 3;
      nuv[u][1] = ay >> 3;
      nuv[u][2] = az >> 3;
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
      const uint32_t off = same ? (uint32_t)(leaf[u] * 125 + nuv[u][0] + 5 * nuv[u][1] + 25 * nuv[u][2]) : 0u;
      // ghost-table entry (in the slot's first int), octant beta of the leaf
      const int beta = (kbv[u] >> 4) & 7;
      const int x2 = 4 * (beta & 1) + nuv[u][0], y2 = 4 * ((beta >> 1) & 1) + nuv[u][1],
                z2 = 4 * ((beta >> 2) & 1) + nuv[u][2];
      const double* pa = coarse ? cs + ((int64_t)leaf[u] * F * 729 + (z2 * 9 + y2) * 9 + x2) : Us + off;
      const int fst = coarse ? 729 : fsz;
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
        const int cx = min(nuv[u][0] >> 1, 1), cy = min(nuv[u][1] >> 1, 1), cz = min(nuv[u][2] >> 1, 1);
        const uint32_t off = (uint32_t)((leaf[u] + cx + 2 * cy + 4 * cz) * 125 + 2 * (nuv[u][0] - 2 * cx) +
                                        10 * (nuv[u][1] - 2 * cy) + 50 * (nuv[u][2] - 2 * cz));
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
      }
    }
  }
  TileTables tb{0, 0, 0.0};
  if (more) tb = tables_issue<TT, F, KF32, NT>(sp, nxt, ntrec);
  __syncthreads();
  // the last stage's RK operands are loaded in the zip: holding them across the
  // stencils would cost the registers that 3 resident side-2 workgroups leave
  constexpr int NN = TT * TT * TT * 125;
  constexpr int KZ = (NN + NT - 1) / NT;
  // (2a) stencils once per tile grid point (4tt+1)^3; results staged in LDS
  constexpr int G = X::G;
  constexpr int G3 = G * G * G;
  for (int gi = threadIdx.x; gi < G3; gi += NT) {
    const int gx = gi % G, gy = (gi / G) % G, gz = gi / (G * G);
    const int ce = (gz * P + gy + 3) * P + gx + 3;
    double k[F];
    // one axis at a time: fewer live registers (same operations, same order)
    rhs_at<LT, EQ, F, true>(CrossAt<LT, TT>{Y, ce, X::HB + gy * G + gx, gz}, (LT)c.h, (LT)v.sigma, ref, k);
#pragma unroll
    for (int f = 0; f < F; ++f) R[f * G3 + gi] = k[f];
  }
  if (more) tables_store(L, b ^ 1, tb);
  __syncthreads();
  // (2b) zip: every DG node of the tile's (contiguous) octants takes its grid
  // value; node e of the tile is element first*125 + e of every field array;
  // the last stage also forms the RK update
  double bs = sp.b[0];   // b_s without a dynamic index into the kernel arguments
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i == sp.stage) bs = sp.b[i];
#pragma unroll
  for (int u = 0; u < KZ; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e >= NN) continue;
    const uint32_t off = (uint32_t)(first * 125 + e);
    double zu[F], zk[F][3];
    if (last) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        zu[f] = ld32(Us + (uint32_t)(f * fsz), off);
#pragma unroll
        for (int i = 0; i < 3; ++i)
          zk[f][i] = (i < sp.stage) ? (double)ld32(Kr + (uint32_t)((i * F + f) * fsz), off) : 0.0;
      }
    }
    const int o = e / 125, node = e - 125 * (e / 125);
    const int a = node % 5, b = (node / 5) % 5, cc = node / 25;
    const int gi = ((4 * ((o >> 2) & 1) + cc) * G + (4 * ((o >> 1) & 1) + b)) * G + (4 * (o & 1) + a);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      double kv = R[f * G3 + gi];
      if constexpr (KF32) {
        const float kf = (float)kv;
        st32(Kw + (uint32_t)(f * fsz), off, kf);
        kv = (double)kf;
      } else {
        st32(Kw + (uint32_t)(f * fsz), off, kv);
      }
      if (last) {
        // compute_step_partial: U_new = U0 + dt (b_0 K_0 + ... + b_s K_s),
        // s = p - 1, accumulated in stage order, into the other buffer
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          if (i < sp.stage) acc = fma(sp.b[i], zk[f][i], acc);
        acc = fma(bs, kv, acc);
        st32(Uw1 + (uint32_t)(f * fsz), off, zu[f] + c.dt * acc);
      }
    }
  }
}

template <int TT, int F, bool KF32>
__device__ __forceinline__ void fused_init(FusedLds<TT, F, KF32>& L, const StageParams& sp) {
  if (threadIdx.x < 16) L.wsh[threadIdx.x] = stage_weight(sp, threadIdx.x);
}

// Waves per SIMD that the LDS of one workgroup allows: the register budget the
// compiler is asked to keep so that registers do not cost occupancy.  Capped
// where a tighter budget spills: 6 (80 registers) for FP64 side-2 tiles, 8 (64)
// with FP32 stencils, 5 for side-1 tiles; left free for 6 fields.
template <int TT, int F, bool KF32, int NT>
constexpr int fused_waves_per_eu() {
  const int wg = (160 * 1024) / (int)sizeof(FusedLds<TT, F, KF32>);
  const int w = wg * (NT / 64) / 4;
  const int cap = TT == 1 ? 5 : (KF32 ? 8 : 6);
  return (F > 2 || w < 1) ? 1 : (w > cap ? cap : w);
}

// Tile range [lo, hi) of XCD x (uniform): unrolled selects, so that the kernel
// argument array is not indexed at run time (which would copy it to scratch).
__device__ __forceinline__ void xcd_range(const XcdRanges& xr, int x, int& lo, int& hi) {
  lo = xr.b[0];
  hi = xr.b[1];
#pragma unroll
  for (int k = 1; k < 8; ++k)
    if (k == x) {
      lo = xr.b[k];
      hi = xr.b[k + 1];
    }
}

// A workgroup's walk over tiles lo, lo + step, ... < hi; ref_of(i) gives tile i.
// The first tile's tables are loaded here, every later one's by the tile before.
template <int TT, int F, int EQ, bool KF32, int NT, int KS, typename RefOf>
__device__ __forceinline__ void fused_walk(FusedLds<TT, F, KF32>& L, const StageParams& sp, int lo, int step, int hi,
                                           const RefOf& ref_of) {
  if (lo >= hi) return;
  TileRef cur = ref_of(lo);
  int32_t trec[8];
  load_trec(cur.tile, trec);
  tables_store(L, 0, tables_issue<TT, F, KF32, NT>(sp, cur, trec));
  __syncthreads();
  int b = 0;
  for (int ti = lo;; ti += step) {
    const bool more = ti + step < hi;
    TileRef nxt = more ? ref_of(ti + step) : cur;
    int32_t ntrec[8];
    fused_tile<TT, F, EQ, KF32, NT, KS>(L, sp, cur, trec, b, nxt, more, ntrec);
    if (!more) break;
    cur = nxt;
#pragma unroll
    for (int k = 0; k < 8; ++k) trec[k] = ntrec[k];
    b ^= 1;
  }
}

// One mesh: workgroups are dealt to the 8 XCDs round robin; XCD x walks its own
// contiguous (Morton-ordered, cost-balanced) range of tiles.  Coarser ghosts come
// prolongated from the ghost-table pre-pass (scr).
template <int TT, int F, int EQ, bool KF32, int NT, int KS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(fused_waves_per_eu<TT, F, KF32, NT>())))
void k_fused(StageParams sp, const int32_t* __restrict__ tiles, const int32_t* __restrict__ slots,
             const double* __restrict__ scr, XcdRanges xr) {
  __shared__ FusedLds<TT, F, KF32> L;
  fused_init(L, sp);
  const int n4 = (int)(*sp.step & 3);
  const int nslot = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7;
  const int sid = blockIdx.x >> 3;
  const SimView v{sp.U, sp.Uw, sp.K, sp.Kw, sp.N, sp.lmin, sp.lmax, sp.j, sp.sigma};
  int lo, hi;
  xcd_range(xr, xcd, lo, hi);
  fused_walk<TT, F, EQ, KF32, NT, KS>(L, sp, lo + sid, nslot, hi, [&](int ti) {
    return TileRef{v, n4, tiles + 8 * (int64_t)ti, slots, scr};
  });
}

// Several independent meshes advanced together (continuous batching): in round r
// every simulation of the table is at its own substep (BatchSim); one launch per
// stage covers the union of the active tiles of side TT of all of them, in table
// order.  Union tile t belongs to the simulation whose cumulative-count range
// holds it; the union is cut into 8 contiguous ranges, one per XCD.  The
// arithmetic of every tile is that of the one-mesh kernel; coarser ghosts come
// from the batch's ghost pre-pass (scr, simulation s at entry gbase_s).
template <int TT, int F, int EQ, bool KF32, int NT, int KS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(fused_waves_per_eu<TT, F, KF32, NT>())))
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

// ------------------------------------------------------------------ streamed blocks
// Whole 4^3-octant blocks (side-4 tiles) are streamed along z: the padded block
// (23^3 points per field) never sits in LDS at once.  A ring of 8 padded planes
// holds the 7 planes one output plane of the 17^3 block grid needs plus the plane
// being loaded, so the loads of padded plane z+7 are in flight while the stencils
// of output plane z run.  Of each plane only the points a stencil reads are
// gathered: 1.26 points per DG node, against 2.19 for side-2 tiles.

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
                                                         double* __restrict__ scr) {
  __shared__ GhostLds<F> L;
  __shared__ int cum[kMaxBatch + 1];
  ghost_init(L, sp0);
  const int64_t r = *round;
  for (int s = threadIdx.x; s < nsims; s += blockDim.x) {
    const BatchSim& b = sims[s];
    const int64_t rr = r - b.r0;
    int cnt = 0;
    if (rr >= 0 && rr < b.rounds) {
      const int j = (int)(rr & ((1 << (b.lmax - b.lmin)) - 1));
      const int lo = (sp0.mode == LTS_MODE_GTS || j == 0) ? b.lmin : b.lmax - __builtin_ctz(j);
      cnt = b.ghost_ge[lo];
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
      if constexpr (KF32) {
        const float kf = (float)kv;
        st32(x.Kw + (uint32_t)(f * x.fsz), off, kf);
        kv = (double)kf;
      } else {
        st32(x.Kw + (uint32_t)(f * x.fsz), off, kv);
      }
      if constexpr (LAST) {
        // U0 + dt (b_0 K_0 + ... + b_s K_s), s = p - 1, accumulated in stage order
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          if (i < sp.stage) acc = fma(sp.b[i], kp[f][i], acc);
        acc = fma(bs, kv, acc);
        st32(x.Uw1 + (uint32_t)(f * x.fsz), off, u0[f] + x.dt * acc);
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

// ------------------------------------------------------------------ standalone kernels
template <bool KF32, int F>
__global__ __launch_bounds__(256) void k_unzip(StageParams sp, const int32_t* __restrict__ tiles,
                                               const int32_t* __restrict__ slots, const int32_t* __restrict__ list,
                                               const int64_t* __restrict__ off, int64_t total, double* out) {
  __shared__ double wsh[16];
  if (threadIdx.x < 16) wsh[threadIdx.x] = stage_weight(sp, threadIdx.x);
  __syncthreads();
  const int bi = blockIdx.y;
  const int b = list[bi];
  const int32_t* t = tiles + 8 * (int64_t)b;
  const int n4 = (int)(*sp.step & 3);
  const TileCtx c = tile_ctx(t, sp, n4);
  const int P = 4 * c.m + 7;
  const int P3 = P * P * P;
  const int32_t* sl = slots + 2 * (int64_t)t[TI_SLOT];
  for (int pi = blockIdx.x * blockDim.x + threadIdx.x; pi < P3; pi += gridDim.x * blockDim.x) {
    const int qx = pi % P, qy = (pi / P) % P, qz = pi / (P * P);
    double v[F];
    point_values<KF32, F>(sp, c, sl, wsh, qx, qy, qz, v);
    #pragma unroll
    for (int f = 0; f < F; ++f) out[f * total + off[bi] + pi] = v[f];
  }
}

template <int EQ, int F, bool F32>
__global__ __launch_bounds__(256) void k_rhs(const int32_t* __restrict__ tiles, const int32_t* __restrict__ list,
                                             const int64_t* __restrict__ poff, int64_t ptotal,
                                             const int64_t* __restrict__ goff, int64_t gtotal,
                                             const double* __restrict__ padded, void* kout, double sigma) {
  const int bi = blockIdx.y;
  const int32_t* t = tiles + 8 * (int64_t)list[bi];
  const int m = t[TI_M];
  const int P = 4 * m + 7, G = 4 * m + 1;
  const int G3 = G * G * G;
  const double h = ldexp(1.0, -t[TI_LEVEL] - 1);
  for (int gi = blockIdx.x * blockDim.x + threadIdx.x; gi < G3; gi += gridDim.x * blockDim.x) {
    const int gx = gi % G, gy = (gi / G) % G, gz = gi / (G * G);
    const int ci = ((gz + 3) * P + (gy + 3)) * P + (gx + 3);
    double k[F];
    if constexpr (F32) {
      // float stencils on Y - ref, ref = the block's first grid value
      double ref[F];
      const int c0 = (3 * P + 3) * P + 3;
      #pragma unroll
      for (int f = 0; f < F; ++f) ref[f] = padded[f * ptotal + poff[bi] + c0];
      const int st[3] = {1, P, P * P};
      if constexpr (EQ == LTS_EQ_WAVE) {
        const double* u = padded + poff[bi];
        const double* v = padded + ptotal + poff[bi];
        float lap = 0.f, ku = 0.f, kv = 0.f;
        for (int ax = 0; ax < 3; ++ax) {
          const int s = st[ax];
          float uu[7], vv[7];
          for (int q = 0; q < 7; ++q) {
            uu[q] = (float)(u[ci + (q - 3) * s] - ref[0]);
            vv[q] = (float)(v[ci + (q - 3) * s] - ref[1]);
          }
          lap += float(D2C3) * (uu[0] + uu[6]) + float(D2C2) * (uu[1] + uu[5]) + float(D2C1) * (uu[2] + uu[4]) +
                 float(D2C0) * uu[3];
          ku += (uu[0] + uu[6]) - 6.f * (uu[1] + uu[5]) + 15.f * (uu[2] + uu[4]) - 20.f * uu[3];
          kv += (vv[0] + vv[6]) - 6.f * (vv[1] + vv[5]) + 15.f * (vv[2] + vv[4]) - 20.f * vv[3];
        }
        const float hf = (float)h;
        const float kos = (float)sigma / (64.f * hf);
        k[0] = ((double)(float)(v[ci] - ref[1]) + ref[1]) + (double)(kos * ku);
        k[1] = (double)(lap / (hf * hf) + kos * kv);
      } else {
        float d[F][3], ko[F];
        for (int f = 0; f < F; ++f) {
          const double* g = padded + f * ptotal + poff[bi];
          ko[f] = 0.f;
          for (int ax = 0; ax < 3; ++ax) {
            const int s = st[ax];
            float gg[7];
            for (int q = 0; q < 7; ++q) gg[q] = (float)(g[ci + (q - 3) * s] - ref[f]);
            d[f][ax] = (float(D1C1) * (gg[4] - gg[2]) + float(D1C2) * (gg[5] - gg[1]) + float(D1C3) * (gg[6] - gg[0])) /
                       (float)h;
            ko[f] += (gg[0] + gg[6]) - 6.f * (gg[1] + gg[5]) + 15.f * (gg[2] + gg[4]) - 20.f * gg[3];
          }
        }
        const float kos = (float)sigma / (64.f * (float)h);
        k[0] = (double)((d[5][1] - d[4][2]) + kos * ko[0]);
        k[1] = (double)((d[3][2] - d[5][0]) + kos * ko[1]);
        k[2] = (double)((d[4][0] - d[3][1]) + kos * ko[2]);
        k[3] = (double)(-(d[2][1] - d[1][2]) + kos * ko[3]);
        k[4] = (double)(-(d[0][2] - d[2][0]) + kos * ko[4]);
        k[5] = (double)(-(d[1][0] - d[0][1]) + kos * ko[5]);
      }
    } else {
      const double zero[F] = {};
      rhs_point<double, EQ, F>(padded + poff[bi], ptotal, ci, P, P * P, h, sigma, zero, k);
    }
    #pragma unroll
    for (int f = 0; f < F; ++f) {
      if constexpr (F32) ((float*)kout)[f * gtotal + goff[bi] + gi] = (float)k[f];
      else ((double*)kout)[f * gtotal + goff[bi] + gi] = k[f];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zip(const int32_t* __restrict__ tiles, const int32_t* __restrict__ list,
                                             const int64_t* __restrict__ goff, int64_t gtotal, int F, int64_t N,
                                             const T* __restrict__ kblock, T* __restrict__ kout) {
  const int bi = blockIdx.y;
  const int32_t* t = tiles + 8 * (int64_t)list[bi];
  const int m = t[TI_M];
  const int G = 4 * m + 1;
  const int first = t[TI_FIRST];
  const int nn = m * m * m * 125;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) {
    const int o = e / 125, node = e % 125;
    // octant o of the block in Morton order -> lexicographic octant coordinates
    int ox = 0, oy = 0, oz = 0;
    for (int bit = 0; bit < 3; ++bit) {
      ox |= ((o >> (3 * bit)) & 1) << bit;
      oy |= ((o >> (3 * bit + 1)) & 1) << bit;
      oz |= ((o >> (3 * bit + 2)) & 1) << bit;
    }
    const int gx = 4 * ox + node % 5, gy = 4 * oy + (node / 5) % 5, gz = 4 * oz + node / 25;
    const int64_t gi = ((int64_t)gz * G + gy) * G + gx;
    for (int f = 0; f < F; ++f) kout[(f * N + first + o) * 125 + node] = kblock[f * gtotal + goff[bi] + gi];
  }
}

template <bool KF32>
__global__ __launch_bounds__(256) void k_rk(StageParams sp, const int32_t* __restrict__ tiles,
                                            const int32_t* __restrict__ list, const double* __restrict__ coef,
                                            double* out) {
  const int bi = blockIdx.y;
  const int32_t* t = tiles + 8 * (int64_t)list[bi];
  const int n4 = (int)(*sp.step & 3);
  const TileCtx c = tile_ctx(t, sp, n4);
  const int first = t[TI_FIRST];
  const int nn = c.m * c.m * c.m * 125;
  const int64_t fs = sp.N * 125, ps = fs * sp.F;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)first * 125 + e;
    for (int f = 0; f < sp.F; ++f) {
      double acc = 0.0;
      for (int i = 0; i < sp.p; ++i) acc = fma(coef[i], kload<KF32>(sp.K, i * ps + f * fs + idx), acc);
      const double v = sp.U[c.par_same * ps + f * fs + idx] + c.dt * acc;
      if (out) out[f * fs + idx] = v;
      else sp.Uw[(c.par_same ^ 1) * ps + f * fs + idx] = v;
    }
  }
}

// current state: block b's buffer after a whole number of coarse steps
__global__ __launch_bounds__(256) void k_current(StageParams sp, const int32_t* __restrict__ tiles, int nblocks,
                                                 double* out) {
  const int b = blockIdx.y;
  if (b >= nblocks) return;
  const int32_t* t = tiles + 8 * (int64_t)b;
  const int lev = t[TI_LEVEL];
  const int m = t[TI_M];
  const int first = t[TI_FIRST];
  const int64_t n = *sp.step;
  // steps taken: LTS n 2^(lev-lmin), GTS n 2^(lmax-lmin)
  const int64_t steps = sp.mode == LTS_MODE_GTS ? (n << (sp.lmax - sp.lmin)) : (n << (lev - sp.lmin));
  const int par = (int)(steps & 1);
  const int64_t fs = sp.N * 125, ps = fs * sp.F;
  const int nn = m * m * m * 125;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)first * 125 + e;
    for (int f = 0; f < sp.F; ++f) out[f * fs + idx] = sp.U[par * ps + f * fs + idx];
  }
}

__global__ void k_increment(int64_t* ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] += 1;
}

// per-octant partial sums for the norms: [F][N] sum e^2, [F][N] max |e|, nonfinite count
__global__ __launch_bounds__(128) void k_norm_partials(const double* a, const double* b, int F, int64_t N,
                                                       double* sq, double* mx, unsigned long long* bad) {
  const int64_t o = blockIdx.x;
  const int f = blockIdx.y;
  __shared__ double s1[128], s2[128];
  __shared__ int s3[128];
  double q = 0.0, m = 0.0;
  int nb = 0;
  const int node = threadIdx.x;
  if (node < 125) {
    const int64_t idx = ((int64_t)f * N + o) * 125 + node;
    const double x = a[idx];
    const double e = b ? x - b[idx] : x;
    if (!isfinite(x)) nb = 1;
    q = e * e;
    m = fabs(e);
  }
  s1[threadIdx.x] = q;
  s2[threadIdx.x] = m;
  s3[threadIdx.x] = nb;
  __syncthreads();
  for (int w = 64; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + w]);
      s3[threadIdx.x] += s3[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sq[(int64_t)f * N + o] = s1[0];
    mx[(int64_t)f * N + o] = s2[0];
    if (s3[0]) atomicAdd(bad, (unsigned long long)s3[0]);
  }
}

__global__ __launch_bounds__(256) void k_copy(const double4* __restrict__ src, double4* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ------------------------------------------------------------------ launchers
namespace {
int fused_grid(int ntiles, int max_wg) {
  int g = std::min(ntiles, max_wg);
  g = (g + 7) & ~7;
  return std::max(g, 8);
}
}  // namespace

namespace {
struct OneArgs {
  const int32_t* tiles;
  const int32_t* slots;
  const double* scr;
  XcdRanges xr;
};
struct BatchArgs {
  const BatchSim* sims;
  int nsims;
  const int64_t* round;
  int64_t total;
  const double* scr;
};
}  // namespace

// Launch of one template combination; the argument pack selects the kernel.
template <int TT, int F, int EQ, bool KF32, int NT, int KS>
static hipError_t go(const StageParams& sp, const OneArgs& a, int max_wg, hipStream_t s) {
  hipLaunchKernelGGL((k_fused<TT, F, EQ, KF32, NT, KS>), dim3(fused_grid(a.xr.b[8], max_wg)), dim3(NT), 0, s, sp,
                     a.tiles, a.slots, a.scr, a.xr);
  return hipGetLastError();
}
template <int TT, int F, int EQ, bool KF32, int NT, int KS>
static hipError_t go(const StageParams& sp, const BatchArgs& a, int max_wg, hipStream_t s) {
  const int grid = fused_grid((int)std::min<int64_t>(a.total, 1 << 30), std::min(max_wg, kBatchMaxWg));
  hipLaunchKernelGGL((k_fused_batch<TT, F, EQ, KF32, NT, KS>), dim3(grid), dim3(NT), 0, s, sp, a.sims, a.nsims,
                     a.round, a.scr);
  return hipGetLastError();
}

// The same-level stage mask and the workgroup size are template arguments: the
// masks that occur for the built tableaus are RK4: none, {0}, {1}, {2} and
// SSP-RK3: none, {0}, {0,1}.
template <int TT, int F, int EQ, bool KF32, int NT, typename A>
static hipError_t dispatch_ks(const StageParams& sp, const A& a, int max_wg, hipStream_t s) {
  switch (sp.kmask[0]) {
    case 0: return go<TT, F, EQ, KF32, NT, 0>(sp, a, max_wg, s);
    case 1: return go<TT, F, EQ, KF32, NT, 1>(sp, a, max_wg, s);
    case 2: return go<TT, F, EQ, KF32, NT, 2>(sp, a, max_wg, s);
    case 3: return go<TT, F, EQ, KF32, NT, 3>(sp, a, max_wg, s);
    case 4: return go<TT, F, EQ, KF32, NT, 4>(sp, a, max_wg, s);
    default: return hipErrorInvalidValue;
  }
}

template <int TT, int F, int EQ, bool KF32, typename A>
static hipError_t dispatch_nt(const StageParams& sp, const A& a, const LaunchShape& ls, hipStream_t s) {
  switch (ls.threads) {
    case 256: return dispatch_ks<TT, F, EQ, KF32, 256>(sp, a, ls.max_wg, s);
    case 512: return dispatch_ks<TT, F, EQ, KF32, 512>(sp, a, ls.max_wg, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename A>
static hipError_t dispatch_fused(int tt, int eq, bool kf32, const StageParams& sp, const A& a, const LaunchShape& ls,
                                 hipStream_t s) {
  if (eq == LTS_EQ_WAVE) {
    if (tt == 1) return kf32 ? dispatch_nt<1, 2, LTS_EQ_WAVE, true>(sp, a, ls, s)
                             : dispatch_nt<1, 2, LTS_EQ_WAVE, false>(sp, a, ls, s);
    if (tt == 2) return kf32 ? dispatch_nt<2, 2, LTS_EQ_WAVE, true>(sp, a, ls, s)
                             : dispatch_nt<2, 2, LTS_EQ_WAVE, false>(sp, a, ls, s);
    return hipErrorInvalidValue;
  }
  if (tt != 1) return hipErrorInvalidValue;  // 6 FP64 fields of a side-2 tile exceed LDS
  return kf32 ? dispatch_nt<1, 6, LTS_EQ_MAXWELL, true>(sp, a, ls, s)
              : dispatch_nt<1, 6, LTS_EQ_MAXWELL, false>(sp, a, ls, s);
}

hipError_t launch_fused(int tt, int eq, bool kf32, const StageParams& sp, const int32_t* tiles,
                        const int32_t* slots, const double* scr, const XcdRanges& xr, const LaunchShape& ls,
                        hipStream_t s) {
  if (xr.b[8] <= 0) return hipSuccess;
  return dispatch_fused(tt, eq, kf32, sp, OneArgs{tiles, slots, scr, xr}, ls, s);
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

hipError_t launch_fused_batch(int tt, int eq, bool kf32, const StageParams& sp0, const BatchSim* sims, int nsims,
                              const int64_t* round, int64_t total, const double* scr, const LaunchShape& ls,
                              hipStream_t s) {
  if (total <= 0 || nsims <= 0) return hipSuccess;
  if (nsims > kMaxBatch) return hipErrorInvalidValue;
  return dispatch_fused(tt, eq, kf32, sp0, BatchArgs{sims, nsims, round, total, scr}, ls, s);
}

hipError_t launch_ghost_pre_batch(int F, bool kf32, const StageParams& sp0, const BatchSim* sims, int nsims,
                                  const int64_t* round, int64_t total, double* scr, int max_wg, hipStream_t s) {
  if (total <= 0 || nsims <= 0) return hipSuccess;
  if (nsims > kMaxBatch) return hipErrorInvalidValue;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(total, std::min(max_wg, kBatchMaxWg))));
  if (F == 2) {
    if (kf32) hipLaunchKernelGGL((k_ghost_pre_batch<true, 2>), grid, dim3(256), 0, s, sp0, sims, nsims, round, scr);
    else hipLaunchKernelGGL((k_ghost_pre_batch<false, 2>), grid, dim3(256), 0, s, sp0, sims, nsims, round, scr);
  } else if (F == 6) {
    if (kf32) hipLaunchKernelGGL((k_ghost_pre_batch<true, 6>), grid, dim3(256), 0, s, sp0, sims, nsims, round, scr);
    else hipLaunchKernelGGL((k_ghost_pre_batch<false, 6>), grid, dim3(256), 0, s, sp0, sims, nsims, round, scr);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
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

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_set_i64(int64_t* ptr, int64_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, ptr, value);
  return hipGetLastError();
}

hipError_t launch_unzip(bool kf32, const StageParams& sp, const int32_t* tiles, const int32_t* slots,
                        const int32_t* list, const int64_t* off, int nb, int64_t total, double* out, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  dim3 grid(8, nb);
  if (sp.F == 2) {
    if (kf32) hipLaunchKernelGGL((k_unzip<true, 2>), grid, dim3(256), 0, s, sp, tiles, slots, list, off, total, out);
    else hipLaunchKernelGGL((k_unzip<false, 2>), grid, dim3(256), 0, s, sp, tiles, slots, list, off, total, out);
  } else if (sp.F == 6) {
    if (kf32) hipLaunchKernelGGL((k_unzip<true, 6>), grid, dim3(256), 0, s, sp, tiles, slots, list, off, total, out);
    else hipLaunchKernelGGL((k_unzip<false, 6>), grid, dim3(256), 0, s, sp, tiles, slots, list, off, total, out);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rhs(int eq, bool f32, const int32_t* tiles, const int32_t* list, const int64_t* poff,
                      int64_t ptotal, const int64_t* goff, int64_t gtotal, int nb, const double* padded, void* kout,
                      double sigma, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  dim3 grid(8, nb);
  if (eq == LTS_EQ_WAVE) {
    if (f32) hipLaunchKernelGGL((k_rhs<LTS_EQ_WAVE, 2, true>), grid, dim3(256), 0, s, tiles, list, poff, ptotal, goff,
                                gtotal, padded, kout, sigma);
    else hipLaunchKernelGGL((k_rhs<LTS_EQ_WAVE, 2, false>), grid, dim3(256), 0, s, tiles, list, poff, ptotal, goff,
                            gtotal, padded, kout, sigma);
  } else {
    if (f32) hipLaunchKernelGGL((k_rhs<LTS_EQ_MAXWELL, 6, true>), grid, dim3(256), 0, s, tiles, list, poff, ptotal,
                                goff, gtotal, padded, kout, sigma);
    else hipLaunchKernelGGL((k_rhs<LTS_EQ_MAXWELL, 6, false>), grid, dim3(256), 0, s, tiles, list, poff, ptotal,
                            goff, gtotal, padded, kout, sigma);
  }
  return hipGetLastError();
}

hipError_t launch_zip(bool f32, const int32_t* tiles, const int32_t* list, const int64_t* goff, int64_t gtotal, int nb,
                      int F, int64_t N, const void* kblock, void* kout, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  dim3 grid(8, nb);
  if (f32) hipLaunchKernelGGL((k_zip<float>), grid, dim3(256), 0, s, tiles, list, goff, gtotal, F, N,
                              (const float*)kblock, (float*)kout);
  else hipLaunchKernelGGL((k_zip<double>), grid, dim3(256), 0, s, tiles, list, goff, gtotal, F, N,
                          (const double*)kblock, (double*)kout);
  return hipGetLastError();
}

hipError_t launch_rk(bool kf32, const StageParams& sp, const int32_t* tiles, const int32_t* list, int nb,
                     const double* coef, double* out, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  dim3 grid(4, nb);
  if (kf32) hipLaunchKernelGGL((k_rk<true>), grid, dim3(256), 0, s, sp, tiles, list, coef, out);
  else hipLaunchKernelGGL((k_rk<false>), grid, dim3(256), 0, s, sp, tiles, list, coef, out);
  return hipGetLastError();
}

hipError_t launch_current(const StageParams& sp, const int32_t* tiles, int nblocks, double* out, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_current, dim3(4, nblocks), dim3(256), 0, s, sp, tiles, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_increment(int64_t* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_increment, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}

hipError_t launch_norm_partials(const double* a, const double* b, int F, int64_t N, double* sq, double* mx,
                                unsigned long long* bad, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_norm_partials, dim3((unsigned)N, F), dim3(128), 0, s, a, b, F, N, sq, mx, bad);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t nbytes, hipStream_t s) {
  const int64_t n = (int64_t)(nbytes / sizeof(double4));
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(2048), dim3(256), 0, s, (const double4*)src, (double4*)dst, n);
  return hipGetLastError();
}

}  // namespace lts
