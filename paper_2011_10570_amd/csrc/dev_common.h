// Device helpers shared by the HIP kernels of the LTS hot path (gfx950).
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
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lts_impl.h"
#include "lts_kernels.h"

namespace lts {

// Degree-4 Lagrange weights L_k(xi) = prod_{m != k} (xi - m)/(k - m) on nodes
// 0..4 at xi = x2/2 (x2 = 0..8).  Exact binary fractions (denominator 128).
static __constant__ double c_lag[9][5] = {
    {1, 0, 0, 0, 0},
    {35.0 / 128, 140.0 / 128, -70.0 / 128, 28.0 / 128, -5.0 / 128},
    {0, 1, 0, 0, 0},
    {-5.0 / 128, 60.0 / 128, 90.0 / 128, -20.0 / 128, 3.0 / 128},
    {0, 0, 1, 0, 0},
    {3.0 / 128, -20.0 / 128, 90.0 / 128, 60.0 / 128, -5.0 / 128},
    {0, 0, 0, 1, 0},
    {-5.0 / 128, 28.0 / 128, -70.0 / 128, 140.0 / 128, 35.0 / 128},
    {0, 0, 0, 0, 1}};

// The same for degree 6 on nodes 0..6 at xi = x2/2 (x2 = 0..12), 7-node octants.
// Exact binary fractions (denominator 1024).
static __constant__ double c_lag7[13][7] = {
    {1, 0, 0, 0, 0, 0, 0},
    {231.0 / 1024, 693.0 / 512, -1155.0 / 1024, 231.0 / 256, -495.0 / 1024, 77.0 / 512, -21.0 / 1024},
    {0, 1, 0, 0, 0, 0, 0},
    {-21.0 / 1024, 189.0 / 512, 945.0 / 1024, -105.0 / 256, 189.0 / 1024, -27.0 / 512, 7.0 / 1024},
    {0, 0, 1, 0, 0, 0, 0},
    {7.0 / 1024, -35.0 / 512, 525.0 / 1024, 175.0 / 256, -175.0 / 1024, 21.0 / 512, -5.0 / 1024},
    {0, 0, 0, 1, 0, 0, 0},
    {-5.0 / 1024, 21.0 / 512, -175.0 / 1024, 175.0 / 256, 525.0 / 1024, -35.0 / 512, 7.0 / 1024},
    {0, 0, 0, 0, 1, 0, 0},
    {7.0 / 1024, -27.0 / 512, 189.0 / 1024, -105.0 / 256, 945.0 / 1024, 189.0 / 512, -21.0 / 1024},
    {0, 0, 0, 0, 0, 1, 0},
    {-21.0 / 1024, 77.0 / 512, -495.0 / 1024, 231.0 / 256, -1155.0 / 1024, 693.0 / 512, 231.0 / 1024},
    {0, 0, 0, 0, 0, 0, 1}};

// Node spacing of a level-lev octant of [-1, 1]^3 with NI node intervals per
// side, h = 2^(1-lev) / NI (a power of two for NI = 4), and the step dt = h / 4.
template <int NI>
__device__ __forceinline__ double h_level(int lev) {
  if constexpr (NI == 4) return ldexp(1.0, -lev - 1);
  else return ldexp(1.0, 1 - lev) / (double)NI;
}

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

template <int NI = 4>
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
    c.dt = 0.25 * h_level<NI>(lmax);
  } else {
    // a finer neighbour steps twice per receiver step: its step index is 2 s;
    // a coarser one once per two: its index is floor(s / 2) (Sec. 3.6.3).
    c.par_fine = 0;
    c.par_coarse = (s >> 1) & 1;
    c.case_fine = 1;                                   // (delta, rho) = (0, 1/2)
    c.case_coarse = 2 + ((j >> (lmax - c.lev)) & 1);  // (0, 2) or (1, 2)
    c.dt = 0.25 * h_level<NI>(c.lev);
  }
  c.h = h_level<NI>(c.lev);
  return c;
}

template <int NI = 4>
__device__ __forceinline__ TileCtx tile_ctx(const int32_t* t, const StageParams& sp, int n4) {
  return tile_ctx<NI>(t, sp.mode, sp.j, sp.lmin, sp.lmax, n4);
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

// Y = U0 + dt sum_i w_i K_i at one DG node (field stride fs = N*NN, NN nodes
// per octant); only the stages with a non-zero weight (bit mask km, uniform per
// case) are read.
template <bool KF32, int NN = 125>
__device__ __forceinline__ double yval(const StageParams& sp, const double* w, int km, int par, int64_t idx,
                                       double dt) {
  const int64_t fs = sp.N * NN;
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
// slot table; wsh: stage-s weights per case [4][4].  NI: node intervals per
// octant side (4, or 6 for 7-node octants).
template <bool KF32, int F, int NI = 4>
__device__ __forceinline__ void point_values(const StageParams& sp, const TileCtx& c, const int32_t* slots,
                                             const double* wsh, int qx, int qy, int qz, double out[F]) {
  constexpr int NP = NI + 1, NN = NP * NP * NP;
  const Loc L = locate(qx, qy, qz, c.ox, c.oy, c.oz, c.tt, c.m, NI);
  const int leaf = slots[2 * L.slot];
  const int kb = slots[2 * L.slot + 1];
  const int kind = kb & 15;
  const int64_t fs = sp.N * NN;
  if (kind == SRC_NONE) {   // beyond the outer faces: no source
#pragma unroll
    for (int f = 0; f < F; ++f) out[f] = 0.0;
    return;
  }
  if (kind != SRC_COARSE) {
    int node, lf, par, km;
    const double* w;
    if (kind == SRC_FINE) {
      if constexpr (NI == 4) {
        const int cx = min(L.nu[0] >> 1, 1), cy = min(L.nu[1] >> 1, 1), cz = min(L.nu[2] >> 1, 1);
        lf = leaf + cx + 2 * cy + 4 * cz;
        node = 2 * (L.nu[0] - 2 * cx) + 5 * 2 * (L.nu[1] - 2 * cy) + 25 * 2 * (L.nu[2] - 2 * cz);
      } else {
        // 2:1 balance: the slot names a row of the fine table (children next to
        // the block are leaves)
        const int cx = fine_child6(L.nu[0], L.below & 1), cy = fine_child6(L.nu[1], (L.below >> 1) & 1),
                  cz = fine_child6(L.nu[2], (L.below >> 2) & 1);
        lf = sp.fine8[8 * leaf + cx + 2 * cy + 4 * cz];
        node = (2 * L.nu[0] - NI * cx) + NP * (2 * L.nu[1] - NI * cy) + NP * NP * (2 * L.nu[2] - NI * cz);
      }
      par = c.par_fine;
      w = wsh + 4 * c.case_fine;
      km = stage_mask(sp, c.case_fine);
    } else {
      lf = leaf;
      node = L.nu[0] + NP * L.nu[1] + NP * NP * L.nu[2];
      par = c.par_same;
      w = wsh;
      km = sp.kmask[0];
    }
    const int64_t base = (int64_t)lf * NN + node;
    #pragma unroll
    for (int f = 0; f < F; ++f) out[f] = yval<KF32, NN>(sp, w, km, par, f * fs + base, c.dt);
    return;
  }
  // coarser source: tensor degree-NI Lagrange interpolation of its Y values
  const int beta = (kb >> 4) & 7;
  int x2[3];
  for (int d = 0; d < 3; ++d) x2[d] = NI * ((beta >> d) & 1) + L.nu[d];
  const double* w = wsh + 4 * c.case_coarse;
  const int km = stage_mask(sp, c.case_coarse);
  const int par = c.par_coarse;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    if (x2[d] & 1) { lo[d] = 0; hi[d] = NI; }
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
        const double wx = NI == 4 ? c_lag[x2[0]][kx] : c_lag7[x2[0]][kx];
        const int64_t base = (int64_t)leaf * NN + kx + NP * ky + NP * NP * kz;
        #pragma unroll
        for (int f = 0; f < F; ++f) tx[f] = fma(wx, yval<KF32, NN>(sp, w, km, par, f * fs + base, c.dt), tx[f]);
      }
      const double wy = NI == 4 ? c_lag[x2[1]][ky] : c_lag7[x2[1]][ky];
      #pragma unroll
      for (int f = 0; f < F; ++f) ty[f] = fma(wy, tx[f], ty[f]);
    }
    const double wz = NI == 4 ? c_lag[x2[2]][kz] : c_lag7[x2[2]][kz];
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

// ------------------------------------------------------------------ non-linear wave
// The non-linear wave of Sec. 4.2 (eqs. lsm, chi, phi), fields (chi, phi):
//   dchi/dt = phi + KO(chi),  dphi/dt = Lap chi - c sin(2 chi) / r^2 + KO(phi),
// r = |x|; with c != 0 the node r = 0 holds the source's regularity condition
// chi = 0 (a regular solution behaves like chi ~ a(t) r there): its state does
// not change.  On a bounded domain a grid
// point d grid steps from the nearest face along an axis uses the widest centred
// stencil that fits there (sixth order for d >= 3, fourth for d = 2, second for
// d = 1) and Kreiss-Oliger only along axes with d >= 3; a point on a face takes
// the radiative condition of Sec. 4.2, df/dt = -(x . grad f) / r - k f / r
// (k = 1 for chi, 2 for phi, asymptotic value 0), with one-sided fourth-order
// first differences along the axes where it sits on a face.
#define D2C4_1 (4.0 / 3.0)
#define D2C4_2 (-1.0 / 12.0)
#define D2C4_0 (-5.0 / 2.0)
#define D1C4_1 (2.0 / 3.0)
#define D1C4_2 (-1.0 / 12.0)

// Per axis: grid steps to the nearest face (large on a periodic domain) and the
// face a point on it lies on (+1 low, -1 high, 0 none).
__device__ __forceinline__ void face_distance(const Geom& g, const int X[3], int d[3], int side[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (g.periodic) {
      d[a] = 1 << 20;
      side[a] = 0;
    } else {
      d[a] = min(X[a], g.Nu - X[a]) / g.w;
      side[a] = X[a] == 0 ? 1 : (X[a] == g.Nu ? -1 : 0);
    }
  }
}

// First difference (times h) along axis ax at distance d from the nearest face
// (side: which face when d = 0).
template <typename At>
__device__ __forceinline__ double d1_bounded(const At& at, int f, int ax, int d, int side) {
  if (d == 0) {
    // one-sided, fourth order: (-25/12, 4, -3, 4/3, -1/4) into the domain
    const double s = (double)side;
    return s * ((-25.0 / 12.0) * at(f, ax, 0) + 4.0 * at(f, ax, side) + (-3.0) * at(f, ax, 2 * side) +
                (4.0 / 3.0) * at(f, ax, 3 * side) + (-0.25) * at(f, ax, 4 * side));
  }
  if (d == 1) return 0.5 * (at(f, ax, 1) - at(f, ax, -1));
  if (d == 2) return D1C4_1 * (at(f, ax, 1) - at(f, ax, -1)) + D1C4_2 * (at(f, ax, 2) - at(f, ax, -2));
  return D1C1 * (at(f, ax, 1) - at(f, ax, -1)) + D1C2 * (at(f, ax, 2) - at(f, ax, -2)) +
         D1C3 * (at(f, ax, 3) - at(f, ax, -3));
}

// The non-linear wave's RHS at a block grid point with node-unit coordinates X.
template <typename At>
__device__ __forceinline__ void rhs_nl_at(const At& at, double h, double sigma, const Geom& g, const int X[3],
                                          double out[2]) {
  int d[3], side[3];
  face_distance(g, X, d, side);
  double x[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = -1.0 + 2.0 * (double)X[a] / (double)g.Nu;
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  if (d[0] == 0 || d[1] == 0 || d[2] == 0) {
    // on a face: the radiative condition
    const double r = sqrt(r2);
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      double xg = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) xg += x[a] * (d1_bounded(at, f, a, d[a], side[a]) / h);
      out[f] = -xg / r - (f == 0 ? 1.0 : 2.0) * at(f, 0, 0) / r;
    }
    return;
  }
  double lap = 0.0, kc = 0.0, kp = 0.0;
#pragma unroll 1
  for (int a = 0; a < 3; ++a) {
    const double c0 = at(0, a, 0);
    if (d[a] >= 3) {
      const double s1 = at(0, a, -1) + at(0, a, 1), s2 = at(0, a, -2) + at(0, a, 2), s3 = at(0, a, -3) + at(0, a, 3);
      lap += D2C3 * s3 + D2C2 * s2 + D2C1 * s1 + D2C0 * c0;
      kc += s3 - 6.0 * s2 + 15.0 * s1 - 20.0 * c0;
      const double q1 = at(1, a, -1) + at(1, a, 1), q2 = at(1, a, -2) + at(1, a, 2), q3 = at(1, a, -3) + at(1, a, 3);
      kp += q3 - 6.0 * q2 + 15.0 * q1 - 20.0 * at(1, a, 0);
    } else if (d[a] == 2) {
      lap += D2C4_2 * (at(0, a, -2) + at(0, a, 2)) + D2C4_1 * (at(0, a, -1) + at(0, a, 1)) + D2C4_0 * c0;
    } else {
      lap += (at(0, a, -1) + at(0, a, 1)) - 2.0 * c0;
    }
  }
  const double chi = at(0, 0, 0);
  const double lapn = lap / (h * h);
  const double src = r2 > 0.0 ? sin(2.0 * chi) / r2 : 0.0;
  const double kos = sigma / (64.0 * h);
  out[0] = at(1, 0, 0) + kos * kc;
  out[1] = lapn - g.c_nl * src + kos * kp;
  if (g.c_nl != 0.0 && r2 == 0.0) {   // the regularity condition chi = 0 at r = 0
    out[0] = 0.0;
    out[1] = 0.0;
  }
}

// Geometry of the block (or tile) whose grid starts at leaf `first`.
__device__ __forceinline__ Geom geom_of(const StageParams& sp, int first, int level) {
  Geom g;
#pragma unroll
  for (int a = 0; a < 3; ++a) g.X0[a] = 4 * sp.leafxyz[4 * first + a];
  g.w = 1 << (sp.L - level);
  g.Nu = 4 << sp.L;
  g.periodic = sp.periodic;
  g.c_nl = sp.nl_coeff;
  return g;
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

// Workgroups of a tile launch: min(tiles, cap), a multiple of the 8 XCDs.
inline int fused_grid(int ntiles, int max_wg) {
  int g = std::min(ntiles, max_wg);
  g = (g + 7) & ~7;
  return std::max(g, 8);
}

}  // namespace lts
