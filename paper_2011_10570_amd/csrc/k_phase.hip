// Phase-by-phase kernels (unzip, rhs, zip, RK update as separate launches over
// whole blocks through HBM), state gather, counters, norms and the copy probe.
// The phase kernels take NI, the node intervals per octant side (4 for 5^3
// nodes, 6 for 7^3 nodes), as a template argument.
#include "dev_common.h"

namespace lts {

// ------------------------------------------------------------------ standalone kernels
// TAB: coarser ghosts read from the ghost table scr (entry of a leaf: gid[leaf],
// filled by the ghost pre-pass of the same stage) instead of interpolated here
// from the coarser leaf's stage values; both give bitwise the same value.
template <bool KF32, int F, int NI, bool TAB>
__global__ __launch_bounds__(256) void k_unzip(StageParams sp, const int32_t* __restrict__ tiles,
                                               const int32_t* __restrict__ slots, const int32_t* __restrict__ list,
                                               const int64_t* __restrict__ off, int64_t total, double* out,
                                               const double* __restrict__ scr, const int32_t* __restrict__ gid) {
  constexpr int GW = 2 * NI + 1, GE = GW * GW * GW;
  __shared__ double wsh[16];
  if (threadIdx.x < 16) wsh[threadIdx.x] = stage_weight(sp, threadIdx.x);
  __syncthreads();
  const int bi = blockIdx.y;
  const int b = list[bi];
  const int32_t* t = tiles + 8 * (int64_t)b;
  const int n4 = (int)(*sp.step & 3);
  const TileCtx c = tile_ctx<NI>(t, sp, n4);
  const int P = NI * c.m + 7;
  const int P3 = P * P * P;
  const int32_t* sl = slots + 2 * (int64_t)t[TI_SLOT];
  for (int pi = blockIdx.x * blockDim.x + threadIdx.x; pi < P3; pi += gridDim.x * blockDim.x) {
    const int qx = pi % P, qy = (pi / P) % P, qz = pi / (P * P);
    double v[F];
    bool done = false;
    if constexpr (TAB) {
      const Loc Lc = locate(qx, qy, qz, c.ox, c.oy, c.oz, c.tt, c.m, NI);
      const int kb = sl[2 * Lc.slot + 1];
      if ((kb & 15) == SRC_COARSE) {
        const int beta = (kb >> 4) & 7;
        const int g = gid[sl[2 * Lc.slot]];
        const int x2 = NI * (beta & 1) + Lc.nu[0], y2 = NI * ((beta >> 1) & 1) + Lc.nu[1],
                  z2 = NI * ((beta >> 2) & 1) + Lc.nu[2];
        #pragma unroll
        for (int f = 0; f < F; ++f) v[f] = scr[((int64_t)g * F + f) * GE + (z2 * GW + y2) * GW + x2];
        done = true;
      }
    }
    if (!done) point_values<KF32, F, NI>(sp, c, sl, wsh, qx, qy, qz, v);
    #pragma unroll
    for (int f = 0; f < F; ++f) out[f * total + off[bi] + pi] = v[f];
  }
}

template <int EQ, int F, bool F32, int NI>
__global__ __launch_bounds__(256) void k_rhs(const int32_t* __restrict__ tiles, const int32_t* __restrict__ list,
                                             const int64_t* __restrict__ poff, int64_t ptotal,
                                             const int64_t* __restrict__ goff, int64_t gtotal,
                                             const double* __restrict__ padded, void* kout, double sigma,
                                             StageParams geo) {
  const int bi = blockIdx.y;
  const int32_t* t = tiles + 8 * (int64_t)list[bi];
  const int m = t[TI_M];
  const int P = NI * m + 7, G = NI * m + 1;
  const int G3 = G * G * G;
  const double h = h_level<NI>(t[TI_LEVEL]);
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
    } else if constexpr (EQ == LTS_EQ_NLWAVE) {
      const Geom g = geom_of(geo, t[TI_FIRST], t[TI_LEVEL]);
      const int Xp[3] = {g.X0[0] + g.w * gx, g.X0[1] + g.w * gy, g.X0[2] + g.w * gz};
      rhs_nl_at(StridedAt<double>{padded + poff[bi], ptotal, ci, P, P * P}, h, sigma, g, Xp, k);
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

template <typename T, int NI>
__global__ __launch_bounds__(256) void k_zip(const int32_t* __restrict__ tiles, const int32_t* __restrict__ list,
                                             const int64_t* __restrict__ goff, int64_t gtotal, int F, int64_t N,
                                             const T* __restrict__ kblock, T* __restrict__ kout) {
  constexpr int NP = NI + 1, NN = NP * NP * NP;
  const int bi = blockIdx.y;
  const int32_t* t = tiles + 8 * (int64_t)list[bi];
  const int m = t[TI_M];
  const int G = NI * m + 1;
  const int first = t[TI_FIRST];
  const int nn = m * m * m * NN;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) {
    const int o = e / NN, node = e % NN;
    // octant o of the block in Morton order -> lexicographic octant coordinates
    int ox = 0, oy = 0, oz = 0;
    for (int bit = 0; bit < 3; ++bit) {
      ox |= ((o >> (3 * bit)) & 1) << bit;
      oy |= ((o >> (3 * bit + 1)) & 1) << bit;
      oz |= ((o >> (3 * bit + 2)) & 1) << bit;
    }
    const int gx = NI * ox + node % NP, gy = NI * oy + (node / NP) % NP, gz = NI * oz + node / (NP * NP);
    const int64_t gi = ((int64_t)gz * G + gy) * G + gx;
    for (int f = 0; f < F; ++f) kout[(f * N + first + o) * NN + node] = kblock[f * gtotal + goff[bi] + gi];
  }
}

template <bool KF32, int NI>
__global__ __launch_bounds__(256) void k_rk(StageParams sp, const int32_t* __restrict__ tiles,
                                            const int32_t* __restrict__ list, const double* __restrict__ coef,
                                            double* out) {
  constexpr int NN = (NI + 1) * (NI + 1) * (NI + 1);
  const int bi = blockIdx.y;
  const int32_t* t = tiles + 8 * (int64_t)list[bi];
  const int n4 = (int)(*sp.step & 3);
  const TileCtx c = tile_ctx<NI>(t, sp, n4);
  const int first = t[TI_FIRST];
  const int nn = c.m * c.m * c.m * NN;
  const int64_t fs = sp.N * NN, ps = fs * sp.F;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)first * NN + e;
    for (int f = 0; f < sp.F; ++f) {
      double acc = 0.0;
      for (int i = 0; i < sp.p; ++i) acc = fma(coef[i], kload<KF32>(sp.K, i * ps + f * fs + idx), acc);
      const double v = sp.U[c.par_same * ps + f * fs + idx] + c.dt * acc;
      if (out) out[f * fs + idx] = v;
      else sp.Uw[(c.par_same ^ 1) * ps + f * fs + idx] = v;
      if (!out && sp.nonfinite && !isfinite(v)) atomicAdd(sp.nonfinite, 1u);
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
  const int NN = (sp.ni + 1) * (sp.ni + 1) * (sp.ni + 1);
  const int64_t fs = sp.N * NN, ps = fs * sp.F;
  const int nn = m * m * m * NN;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)first * NN + e;
    for (int f = 0; f < sp.F; ++f) out[f * fs + idx] = sp.U[par * ps + f * fs + idx];
  }
}

// restore: the state of every octant into the buffer block b reads after a whole
// number of coarse steps (inverse of k_current)
__global__ __launch_bounds__(256) void k_restore(StageParams sp, const int32_t* __restrict__ tiles, int nblocks,
                                                 const double* __restrict__ in) {
  const int b = blockIdx.y;
  if (b >= nblocks) return;
  const int32_t* t = tiles + 8 * (int64_t)b;
  const int lev = t[TI_LEVEL];
  const int m = t[TI_M];
  const int first = t[TI_FIRST];
  const int64_t n = *sp.step;
  const int64_t steps = sp.mode == LTS_MODE_GTS ? (n << (sp.lmax - sp.lmin)) : (n << (lev - sp.lmin));
  const int par = (int)(steps & 1);
  const int NN = (sp.ni + 1) * (sp.ni + 1) * (sp.ni + 1);
  const int64_t fs = sp.N * NN, ps = fs * sp.F;
  const int nn = m * m * m * NN;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)first * NN + e;
    for (int f = 0; f < sp.F; ++f) sp.Uw[par * ps + f * fs + idx] = in[f * fs + idx];
  }
}

// ------------------------------------------------------------------ remeshing
// Wavelet indicator of one octant's node values v[f][125] (Sec. 3.2.2: the
// failure to be interpolated from the coarser level): max over fields and the
// nodes off the every-second-node grid of |v - I2 v|, I2 the tensor degree-2
// Lagrange interpolant of the 27 nodes at positions 0, 2, 4.
__device__ __forceinline__ double i2_weight(int pos, int e) {
  // degree-2 weights from nodes 0, 2, 4 at positions 0..4 (exact binary fractions)
  constexpr double w[5][3] = {{1, 0, 0}, {0.375, 0.75, -0.125}, {0, 1, 0}, {-0.125, 0.75, 0.375}, {0, 0, 1}};
  return w[pos][e];
}

template <typename Get>
__device__ __forceinline__ double wavelet_of(const Get& get, int F) {
  double mx = 0.0;
  for (int f = 0; f < F; ++f)
    for (int n = 0; n < 125; ++n) {
      const int i = n % 5, j = (n / 5) % 5, k = n / 25;
      if (!((i | j | k) & 1)) continue;
      double t = 0.0;
      for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
          for (int a = 0; a < 3; ++a)
            t += i2_weight(k, c) * i2_weight(j, b) * i2_weight(i, a) * get(f, 2 * a + 10 * b + 50 * c);
      mx = fmax(mx, fabs(get(f, n) - t));
    }
  return mx;
}

__global__ __launch_bounds__(256) void k_wavelet_leaf(const double* __restrict__ st, int F, int64_t N,
                                                      double* __restrict__ out) {
  const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (o >= N) return;
  out[o] = wavelet_of([&](int f, int n) { return st[((int64_t)f * N + o) * 125 + n]; }, F);
}

// the same at the parent of the family whose 8 leaves start at fam[q]: node i of
// the parent is node 2 (i - 2c) of child c = min(i >> 1, 1) per axis
__global__ __launch_bounds__(256) void k_wavelet_family(const double* __restrict__ st, int F, int64_t N,
                                                        const int64_t* __restrict__ fam, int64_t nfam,
                                                        double* __restrict__ out) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nfam) return;
  const int64_t first = fam[q];
  out[q] = wavelet_of(
      [&](int f, int n) {
        const int i = n % 5, j = (n / 5) % 5, k = n / 25;
        const int cx = min(i >> 1, 1), cy = min(j >> 1, 1), cz = min(k >> 1, 1);
        const int64_t leaf = first + cx + 2 * cy + 4 * cz;
        const int node = 2 * (i - 2 * cx) + 10 * (j - 2 * cy) + 50 * (k - 2 * cz);
        return st[((int64_t)f * N + leaf) * 125 + node];
      },
      F);
}

// Intergrid transfer (remeshing): new leaf q takes, per record rec[q] = {old leaf,
// kind, offset x, y, z, shift}: kind 0 -- the old leaf's tensor degree-4 Lagrange
// interpolant at position (offset + i 2^-shift... ) given in old node units as
// (off_d + i) / 2^shift; kind 1 -- the coincident node of child c of the 8 old
// leaves starting at the old leaf (injection).
__global__ __launch_bounds__(128) void k_transfer(const double* __restrict__ st_old, int64_t N_old,
                                                  double* __restrict__ st_new, int64_t N_new, int F,
                                                  const int32_t* __restrict__ rec) {
  const int64_t q = blockIdx.x;
  const int n = threadIdx.x;
  if (q >= N_new || n >= 125) return;
  const int32_t* r = rec + 6 * q;
  const int64_t o = r[0];
  const int i = n % 5, j = (n / 5) % 5, k = n / 25;
  if (r[1] == 1) {
    const int cx = min(i >> 1, 1), cy = min(j >> 1, 1), cz = min(k >> 1, 1);
    const int64_t leaf = o + cx + 2 * cy + 4 * cz;
    const int node = 2 * (i - 2 * cx) + 10 * (j - 2 * cy) + 50 * (k - 2 * cz);
    for (int f = 0; f < F; ++f) st_new[((int64_t)f * N_new + q) * 125 + n] = st_old[((int64_t)f * N_old + leaf) * 125 + node];
    return;
  }
  // position of this node in the old leaf's node units, per axis
  const double sc = ldexp(1.0, -r[5]);
  const double xi[3] = {(r[2] + i) * sc, (r[3] + j) * sc, (r[4] + k) * sc};
  double w[3][5];
  for (int d = 0; d < 3; ++d)
    for (int a = 0; a < 5; ++a) {
      double num = 1.0, den = 1.0;
      for (int m = 0; m < 5; ++m)
        if (m != a) {
          num *= xi[d] - m;
          den *= (double)(a - m);
        }
      w[d][a] = num / den;
    }
  for (int f = 0; f < F; ++f) {
    const double* v = st_old + ((int64_t)f * N_old + o) * 125;
    double t = 0.0;
    for (int c = 0; c < 5; ++c) {
      double ty = 0.0;
      for (int b = 0; b < 5; ++b) {
        double tx = 0.0;
        for (int a = 0; a < 5; ++a) tx = fma(w[0][a], v[a + 5 * b + 25 * c], tx);
        ty = fma(w[1][b], tx, ty);
      }
      t = fma(w[2][c], ty, t);
    }
    st_new[((int64_t)f * N_new + q) * 125 + n] = t;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_poison(const int32_t* __restrict__ tiles, const int32_t* __restrict__ list,
                                                T* Ks, int F, int64_t N, int nn) {
  const int i = blockIdx.x;
  const int32_t* t = tiles + 8 * (int64_t)(list ? list[i] : i);
  const int first = t[TI_FIRST], tt = t[TI_TT];
  const int cnt = tt * tt * tt * nn;
  const T nan = (T)__builtin_nan("");
  for (int f = 0; f < F; ++f)
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) Ks[((int64_t)f * N + first) * nn + e] = nan;
}

hipError_t launch_poison(const int32_t* tiles, const int32_t* list, int n, void* Ks, bool kf32, int F, int64_t N,
                         int nn, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (kf32) hipLaunchKernelGGL((k_poison<float>), dim3(n), dim3(256), 0, s, tiles, list, (float*)Ks, F, N, nn);
  else hipLaunchKernelGGL((k_poison<double>), dim3(n), dim3(256), 0, s, tiles, list, (double*)Ks, F, N, nn);
  return hipGetLastError();
}

__global__ void k_set_u32(unsigned int* p, unsigned int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_increment(int64_t* ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] += 1;
}

// per-octant partial sums for the norms: [F][N] sum e^2, [F][N] max |e|, nonfinite count
__global__ __launch_bounds__(128) void k_norm_partials(const double* a, const double* b, int F, int64_t N, int nn,
                                                       double* sq, double* mx, unsigned long long* bad) {
  const int64_t o = blockIdx.x;
  const int f = blockIdx.y;
  __shared__ double s1[128], s2[128];
  __shared__ int s3[128];
  double q = 0.0, m = 0.0;
  int nb = 0;
  for (int node = threadIdx.x; node < nn; node += 128) {
    const int64_t idx = ((int64_t)f * N + o) * nn + node;
    const double x = a[idx];
    const double e = b ? x - b[idx] : x;
    if (!isfinite(x)) nb += 1;
    q += e * e;
    m = fmax(m, fabs(e));
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

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_set_i64(int64_t* ptr, int64_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, ptr, value);
  return hipGetLastError();
}

template <int NI, bool TAB>
static void unzip_ni(bool kf32, const StageParams& sp, dim3 grid, const int32_t* tiles, const int32_t* slots,
                     const int32_t* list, const int64_t* off, int64_t total, double* out, const double* scr,
                     const int32_t* gid, hipStream_t s) {
  if (sp.F == 2) {
    if (kf32) hipLaunchKernelGGL((k_unzip<true, 2, NI, TAB>), grid, dim3(256), 0, s, sp, tiles, slots, list, off, total,
                                 out, scr, gid);
    else hipLaunchKernelGGL((k_unzip<false, 2, NI, TAB>), grid, dim3(256), 0, s, sp, tiles, slots, list, off, total,
                            out, scr, gid);
  } else {
    if (kf32) hipLaunchKernelGGL((k_unzip<true, 6, NI, TAB>), grid, dim3(256), 0, s, sp, tiles, slots, list, off, total,
                                 out, scr, gid);
    else hipLaunchKernelGGL((k_unzip<false, 6, NI, TAB>), grid, dim3(256), 0, s, sp, tiles, slots, list, off, total,
                            out, scr, gid);
  }
}

hipError_t launch_unzip(bool kf32, const StageParams& sp, const int32_t* tiles, const int32_t* slots,
                        const int32_t* list, const int64_t* off, int nb, int64_t total, double* out,
                        const int32_t* ghosts, int64_t nghost, double* scr, const int32_t* gid, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if ((sp.F != 2 && sp.F != 6) || (sp.ni != 4 && sp.ni != 6)) return hipErrorInvalidValue;
  // the ghost table is built for every 5-node case and for two fields of 7-node
  // octants (six fields of 13^3 points would exceed a workgroup's LDS)
  const bool tab = sp.ni == 4 || sp.F == 2;
  if (tab && nghost > 0) {
    if (!scr || !gid || !ghosts) return hipErrorInvalidValue;
    hipError_t e = launch_ghost_pre(sp.F, kf32, sp, ghosts, nghost, scr, s);
    if (e != hipSuccess) return e;
  }
  dim3 grid(8, nb);
  if (sp.ni == 4) unzip_ni<4, true>(kf32, sp, grid, tiles, slots, list, off, total, out, scr, gid, s);
  else if (tab) unzip_ni<6, true>(kf32, sp, grid, tiles, slots, list, off, total, out, scr, gid, s);
  else unzip_ni<6, false>(kf32, sp, grid, tiles, slots, list, off, total, out, scr, gid, s);
  return hipGetLastError();
}

template <int NI>
static hipError_t rhs_ni(int eq, bool f32, dim3 grid, const int32_t* tiles, const int32_t* list, const int64_t* poff,
                         int64_t ptotal, const int64_t* goff, int64_t gtotal, const double* padded, void* kout,
                         double sigma, const StageParams& geo, hipStream_t s) {
  if (eq == LTS_EQ_NLWAVE) {
    if (f32 || NI != 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_rhs<LTS_EQ_NLWAVE, 2, false, NI>), grid, dim3(256), 0, s, tiles, list, poff, ptotal, goff,
                       gtotal, padded, kout, sigma, geo);
  } else if (eq == LTS_EQ_WAVE) {
    if (f32) hipLaunchKernelGGL((k_rhs<LTS_EQ_WAVE, 2, true, NI>), grid, dim3(256), 0, s, tiles, list, poff, ptotal,
                                goff, gtotal, padded, kout, sigma, geo);
    else hipLaunchKernelGGL((k_rhs<LTS_EQ_WAVE, 2, false, NI>), grid, dim3(256), 0, s, tiles, list, poff, ptotal,
                            goff, gtotal, padded, kout, sigma, geo);
  } else {
    if (f32) hipLaunchKernelGGL((k_rhs<LTS_EQ_MAXWELL, 6, true, NI>), grid, dim3(256), 0, s, tiles, list, poff,
                                ptotal, goff, gtotal, padded, kout, sigma, geo);
    else hipLaunchKernelGGL((k_rhs<LTS_EQ_MAXWELL, 6, false, NI>), grid, dim3(256), 0, s, tiles, list, poff,
                            ptotal, goff, gtotal, padded, kout, sigma, geo);
  }
  return hipGetLastError();
}

hipError_t launch_rhs(int eq, bool f32, const int32_t* tiles, const int32_t* list, const int64_t* poff,
                      int64_t ptotal, const int64_t* goff, int64_t gtotal, int nb, const double* padded, void* kout,
                      double sigma, const StageParams& geo, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  dim3 grid(8, nb);
  if (geo.ni == 4) return rhs_ni<4>(eq, f32, grid, tiles, list, poff, ptotal, goff, gtotal, padded, kout, sigma, geo, s);
  if (geo.ni == 6) return rhs_ni<6>(eq, f32, grid, tiles, list, poff, ptotal, goff, gtotal, padded, kout, sigma, geo, s);
  return hipErrorInvalidValue;
}

template <int NI>
static void zip_ni(bool f32, dim3 grid, const int32_t* tiles, const int32_t* list, const int64_t* goff,
                   int64_t gtotal, int F, int64_t N, const void* kblock, void* kout, hipStream_t s) {
  if (f32) hipLaunchKernelGGL((k_zip<float, NI>), grid, dim3(256), 0, s, tiles, list, goff, gtotal, F, N,
                              (const float*)kblock, (float*)kout);
  else hipLaunchKernelGGL((k_zip<double, NI>), grid, dim3(256), 0, s, tiles, list, goff, gtotal, F, N,
                          (const double*)kblock, (double*)kout);
}

hipError_t launch_zip(bool f32, int ni, const int32_t* tiles, const int32_t* list, const int64_t* goff, int64_t gtotal,
                      int nb, int F, int64_t N, const void* kblock, void* kout, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  dim3 grid(8, nb);
  if (ni == 4) zip_ni<4>(f32, grid, tiles, list, goff, gtotal, F, N, kblock, kout, s);
  else if (ni == 6) zip_ni<6>(f32, grid, tiles, list, goff, gtotal, F, N, kblock, kout, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_rk(bool kf32, const StageParams& sp, const int32_t* tiles, const int32_t* list, int nb,
                     const double* coef, double* out, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  dim3 grid(4, nb);
  if (sp.ni == 4) {
    if (kf32) hipLaunchKernelGGL((k_rk<true, 4>), grid, dim3(256), 0, s, sp, tiles, list, coef, out);
    else hipLaunchKernelGGL((k_rk<false, 4>), grid, dim3(256), 0, s, sp, tiles, list, coef, out);
  } else if (sp.ni == 6) {
    if (kf32) hipLaunchKernelGGL((k_rk<true, 6>), grid, dim3(256), 0, s, sp, tiles, list, coef, out);
    else hipLaunchKernelGGL((k_rk<false, 6>), grid, dim3(256), 0, s, sp, tiles, list, coef, out);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_current(const StageParams& sp, const int32_t* tiles, int nblocks, double* out, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_current, dim3(4, nblocks), dim3(256), 0, s, sp, tiles, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_restore(const StageParams& sp, const int32_t* tiles, int nblocks, const double* in, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_restore, dim3(4, nblocks), dim3(256), 0, s, sp, tiles, nblocks, in);
  return hipGetLastError();
}

hipError_t launch_wavelet(const double* st, int F, int64_t N, const int64_t* fam, int64_t nfam, double* leaf_out,
                          double* fam_out, hipStream_t s) {
  if (N > 0) hipLaunchKernelGGL(k_wavelet_leaf, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, st, F, N, leaf_out);
  if (nfam > 0)
    hipLaunchKernelGGL(k_wavelet_family, dim3((unsigned)((nfam + 255) / 256)), dim3(256), 0, s, st, F, N, fam, nfam,
                       fam_out);
  return hipGetLastError();
}

hipError_t launch_transfer(const double* st_old, int64_t N_old, double* st_new, int64_t N_new, int F,
                           const int32_t* rec, hipStream_t s) {
  if (N_new <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transfer, dim3((unsigned)N_new), dim3(128), 0, s, st_old, N_old, st_new, N_new, F, rec);
  return hipGetLastError();
}

hipError_t launch_set_u32(unsigned int* ptr, unsigned int value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, s, ptr, value);
  return hipGetLastError();
}

hipError_t launch_increment(int64_t* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_increment, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}

hipError_t launch_norm_partials(const double* a, const double* b, int F, int64_t N, int nn, double* sq, double* mx,
                                unsigned long long* bad, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_norm_partials, dim3((unsigned)N, F), dim3(128), 0, s, a, b, F, N, nn, sq, mx, bad);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t nbytes, hipStream_t s) {
  const int64_t n = (int64_t)(nbytes / sizeof(double4));
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(2048), dim3(256), 0, s, (const double4*)src, (double4*)dst, n);
  return hipGetLastError();
}

}  // namespace lts
