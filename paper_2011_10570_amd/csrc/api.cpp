// C ABI of the library (include/lts.h): argument checking, device tables, the
// phase-by-phase path, the fused stage and the LTS / GTS drivers (Alg. 1 / 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lts_impl.h"
#include "lts_kernels.h"

namespace lts {

static thread_local std::string g_err;

lts_status fail(lts_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
void clear_error() { g_err.clear(); }

static lts_status hip_fail(hipError_t e, const char* where) {
  return fail(LTS_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                   \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

static void free_set(TileSet& ts) {
  for (int32_t** p : {&ts.d_tiles, &ts.d_slots}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
}

static lts_status upload_vec(const std::vector<int32_t>& v, int32_t** d, const char* what) {
  if (v.empty()) return LTS_OK;
  HIP_TRY(hipMalloc(d, v.size() * 4), what);
  HIP_TRY(hipMemcpy(*d, v.data(), v.size() * 4, hipMemcpyHostToDevice), what);
  return LTS_OK;
}

static lts_status upload_set(TileSet& ts) {
  free_set(ts);
  if (ts.tiles.empty()) return LTS_OK;
  lts_status st;
  if ((st = upload_vec(ts.tiles, &ts.d_tiles, "upload tiles")) != LTS_OK) return st;
  return upload_vec(ts.slots, &ts.d_slots, "upload slots");
}

// tile sets of the fused kernels and the ghost table (rebuilt together)
static lts_status upload_fused_sets(Mesh& m) {
  lts_status st;
  for (int k : {1, 2, 4})
    if ((st = upload_set(m.ts[k])) != LTS_OK) return st;
  if (m.d_ghosts) (void)hipFree(m.d_ghosts);
  m.d_ghosts = nullptr;
  if (m.d_ghost_of_leaf) (void)hipFree(m.d_ghost_of_leaf);
  m.d_ghost_of_leaf = nullptr;
  if ((st = upload_vec(m.ghost_of_leaf, &m.d_ghost_of_leaf, "upload ghost entries of leaves")) != LTS_OK) return st;
  return upload_vec(m.ghosts, &m.d_ghosts, "upload ghost table");
}

static lts_status ensure_device(Mesh& m) {
  if (m.uploaded) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != m.device) return fail(LTS_EINVAL, "mesh tables were uploaded to another device");
    return LTS_OK;
  }
  HIP_TRY(hipGetDevice(&m.device), "hipGetDevice");
  lts_status st;
  if ((st = upload_set(m.bt)) != LTS_OK) return st;
  if ((st = upload_fused_sets(m)) != LTS_OK) return st;
  std::vector<int32_t> xyz(4 * (size_t)m.n());
  for (int64_t i = 0; i < m.n(); ++i) {
    xyz[4 * i] = m.ax[i]; xyz[4 * i + 1] = m.ay[i]; xyz[4 * i + 2] = m.az[i]; xyz[4 * i + 3] = m.lev[i];
  }
  if ((st = upload_vec(xyz, &m.d_leafxyz, "upload leaf anchors")) != LTS_OK) return st;
  if ((st = upload_vec(m.fine8, &m.d_fine8, "upload fine table")) != LTS_OK) return st;
  m.uploaded = true;
  return LTS_OK;
}

// device copy of a block list with its padded / grid offsets (phase-by-phase path)
struct ListDev {
  int nb = 0;
  int64_t ptotal = 0, gtotal = 0;
  const int32_t* list = nullptr;
  const int64_t* poff = nullptr;
  const int64_t* goff = nullptr;
};

static lts_status stage_list(Mesh& m, const int32_t* blocks, int nb, const lts_position* pos, hipStream_t s,
                             ListDev& out) {
  std::vector<int32_t> lst;
  if (blocks) {
    if (nb < 0) return fail(LTS_EINVAL, "nb < 0");
    for (int i = 0; i < nb; ++i) {
      if (blocks[i] < 0 || blocks[i] >= (int)m.blocks.size()) return fail(LTS_EINVAL, "block index out of range");
      lst.push_back(blocks[i]);
    }
  } else {
    if (!pos) return fail(LTS_EINVAL, "blocks == NULL needs a position");
    const int j = pos->substep;
    for (size_t b = 0; b < m.blocks.size(); ++b) {
      const int r = 1 << (m.lmax - m.blocks[b].level);
      if (pos->mode == LTS_MODE_GTS || j % r == 0) lst.push_back((int32_t)b);
    }
  }
  out.nb = (int)lst.size();
  const size_t n = lst.size();
  std::vector<int64_t> pack(3 * n + 1, 0);
  int64_t p = 0, g = 0;
  const int ni = m.ni();
  for (size_t i = 0; i < n; ++i) {
    const int mm = m.blocks[lst[i]].m;
    pack[n + i] = p;
    pack[2 * n + i] = g;
    p += (int64_t)(ni * mm + 7) * (ni * mm + 7) * (ni * mm + 7);
    g += (int64_t)(ni * mm + 1) * (ni * mm + 1) * (ni * mm + 1);
  }
  for (size_t i = 0; i < n; ++i) pack[i] = lst[i];
  out.ptotal = p;
  out.gtotal = g;
  const size_t bytes = pack.size() * 8;
  if (bytes > m.list_cap) {
    if (m.d_off) (void)hipFree(m.d_off);
    m.d_off = nullptr;
    m.list_cap = 0;
    HIP_TRY(hipMalloc(&m.d_off, bytes), "hipMalloc list");
    m.list_cap = bytes;
  }
  // list entries are stored as int64 in the pack; kernels read int32: convert
  std::vector<int32_t> l32(lst);
  std::vector<char> buf(bytes);
  std::memcpy(buf.data(), l32.data(), n * 4);
  std::memcpy(buf.data() + n * 8, pack.data() + n, 2 * n * 8);
  HIP_TRY(hipMemcpyAsync(m.d_off, buf.data(), bytes, hipMemcpyHostToDevice, s), "upload list");
  HIP_TRY(hipStreamSynchronize(s), "sync list upload");
  out.list = (const int32_t*)m.d_off;
  out.poff = m.d_off + n;
  out.goff = m.d_off + 2 * n;
  return LTS_OK;
}

static void set_kmask(StageParams& sp) {
  for (int c = 0; c < 4; ++c) {
    sp.kmask[c] = 0;
    for (int i = 0; i < sp.p; ++i)
      if (sp.w[c][i] != 0.0) sp.kmask[c] |= 1 << i;
  }
}

static lts_status check_view(const Mesh& m, const lts_stage_view* v, int& p) {
  if (!v || !v->U || !v->K) return fail(LTS_EINVAL, "stage view needs U and K");
  if (v->nfields != 2 && v->nfields != 6) return fail(LTS_EINVAL, "nfields must be 2 or 6");
  if (v->precision != LTS_FP64 && v->precision != LTS_FP32_RHS) return fail(LTS_EINVAL, "bad precision");
  p = tableau_stages(v->tableau);
  if (!p) return fail(LTS_EINVAL, "bad tableau");
  (void)m;
  return LTS_OK;
}

static lts_status fill_params(const Mesh& m, const lts_stage_view* v, int stage, const lts_position* pos,
                              const int64_t* d_step, StageParams& sp) {
  int p = 0;
  lts_status st = check_view(m, v, p);
  if (st != LTS_OK) return st;
  if (!pos) return fail(LTS_EINVAL, "position is NULL");
  if (stage < 0 || stage >= p) return fail(LTS_EINVAL, "stage out of range");
  if (pos->mode != LTS_MODE_LTS && pos->mode != LTS_MODE_GTS) return fail(LTS_EINVAL, "bad mode");
  if (pos->substep < 0 || pos->substep >= (1 << (m.lmax - m.lmin))) return fail(LTS_EINVAL, "substep out of range");
  if ((int64_t)p * v->nfields * m.n() * m.nn() >= (1ll << 31) || m.n() * m.nn() * 8 >= (1ll << 32))
    return fail(LTS_EUNSUPPORTED, "arrays too large for the kernels' 32-bit offsets");
  double w[64], a[16], b[4];
  coefficient_tables(v->tableau, w, a, b);
  std::memset(&sp, 0, sizeof(sp));
  sp.U = (const double*)v->U;
  sp.Uw = (double*)v->U;
  sp.K = v->K;
  sp.Kw = v->K;
  sp.N = m.n();
  sp.F = v->nfields;
  sp.p = p;
  sp.stage = stage;
  sp.mode = pos->mode;
  sp.j = pos->substep;
  sp.lmin = m.lmin;
  sp.lmax = m.lmax;
  sp.step = d_step;
  for (int c = 0; c < 4; ++c)
    for (int i = 0; i < p; ++i) sp.w[c][i] = w[(c * p + stage) * p + i];
  for (int i = 0; i < p; ++i) sp.b[i] = b[i];
  set_kmask(sp);
  sp.leafxyz = m.d_leafxyz;
  sp.fine8 = m.d_fine8;
  sp.ni = m.ni();
  sp.L = m.L;
  sp.periodic = m.periodic ? 1 : 0;
  sp.nl_coeff = 1.0;
  return LTS_OK;
}

// Fields of an equation (0: unknown).
static int equation_fields(int eq) {
  return eq == LTS_EQ_WAVE || eq == LTS_EQ_NLWAVE ? 2 : (eq == LTS_EQ_MAXWELL ? 6 : 0);
}

// Equation / mesh / precision / tile combinations the fused kernels are built for.
static lts_status check_combination(const Mesh& m, int eq, int prec, bool batch) {
  if (m.nodes != 5) {
    if (batch) return fail(LTS_EUNSUPPORTED, "7-node octants are not built for batched launches");
    if (eq != LTS_EQ_WAVE)
      return fail(LTS_EUNSUPPORTED, "the fused stage for 7-node octants is built for the wave equation (other "
                                    "equations run on the phase kernels: lts_advance, lts_advance_unfused)");
    if (m.ts[2].count() + m.ts[4].count() > 0)
      return fail(LTS_EUNSUPPORTED, "the fused stage for 7-node octants needs tile side 1 (lts_mesh_set_tile)");
  }
  if (!m.periodic && eq != LTS_EQ_NLWAVE)
    return fail(LTS_EUNSUPPORTED, "a bounded mesh needs the non-linear wave equation (radiative boundary)");
  if (eq == LTS_EQ_NLWAVE) {
    if (prec != LTS_FP64) return fail(LTS_EUNSUPPORTED, "the non-linear wave runs in FP64");
    if (m.ts[4].count() > 0) return fail(LTS_EUNSUPPORTED, "the non-linear wave needs tile side 1 or 2");
    if (batch) return fail(LTS_EUNSUPPORTED, "the non-linear wave is not built for batched launches");
  }
  if (eq == LTS_EQ_MAXWELL && m.ts[4].count() > 0)
    return fail(LTS_EUNSUPPORTED, "Maxwell fused stage needs tile side 1 or 2 (lts_mesh_set_tile)");
  return LTS_OK;
}

}  // namespace lts

using namespace lts;


// Whether a simulation's coarse steps run on the fused stage kernels (else on the
// phase kernels): every 5-node mesh; 7-node meshes for the wave equation on
// side-1 tiles.
static bool fused_path(const Mesh& m, int eq) {
  return m.nodes == 5 || (eq == LTS_EQ_WAVE && m.ts[2].count() + m.ts[4].count() == 0);
}

static lts_status set_step(int64_t** slot, int64_t value, hipStream_t s) {
  if (!*slot) HIP_TRY(hipMalloc(slot, sizeof(int64_t)), "hipMalloc step");
  // a kernel-argument write keeps the value with the enqueued work (no sync)
  HIP_TRY(launch_set_i64(*slot, value, s), "set step");
  return LTS_OK;
}

struct MeshExtra {
  int64_t* d_step = nullptr;
  double* d_norm = nullptr;
  size_t norm_cap = 0;
  double* d_coef = nullptr;
  double* d_cscr = nullptr;   // ghost table of the single-stage calls (lts_fused_stage, lts_unzip)
  size_t cscr_cap = 0;
};

// Half-node points of one ghost-table entry per field, GW^3 with GW = 2 ni + 1.
static size_t ghost_points(const Mesh& m) {
  const size_t gw = (size_t)(2 * m.ni() + 1);
  return gw * gw * gw;
}

// Doubles of one stage's ghost table: F x GW^3 per entry (GW = 2 ni + 1: 729
// doubles for 5-node octants, 2197 for 7-node octants).
static size_t cscr_slot(const Mesh& m, int F) { return (m.ghosts.size() / 2) * (size_t)F * ghost_points(m); }

// Ghost-table scratch of `slots` stages (lts_advance keeps one per stage of a
// substep, the single-stage calls one).  Grown outside graph capture only.
static lts_status ensure_cscr(const Mesh& m, int F, int slots, double** p, size_t* cap) {
  const size_t need = (size_t)slots * cscr_slot(m, F) * sizeof(double);
  if (need <= *cap) return LTS_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  HIP_TRY(hipMalloc(p, need), "hipMalloc ghost scratch");
  *cap = need;
  return LTS_OK;
}

// Lowest level of the blocks B_j (Alg. 2, fig. blk_loop): all levels at j = 0
// and in GTS, else lmax - ctz(j).
static int lowest_active_level(const Mesh& m, int mode, int j) {
  if (mode == LTS_MODE_GTS || j == 0) return m.lmin;
  int tz = 0;
  while (!(j & 1)) { j >>= 1; ++tz; }
  return m.lmax - tz;
}

// Every fused launch of one stage for the tiles of levels >= lo: the ghost-table
// pre-pass of entries [0, nghost) (receivers of levels >= lo, or the part of them
// that the multi-stage pre-pass has not filled), then streamed side-4 tiles,
// side-2 and side-1 tiles, in stream order.
static lts_status launch_stage(const Mesh& m, int eq, bool kf32, const StageParams& sp, int lo, int64_t nghost,
                               double* cscr, const LaunchShape& ls, hipStream_t s) {
  HIP_TRY(launch_ghost_pre(sp.F, kf32, sp, m.d_ghosts, nghost, cscr, s), "ghost pre-pass");
  for (int tt : {4, 2, 1}) {
    const TileSet& ts = m.ts[tt];
    if (ts.count() == 0 || ts.n_ge[lo] == 0) continue;
    XcdRanges xr;
    for (int x = 0; x < 9; ++x) xr.b[x] = ts.xcd[lo][x];
    if (tt == 4) HIP_TRY(launch_stream(eq, kf32, sp, ts.d_tiles, ts.d_slots, cscr, xr, ls, s), "stream launch");
    else HIP_TRY(launch_fused(tt, eq, kf32, sp, ts.d_tiles, ts.d_slots, cscr, xr, ls, s), "fused launch");
  }
  return LTS_OK;
}

// Extra device buffers live beside the mesh handle.
struct lts_mesh_full : lts_mesh {
  MeshExtra x;
};

extern "C" {

const char* lts_last_error(void) { return g_err.c_str(); }
const char* lts_version(void) { return "lts-mi355x 0.1 (gfx950)"; }

lts_status lts_build_mesh(const lts_mesh_spec* spec, lts_mesh** out) {
  clear_error();
  if (!out) return fail(LTS_EINVAL, "out is NULL");
  *out = nullptr;
  lts_mesh_full* h = new (std::nothrow) lts_mesh_full();
  if (!h) return fail(LTS_ENOMEM, "host allocation");
  lts_status st;
  try {
    st = build_mesh(spec, h->m);
  } catch (const std::bad_alloc&) {
    st = fail(LTS_ENOMEM, "host allocation during mesh build");
  } catch (...) {
    st = fail(LTS_EINVAL, "mesh build failed");
  }
  if (st != LTS_OK) {
    delete h;
    return st;
  }
  *out = h;
  return LTS_OK;
}

void lts_mesh_destroy(lts_mesh* mesh) {
  if (!mesh) return;
  lts_mesh_full* h = static_cast<lts_mesh_full*>(mesh);
  free_set(h->m.bt);
  for (int k : {1, 2, 4}) free_set(h->m.ts[k]);
  if (h->m.d_ghosts) (void)hipFree(h->m.d_ghosts);
  if (h->m.d_ghost_of_leaf) (void)hipFree(h->m.d_ghost_of_leaf);
  if (h->m.d_leafxyz) (void)hipFree(h->m.d_leafxyz);
  if (h->m.d_fine8) (void)hipFree(h->m.d_fine8);
  if (h->x.d_cscr) (void)hipFree(h->x.d_cscr);
  if (h->m.d_off) (void)hipFree(h->m.d_off);
  if (h->x.d_step) (void)hipFree(h->x.d_step);
  if (h->x.d_norm) (void)hipFree(h->x.d_norm);
  if (h->x.d_coef) (void)hipFree(h->x.d_coef);
  delete h;
}

lts_status lts_mesh_query(const lts_mesh* mesh, lts_mesh_info* info) {
  clear_error();
  if (!mesh || !info) return fail(LTS_EINVAL, "NULL argument");
  const Mesh& m = mesh->m;
  std::memset(info, 0, sizeof(*info));
  info->n_oct = m.n();
  info->n_blocks = (int64_t)m.blocks.size();
  info->n_tiles = m.ts[1].count() + m.ts[2].count() + m.ts[4].count();
  info->L = m.L;
  info->lmin = m.lmin;
  info->lmax = m.lmax;
  info->n_substeps = 1 << (m.lmax - m.lmin);
  info->tile = m.tile;
  for (int8_t l : m.lev) info->level_count[l] += 1;
  int64_t up = 0, gp = 0, wl = 0, wg = 0;
  const int64_t nsub = 1ll << (m.lmax - m.lmin);
  const int ni = m.ni();
  for (const Block& b : m.blocks) {
    up += (int64_t)(ni * b.m + 7) * (ni * b.m + 7) * (ni * b.m + 7);
    gp += (int64_t)(ni * b.m + 1) * (ni * b.m + 1) * (ni * b.m + 1);
    const int64_t nodes = m.nn() * b.m * b.m * b.m;
    wl += nodes * (1ll << (b.level - m.lmin));
    wg += nodes * nsub;
  }
  info->unzip_points = up;
  info->grid_points = gp;
  // device tables: tile records and slot tables of the block tiles (phase
  // kernels) and of the fused tiles
  int64_t tb = (int64_t)(m.bt.tiles.size() + m.bt.slots.size());
  for (int k : {1, 2, 4}) tb += (int64_t)(m.ts[k].tiles.size() + m.ts[k].slots.size());
  tb += (int64_t)m.ghosts.size() + (int64_t)m.fine8.size();
  info->table_bytes = 4 * tb;
  info->ghost_entries = (int64_t)(m.ghosts.size() / 2);
  info->boundary = m.periodic ? LTS_BOUNDARY_PERIODIC : LTS_BOUNDARY_OUTER;
  info->nodes = m.nodes;
  info->node_updates_lts = wl;
  info->node_updates_gts = wg;
  // eq. invS with alpha_l = DG nodes at level lmax - l
  double inv = 0.0, tot = 0.0, a0 = 0.0;
  for (int l = m.lmin; l <= m.lmax; ++l) {
    const double al = (double)m.nn() * (double)info->level_count[l];
    inv += al / std::ldexp(1.0, m.lmax - l);
    tot += al;
    if (l == m.lmax) a0 = al;
  }
  info->s_est = tot / inv;
  info->s_max = a0 > 0 ? tot / a0 : 0.0;
  return LTS_OK;
}

lts_status lts_mesh_export(const lts_mesh* mesh, int32_t kind, void* buf, size_t cap, size_t* needed) {
  clear_error();
  if (!mesh) return fail(LTS_EINVAL, "mesh is NULL");
  const Mesh& m = mesh->m;
  std::vector<int32_t> out;
  switch (kind) {
    case LTS_EXPORT_LEAVES:
      out.resize(4 * m.n());
      for (int64_t i = 0; i < m.n(); ++i) {
        out[4 * i] = m.ax[i]; out[4 * i + 1] = m.ay[i]; out[4 * i + 2] = m.az[i]; out[4 * i + 3] = m.lev[i];
      }
      break;
    case LTS_EXPORT_BLOCKS:
      for (const Block& b : m.blocks) {
        const int32_t r[6] = {b.first, b.m, b.level, b.ax, b.ay, b.az};
        out.insert(out.end(), r, r + 6);
      }
      break;
    case LTS_EXPORT_UNZIP_MAP: {
      size_t tot = 0;
      const int ni = m.ni();
      for (const Block& b : m.blocks) tot += (size_t)(ni * b.m + 7) * (ni * b.m + 7) * (ni * b.m + 7);
      out.resize(5 * tot);
      size_t o = 0;
      for (size_t b = 0; b < m.blocks.size(); ++b) {
        const int S = ni * m.blocks[b].m + 7;
        unzip_map_block(m, (int)b, out.data() + 5 * o);
        o += (size_t)S * S * S;
      }
      break;
    }
    case LTS_EXPORT_SCHEDULE: {
      const int nsub = 1 << (m.lmax - m.lmin);
      for (int j = 0; j < nsub; ++j) {
        std::vector<int32_t> act;
        for (size_t b = 0; b < m.blocks.size(); ++b)
          if (j % (1 << (m.lmax - m.blocks[b].level)) == 0) act.push_back((int32_t)b);
        out.push_back((int32_t)act.size());
        out.insert(out.end(), act.begin(), act.end());
      }
      break;
    }
    case LTS_EXPORT_TILES:
      for (int k : {1, 2, 4}) out.insert(out.end(), m.ts[k].tiles.begin(), m.ts[k].tiles.end());
      break;
    case LTS_EXPORT_GHOSTS:
      out = m.ghosts;
      break;
    default:
      return fail(LTS_EINVAL, "unknown export kind");
  }
  const size_t bytes = out.size() * 4;
  if (needed) *needed = bytes;
  if (!buf) return LTS_OK;
  if (cap < bytes) return fail(LTS_EINVAL, "export buffer too small");
  std::memcpy(buf, out.data(), bytes);
  return LTS_OK;
}

lts_status lts_mesh_set_tile(lts_mesh* mesh, int32_t tile) {
  clear_error();
  if (!mesh) return fail(LTS_EINVAL, "mesh is NULL");
  Mesh& m = mesh->m;
  if (tile == m.tile) return LTS_OK;
  if (m.attached > 0) return fail(LTS_EINVAL, "a sim of this mesh is attached to a batch");
  lts_status st = build_tiles(m, tile);
  if (st != LTS_OK) return st;
  m.tables_gen += 1;   // device tile tables move: captured graphs must be redone
  if (m.uploaded && (st = upload_fused_sets(m)) != LTS_OK) return st;
  return LTS_OK;
}

lts_status lts_coefficients(int32_t tableau, double* out, size_t cap) {
  clear_error();
  const int p = tableau_stages(tableau);
  if (!p) return fail(LTS_EINVAL, "bad tableau");
  const size_t n = (size_t)(4 * p * p + p * p + p);
  if (!out || cap < n * sizeof(double)) return fail(LTS_EINVAL, "output too small");
  coefficient_tables(tableau, out, out + 4 * p * p, out + 5 * p * p);
  return LTS_OK;
}

lts_status lts_unzip(lts_mesh* mesh, const lts_stage_view* view, int32_t stage, const lts_position* pos,
                     const int32_t* blocks, int32_t nb, double* padded, void* stream) {
  clear_error();
  if (!mesh || !padded) return fail(LTS_EINVAL, "NULL argument");
  lts_mesh_full* h = static_cast<lts_mesh_full*>(mesh);
  Mesh& m = mesh->m;
  hipStream_t s = (hipStream_t)stream;
  lts_status st = ensure_device(m);
  if (st != LTS_OK) return st;
  if ((st = set_step(&h->x.d_step, pos ? pos->coarse_step : 0, s)) != LTS_OK) return st;
  StageParams sp;
  if ((st = fill_params(m, view, stage, pos, h->x.d_step, sp)) != LTS_OK) return st;
  ListDev L;
  if ((st = stage_list(m, blocks, nb, pos, s, L)) != LTS_OK) return st;
  // coarser ghosts come prolongated from the ghost table: the entries of every
  // receiver level the call can touch (the lowest level of its blocks up)
  int lo = m.lmax;
  if (blocks) {
    for (int i = 0; i < nb; ++i) lo = std::min(lo, (int)m.blocks[blocks[i]].level);
  } else {
    lo = lowest_active_level(m, pos->mode, pos->substep);
  }
  if ((st = ensure_cscr(m, sp.F, 1, &h->x.d_cscr, &h->x.cscr_cap)) != LTS_OK) return st;
  HIP_TRY(launch_unzip(view->precision == LTS_FP32_RHS, sp, m.bt.d_tiles, m.bt.d_slots, L.list, L.poff, L.nb,
                       L.ptotal, padded, m.d_ghosts, m.ghost_ge[lo], h->x.d_cscr, m.d_ghost_of_leaf, s),
          "unzip launch");
  return LTS_OK;
}

lts_status lts_rhs(lts_mesh* mesh, int32_t equation, const lts_rhs_params* params, const double* padded,
                   int32_t precision, const int32_t* blocks, int32_t nb, void* k_block, void* stream) {
  clear_error();
  if (!mesh || !padded || !k_block || !params) return fail(LTS_EINVAL, "NULL argument");
  if (!equation_fields(equation)) return fail(LTS_EINVAL, "bad equation");
  if (precision != LTS_FP64 && precision != LTS_FP32_RHS) return fail(LTS_EINVAL, "bad precision");
  if (!blocks) return fail(LTS_EINVAL, "lts_rhs needs an explicit block list");
  Mesh& m = mesh->m;
  if (!m.periodic && equation != LTS_EQ_NLWAVE)
    return fail(LTS_EUNSUPPORTED, "a bounded mesh needs the non-linear wave equation (radiative boundary)");
  if (equation == LTS_EQ_NLWAVE && precision != LTS_FP64)
    return fail(LTS_EUNSUPPORTED, "the non-linear wave runs in FP64");
  if (equation == LTS_EQ_NLWAVE && m.nodes != 5)
    return fail(LTS_EUNSUPPORTED, "the non-linear wave is built for 5-node octants");
  hipStream_t s = (hipStream_t)stream;
  lts_status st = ensure_device(m);
  if (st != LTS_OK) return st;
  ListDev L;
  if ((st = stage_list(m, blocks, nb, nullptr, s, L)) != LTS_OK) return st;
  StageParams geo;
  std::memset(&geo, 0, sizeof(geo));
  geo.leafxyz = m.d_leafxyz;
  geo.ni = m.ni();
  geo.L = m.L;
  geo.periodic = m.periodic ? 1 : 0;
  geo.nl_coeff = params->nl_coeff;
  HIP_TRY(launch_rhs(equation, precision == LTS_FP32_RHS, m.bt.d_tiles, L.list, L.poff, L.ptotal, L.goff, L.gtotal,
                     L.nb, padded, k_block, params->ko_sigma, geo, s),
          "rhs launch");
  return LTS_OK;
}

lts_status lts_zip(lts_mesh* mesh, int32_t nfields, int32_t precision, const void* k_block, const int32_t* blocks,
                   int32_t nb, void* k_octant, void* stream) {
  clear_error();
  if (!mesh || !k_block || !k_octant) return fail(LTS_EINVAL, "NULL argument");
  if (nfields != 2 && nfields != 6) return fail(LTS_EINVAL, "nfields must be 2 or 6");
  if (!blocks) return fail(LTS_EINVAL, "lts_zip needs an explicit block list");
  Mesh& m = mesh->m;
  hipStream_t s = (hipStream_t)stream;
  lts_status st = ensure_device(m);
  if (st != LTS_OK) return st;
  ListDev L;
  if ((st = stage_list(m, blocks, nb, nullptr, s, L)) != LTS_OK) return st;
  HIP_TRY(launch_zip(precision == LTS_FP32_RHS, m.ni(), m.bt.d_tiles, L.list, L.goff, L.gtotal, L.nb, nfields, m.n(), k_block,
                     k_octant, s),
          "zip launch");
  return LTS_OK;
}

lts_status lts_rk_stage(lts_mesh* mesh, const lts_stage_view* view, const double* coef, int32_t ncoef,
                        const lts_position* pos, const int32_t* blocks, int32_t nb, double* out, void* stream) {
  clear_error();
  if (!mesh || !coef) return fail(LTS_EINVAL, "NULL argument");
  lts_mesh_full* h = static_cast<lts_mesh_full*>(mesh);
  Mesh& m = mesh->m;
  hipStream_t s = (hipStream_t)stream;
  lts_status st = ensure_device(m);
  if (st != LTS_OK) return st;
  if ((st = set_step(&h->x.d_step, pos ? pos->coarse_step : 0, s)) != LTS_OK) return st;
  StageParams sp;
  if ((st = fill_params(m, view, 0, pos, h->x.d_step, sp)) != LTS_OK) return st;
  if (ncoef != sp.p) return fail(LTS_EINVAL, "ncoef must equal the number of stages");
  if (!h->x.d_coef) HIP_TRY(hipMalloc(&h->x.d_coef, 4 * sizeof(double)), "hipMalloc coef");
  HIP_TRY(hipMemcpyAsync(h->x.d_coef, coef, ncoef * sizeof(double), hipMemcpyHostToDevice, s), "upload coef");
  ListDev L;
  if ((st = stage_list(m, blocks, nb, pos, s, L)) != LTS_OK) return st;
  HIP_TRY(launch_rk(view->precision == LTS_FP32_RHS, sp, m.bt.d_tiles, L.list, L.nb, h->x.d_coef, out, s),
          "rk launch");
  return LTS_OK;
}

static LaunchShape g_shape;  // defaults: 512 threads (tile and streaming kernels), grid cap 65536
static int64_t g_shape_gen = 0;  // bumped by every change (captured graphs bake the shape in)

lts_status lts_set_launch(int32_t threads, int32_t max_workgroups, int32_t stream_threads) {
  clear_error();
  if (threads != 256 && threads != 512) return fail(LTS_EINVAL, "threads must be 256 or 512");
  if (stream_threads != 256 && stream_threads != 512) return fail(LTS_EINVAL, "stream_threads must be 256 or 512");
  if (max_workgroups < 8) return fail(LTS_EINVAL, "max_workgroups must be >= 8");
  if (g_shape.threads != threads || g_shape.max_wg != max_workgroups || g_shape.stream_threads != stream_threads)
    ++g_shape_gen;
  g_shape.threads = threads;
  g_shape.max_wg = max_workgroups;
  g_shape.stream_threads = stream_threads;
  return LTS_OK;
}

lts_status lts_set_batch_launch(int32_t threads, int32_t max_workgroups) {
  clear_error();
  if (threads != 256 && threads != 512) return fail(LTS_EINVAL, "threads must be 256 or 512");
  if (max_workgroups < 8) return fail(LTS_EINVAL, "max_workgroups must be >= 8");
  if (g_shape.batch_threads != threads || g_shape.batch_max_wg != max_workgroups) ++g_shape_gen;
  g_shape.batch_threads = threads;
  g_shape.batch_max_wg = max_workgroups;
  return LTS_OK;
}

lts_status lts_get_batch_launch(int32_t* threads, int32_t* max_workgroups) {
  if (threads) *threads = g_shape.batch_threads;
  if (max_workgroups) *max_workgroups = g_shape.batch_max_wg;
  return LTS_OK;
}

lts_status lts_get_launch(int32_t* threads, int32_t* max_workgroups, int32_t* stream_threads) {
  if (threads) *threads = g_shape.threads;
  if (max_workgroups) *max_workgroups = g_shape.max_wg;
  if (stream_threads) *stream_threads = g_shape.stream_threads;
  return LTS_OK;
}

lts_status lts_fused_stage(lts_mesh* mesh, const lts_stage_view* view, int32_t equation,
                           const lts_rhs_params* params, int32_t stage, const lts_position* pos, void* stream) {
  clear_error();
  if (!mesh || !params) return fail(LTS_EINVAL, "NULL argument");
  if (!equation_fields(equation)) return fail(LTS_EINVAL, "bad equation");
  lts_mesh_full* h = static_cast<lts_mesh_full*>(mesh);
  Mesh& m = mesh->m;
  hipStream_t s = (hipStream_t)stream;
  lts_status st = ensure_device(m);
  if (st != LTS_OK) return st;
  if (!view || view->nfields != equation_fields(equation)) return fail(LTS_EINVAL, "nfields does not match the equation");
  if ((st = check_combination(m, equation, view->precision, false)) != LTS_OK) return st;
  if ((st = set_step(&h->x.d_step, pos ? pos->coarse_step : 0, s)) != LTS_OK) return st;
  StageParams sp;
  if ((st = fill_params(m, view, stage, pos, h->x.d_step, sp)) != LTS_OK) return st;
  sp.sigma = params->ko_sigma;
  sp.nl_coeff = params->nl_coeff;
  const int lo = lowest_active_level(m, pos->mode, pos->substep);
  if ((st = ensure_cscr(m, sp.F, 1, &h->x.d_cscr, &h->x.cscr_cap)) != LTS_OK) return st;
  return launch_stage(m, equation, view->precision == LTS_FP32_RHS, sp, lo, m.ghost_ge[lo], h->x.d_cscr, g_shape, s);
}

}  // extern "C"

// ---------------------------------------------------------------- no-allocation variant
// Fixed device scratch of lts_fused_stage_noalloc: the coarse-step counter in the
// first 256 bytes, then the ghost table of the stage.  Every GPU the library runs
// on holds its own copy (its address is looked up once per device).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr size_t kNoAllocHeader = 256;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved on the first call
// on that device.
lts_status scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(LTS_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return fail(LTS_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LTS_OK;
}
}  // namespace

extern "C" lts_status lts_fused_stage_noalloc(lts_mesh* mesh, const lts_stage_view* view, int32_t equation,
                                              const lts_rhs_params* params, int32_t stage, const lts_position* pos,
                                              void* stream) {
  clear_error();
  if (!mesh || !params || !pos) return fail(LTS_EINVAL, "NULL argument");
  if (!equation_fields(equation)) return fail(LTS_EINVAL, "bad equation");
  Mesh& m = mesh->m;
  if (!m.uploaded) return fail(LTS_EINVAL, "mesh tables are not on the device (make one device call on the mesh first)");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != m.device) return fail(LTS_EINVAL, "mesh tables were uploaded to another device");
  if (!view || view->nfields != equation_fields(equation)) return fail(LTS_EINVAL, "nfields does not match the equation");
  lts_status st = check_combination(m, equation, view->precision, false);
  if (st != LTS_OK) return st;
  void* base = nullptr;
  if ((st = scratch_address(&base)) != LTS_OK) return st;
  int64_t* d_step = (int64_t*)base;
  double* gtab = (double*)((char*)base + kNoAllocHeader);
  StageParams sp;
  if ((st = fill_params(m, view, stage, pos, d_step, sp)) != LTS_OK) return st;
  sp.sigma = params->ko_sigma;
  sp.nl_coeff = params->nl_coeff;
  const int lo = lowest_active_level(m, pos->mode, pos->substep);
  const size_t need = (size_t)m.ghost_ge[lo] * sp.F * ghost_points(m) * sizeof(double);
  if (need > kNoAllocScratchBytes - kNoAllocHeader)
    return fail(LTS_EINVAL, "the stage's ghost table (" + std::to_string(need) + " B) exceeds the fixed scratch (" +
                                std::to_string(kNoAllocScratchBytes - kNoAllocHeader) + " B)");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_set_i64(d_step, pos->coarse_step, s), "set step");
  return launch_stage(m, equation, view->precision == LTS_FP32_RHS, sp, lo, m.ghost_ge[lo], gtab, g_shape, s);
}

// ------------------------------------------------------------------------ sims
struct lts_sim {
  lts_mesh* mesh = nullptr;
  int eq = 0, prec = 0, tab = 0, F = 2, p = 4;
  lts_rhs_params prm{};
  void* U = nullptr;
  void* K = nullptr;
  int64_t n = 0;
  int mode = -1;
  int64_t* d_step = nullptr;
  unsigned int* d_nonfinite = nullptr;   // non-finite values written by RK updates
  double w[64], a[16], b[4];
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int64_t graph_tables[2] = {0, 0};  // mesh table generation of each captured graph
  int64_t graph_gen[2] = {0, 0};   // launch-shape generation of each captured graph
  bool poison = false;             // LTS_ADVANCE_POISON: K_s set to NaN before each stage
  bool graph_poison[2] = {false, false};
  // unfused path: device block lists per substep class
  std::vector<ListDev> ulists;
  std::vector<void*> ualloc;
  double* d_pad = nullptr;
  void* d_kb = nullptr;
  double* d_coef = nullptr;
  double* d_cscr = nullptr;     // ghost tables: one per stage of a substep (lts_advance), the first for the phase path
  size_t cscr_cap = 0;
  // continuous batching: the batch the sim is attached to, its round range
  lts_batch* batch = nullptr;
  int slot = -1;
  int64_t r0 = 0, rounds = 0;
};

namespace {

void release_slot(lts_batch* b, lts_sim* sim, bool upload);

void fill_sim_params(const lts_sim* sim, int stage, int mode, int j, StageParams& sp) {
  const Mesh& m = sim->mesh->m;
  std::memset(&sp, 0, sizeof(sp));
  sp.U = (const double*)sim->U;
  sp.Uw = (double*)sim->U;
  sp.K = sim->K;
  sp.Kw = sim->K;
  sp.N = m.n();
  sp.F = sim->F;
  sp.p = sim->p;
  sp.stage = stage;
  sp.mode = mode;
  sp.j = j;
  sp.lmin = m.lmin;
  sp.lmax = m.lmax;
  sp.step = sim->d_step;
  const int p = sim->p;
  for (int c = 0; c < 4; ++c)
    for (int i = 0; i < p; ++i) sp.w[c][i] = sim->w[(c * p + stage) * p + i];
  for (int i = 0; i < p; ++i) sp.b[i] = sim->b[i];
  sp.sigma = sim->prm.ko_sigma;
  sp.leafxyz = m.d_leafxyz;
  sp.fine8 = m.d_fine8;
  sp.ni = m.ni();
  sp.L = m.L;
  sp.periodic = m.periodic ? 1 : 0;
  sp.nl_coeff = sim->prm.nl_coeff;
  sp.nonfinite = sim->d_nonfinite;
  set_kmask(sp);
}


// The stage-s slice of the sim's K array ([F][N][n^3] of doubles or floats).
static void* stage_slice(const lts_sim* sim, int s) {
  const Mesh& m = sim->mesh->m;
  const size_t kb = sim->prec == LTS_FP32_RHS ? 4 : 8;
  return (char*)sim->K + (size_t)s * sim->F * m.n() * m.nn() * kb;
}

lts_status enqueue_coarse_step(lts_sim* sim, int mode, hipStream_t s) {
  Mesh& m = sim->mesh->m;
  const int nsub = 1 << (m.lmax - m.lmin);
  const size_t slot = cscr_slot(m, sim->F);   // stage s reads ghost table s
  for (int j = 0; j < nsub; ++j) {
    const int lo = lowest_active_level(m, mode, j);
    // entries whose receivers lie above lo have an active coarser source: one
    // pre-pass per stage; those with receivers at lo (coarser sources idle during
    // the substep) get all stages at the first
    const int64_t e_hi = lo < LTS_MAX_LEVEL ? m.ghost_ge[lo + 1] : 0, e_lo = m.ghost_ge[lo];
    for (int st = 0; st < sim->p; ++st) {
      StageParams sp;
      fill_sim_params(sim, st, mode, j, sp);
      if (st == 0 && e_lo > e_hi) {
        GhostStages gs{};
        gs.p = sim->p;
        for (int k = 0; k < sim->p; ++k) {
          StageParams sk;
          fill_sim_params(sim, k, mode, j, sk);
          for (int c = 0; c < 4; ++c) {
            for (int i = 0; i < 4; ++i) gs.w[k][c][i] = sk.w[c][i];
            gs.kmask[k] |= (sk.kmask[c] & 15) << (4 * c);
          }
        }
        HIP_TRY(launch_ghost_multi(sim->F, sim->prec == LTS_FP32_RHS, sp, gs, m.d_ghosts, e_hi, e_lo - e_hi,
                                   sim->d_cscr, (int64_t)slot, s),
                "multi-stage ghost pre-pass");
      }
      if (sim->poison) {
        for (int k : {1, 2, 4}) {
          const TileSet& ts = m.ts[k];
          if (ts.count() == 0 || ts.n_ge[lo] == 0) continue;
          HIP_TRY(launch_poison(ts.d_tiles, nullptr, (int)ts.n_ge[lo], stage_slice(sim, st), sim->prec == LTS_FP32_RHS,
                                sim->F, m.n(), (int)m.nn(), s),
                  "poison launch");
        }
      }
      lts_status r = launch_stage(m, sim->eq, sim->prec == LTS_FP32_RHS, sp, lo, e_hi, sim->d_cscr + st * slot,
                                  g_shape, s);
      if (r != LTS_OK) return r;
    }
  }
  HIP_TRY(launch_increment(sim->d_step, s), "step increment");
  return LTS_OK;
}

void drop_graphs(lts_sim* sim) {
  for (int k = 0; k < 2; ++k) {
    if (sim->exec[k]) (void)hipGraphExecDestroy(sim->exec[k]);
    if (sim->graph[k]) (void)hipGraphDestroy(sim->graph[k]);
    sim->exec[k] = nullptr;
    sim->graph[k] = nullptr;
  }
}

}  // namespace

extern "C" {

lts_status lts_sim_create(lts_mesh* mesh, int32_t equation, int32_t precision, int32_t tableau,
                          const lts_rhs_params* params, lts_sim** out) {
  clear_error();
  if (!mesh || !out || !params) return fail(LTS_EINVAL, "NULL argument");
  *out = nullptr;
  if (!equation_fields(equation)) return fail(LTS_EINVAL, "bad equation");
  if (precision != LTS_FP64 && precision != LTS_FP32_RHS) return fail(LTS_EINVAL, "bad precision");
  const int p = tableau_stages(tableau);
  if (!p) return fail(LTS_EINVAL, "bad tableau");
  if (!mesh->m.periodic && equation != LTS_EQ_NLWAVE)
    return fail(LTS_EUNSUPPORTED, "a bounded mesh needs the non-linear wave equation (radiative boundary)");
  if (equation == LTS_EQ_NLWAVE && precision != LTS_FP64)
    return fail(LTS_EUNSUPPORTED, "the non-linear wave runs in FP64");
  if (equation == LTS_EQ_NLWAVE && mesh->m.nodes != 5)
    return fail(LTS_EUNSUPPORTED, "the non-linear wave is built for 5-node octants");
  if ((int64_t)p * equation_fields(equation) * mesh->m.n() * mesh->m.nn() >= (1ll << 31) ||
      mesh->m.n() * mesh->m.nn() * 8 >= (1ll << 32))
    return fail(LTS_EUNSUPPORTED, "arrays too large for the kernels' 32-bit offsets");
  lts_status st = ensure_device(mesh->m);
  if (st != LTS_OK) return st;
  lts_sim* sim = new (std::nothrow) lts_sim();
  if (!sim) return fail(LTS_ENOMEM, "host allocation");
  sim->mesh = mesh;
  sim->eq = equation;
  sim->prec = precision;
  sim->tab = tableau;
  sim->F = equation_fields(equation);
  sim->p = p;
  sim->prm = *params;
  coefficient_tables(tableau, sim->w, sim->a, sim->b);
  hipError_t e = hipMalloc(&sim->d_step, sizeof(int64_t));
  if (e == hipSuccess) e = hipMemset(sim->d_step, 0, sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&sim->d_nonfinite, sizeof(unsigned int));
  if (e == hipSuccess) e = hipMemset(sim->d_nonfinite, 0, sizeof(unsigned int));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&sim->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    lts_sim_destroy(sim);
    return hip_fail(e, "sim create");
  }
  *out = sim;
  return LTS_OK;
}

lts_status lts_sim_bind(lts_sim* sim, void* U, void* K) {
  clear_error();
  if (!sim || !U || !K) return fail(LTS_EINVAL, "NULL argument");
  if (sim->batch) return fail(LTS_EINVAL, "sim is attached to a batch");
  sim->U = U;
  sim->K = K;
  sim->n = 0;
  sim->mode = -1;
  drop_graphs(sim);
  HIP_TRY(hipMemset(sim->d_step, 0, sizeof(int64_t)), "reset step");
  return LTS_OK;
}

static lts_status advance_steps(lts_sim* sim, int64_t n_coarse_steps, int32_t mode, bool use_graph, hipStream_t s);
static lts_status prepare_unfused(lts_sim* sim);
static lts_status enqueue_unfused_step(lts_sim* sim, int32_t mode, hipStream_t s);

lts_status lts_advance(lts_sim* sim, int64_t n_coarse_steps, int32_t mode, int32_t flags, void* stream) {
  clear_error();
  if (!sim || !sim->U) return fail(LTS_EINVAL, "sim not bound");
  if (flags & ~(LTS_ADVANCE_GRAPH | LTS_ADVANCE_CHECK_FINITE | LTS_ADVANCE_POISON))
    return fail(LTS_EINVAL, "unknown advance flags");
  sim->poison = (flags & LTS_ADVANCE_POISON) != 0;
  hipStream_t s = (hipStream_t)stream;
  const bool check = (flags & LTS_ADVANCE_CHECK_FINITE) != 0;
  if (check) HIP_TRY(launch_set_u32(sim->d_nonfinite, 0u, s), "reset finiteness counter");
  lts_status st = advance_steps(sim, n_coarse_steps, mode, (flags & LTS_ADVANCE_GRAPH) != 0, s);
  if (st != LTS_OK || !check) return st;
  unsigned int bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, sim->d_nonfinite, sizeof(bad), hipMemcpyDeviceToHost, s), "read finiteness counter");
  HIP_TRY(hipStreamSynchronize(s), "finiteness sync");
  if (bad) return fail(LTS_ENONFINITE, std::to_string(bad) + " non-finite values written by the RK updates");
  return LTS_OK;
}

static lts_status advance_steps(lts_sim* sim, int64_t n_coarse_steps, int32_t mode, bool use_graph, hipStream_t s) {
  if (!sim || !sim->U) return fail(LTS_EINVAL, "sim not bound");
  if (sim->batch) return fail(LTS_EINVAL, "sim is attached to a batch");
  if (mode != LTS_MODE_LTS && mode != LTS_MODE_GTS) return fail(LTS_EINVAL, "bad mode");
  if (n_coarse_steps < 0) return fail(LTS_EINVAL, "n < 0");
  if (sim->mode >= 0 && sim->mode != mode && sim->n > 0)
    return fail(LTS_EINVAL, "mode differs from the bound state's history; rebind first");
  Mesh& m = sim->mesh->m;
  // the fused stage where it is built for the mesh and equation, else the phase kernels
  const bool phase = !fused_path(m, sim->eq);
  if (phase) {
    lts_status st = prepare_unfused(sim);
    if (st != LTS_OK) return st;
  } else {
    lts_status cc = check_combination(m, sim->eq, sim->prec, false);
    if (cc != LTS_OK) return cc;
    lts_status sc = ensure_cscr(m, sim->F, sim->p, &sim->d_cscr, &sim->cscr_cap);
    if (sc != LTS_OK) return sc;
  }
  auto one_step = [&](hipStream_t st) {
    return phase ? enqueue_unfused_step(sim, mode, st) : enqueue_coarse_step(sim, mode, st);
  };
  sim->mode = mode;
  if (!use_graph) {
    for (int64_t c = 0; c < n_coarse_steps; ++c) {
      lts_status st = one_step(s);
      if (st != LTS_OK) return st;
      sim->n += 1;
    }
    return LTS_OK;
  }
  if (sim->exec[mode] && (sim->graph_tables[mode] != m.tables_gen || sim->graph_gen[mode] != g_shape_gen ||
                          sim->graph_poison[mode] != sim->poison)) {
    drop_graphs(sim);
  }
  if (!sim->exec[mode]) {
    HIP_TRY(hipStreamBeginCapture(sim->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    lts_status st = one_step(sim->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(sim->cap_stream, &g);
    if (st != LTS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    sim->graph[mode] = g;
    HIP_TRY(hipGraphInstantiate(&sim->exec[mode], g, nullptr, nullptr, 0), "graph instantiate");
    sim->graph_tables[mode] = m.tables_gen;
    sim->graph_gen[mode] = g_shape_gen;
    sim->graph_poison[mode] = sim->poison;
  }
  for (int64_t c = 0; c < n_coarse_steps; ++c) {
    HIP_TRY(hipGraphLaunch(sim->exec[mode], s), "graph launch");
    sim->n += 1;
  }
  return LTS_OK;
}

// Device block lists of every substep class and the padded / block-grid scratch
// of the phase kernels, allocated once (outside any graph capture).
static lts_status prepare_unfused(lts_sim* sim) {
  Mesh& m = sim->mesh->m;
  if (sim->ulists.empty()) {
    int64_t pmax = 0, gmax = 0;
    for (int cls = 0; cls <= m.lmax - m.lmin + 1; ++cls) {
      // class 0..dL: lowest active level lmax - cls (LTS); class dL+1: all (GTS)
      const int lo = cls <= m.lmax - m.lmin ? m.lmax - cls : m.lmin;
      std::vector<int32_t> lst;
      for (size_t b = 0; b < m.blocks.size(); ++b)
        if (m.blocks[b].level >= lo) lst.push_back((int32_t)b);
      const size_t n = lst.size();
      std::vector<int64_t> off(2 * n);
      int64_t p = 0, g = 0;
      for (size_t i = 0; i < n; ++i) {
        const int mm = m.blocks[lst[i]].m;
        off[i] = p;
        off[n + i] = g;
        const int ni = m.ni();
        p += (int64_t)(ni * mm + 7) * (ni * mm + 7) * (ni * mm + 7);
        g += (int64_t)(ni * mm + 1) * (ni * mm + 1) * (ni * mm + 1);
      }
      pmax = std::max(pmax, p);
      gmax = std::max(gmax, g);
      ListDev L;
      L.nb = (int)n;
      L.ptotal = p;
      L.gtotal = g;
      void* d = nullptr;
      const size_t bytes = n * 4 + 2 * n * 8 + 16;
      HIP_TRY(hipMalloc(&d, bytes), "hipMalloc lists");
      sim->ualloc.push_back(d);
      char* c8 = (char*)d;
      const size_t o64 = ((n * 4 + 15) / 16) * 16;
      if (n) {
        HIP_TRY(hipMemcpy(c8, lst.data(), n * 4, hipMemcpyHostToDevice), "upload list");
        HIP_TRY(hipMemcpy(c8 + o64, off.data(), 2 * n * 8, hipMemcpyHostToDevice), "upload off");
      }
      L.list = (const int32_t*)c8;
      L.poff = (const int64_t*)(c8 + o64);
      L.goff = L.poff + n;
      sim->ulists.push_back(L);
    }
    const size_t kbytes = sim->prec == LTS_FP32_RHS ? 4 : 8;
    HIP_TRY(hipMalloc(&sim->d_pad, (size_t)pmax * sim->F * 8 + 8), "hipMalloc padded");
    HIP_TRY(hipMalloc(&sim->d_kb, (size_t)gmax * sim->F * kbytes + 8), "hipMalloc kblock");
    HIP_TRY(hipMalloc(&sim->d_coef, 4 * sizeof(double)), "hipMalloc coef");
    HIP_TRY(hipMemcpy(sim->d_coef, sim->b, sim->p * sizeof(double), hipMemcpyHostToDevice), "upload b");
  }
  // the ghost table the unzip reads its coarser ghosts from
  return ensure_cscr(m, sim->F, 1, &sim->d_cscr, &sim->cscr_cap);
}

// One coarse step through the phase kernels (unzip, rhs, zip per stage, then the
// RK update) and the step counter increment.
static lts_status enqueue_unfused_step(lts_sim* sim, int32_t mode, hipStream_t s) {
  Mesh& m = sim->mesh->m;
  const int nsub = 1 << (m.lmax - m.lmin);
  const bool kf32 = sim->prec == LTS_FP32_RHS;
  const size_t kbytes = kf32 ? 4 : 8;
  for (int j = 0; j < nsub; ++j) {
    int cls;
    if (mode == LTS_MODE_GTS) cls = m.lmax - m.lmin + 1;
    else cls = m.lmax - lowest_active_level(m, mode, j);
    const int lo = lowest_active_level(m, mode, j);
    const ListDev& L = sim->ulists[cls];
    for (int st = 0; st < sim->p; ++st) {
      StageParams sp;
      fill_sim_params(sim, st, mode, j, sp);
      if (sim->poison)
        HIP_TRY(launch_poison(m.bt.d_tiles, L.list, L.nb, stage_slice(sim, st), kf32, sim->F, m.n(), (int)m.nn(), s),
                "poison launch");
      HIP_TRY(launch_unzip(kf32, sp, m.bt.d_tiles, m.bt.d_slots, L.list, L.poff, L.nb, L.ptotal, sim->d_pad,
                           m.d_ghosts, m.ghost_ge[lo], sim->d_cscr, m.d_ghost_of_leaf, s),
              "unzip launch");
      HIP_TRY(launch_rhs(sim->eq, kf32, m.bt.d_tiles, L.list, L.poff, L.ptotal, L.goff, L.gtotal, L.nb, sim->d_pad,
                         sim->d_kb, sim->prm.ko_sigma, sp, s),
              "rhs launch");
      char* kslice = (char*)sim->K + (size_t)st * sim->F * m.n() * m.nn() * kbytes;
      HIP_TRY(launch_zip(kf32, m.ni(), m.bt.d_tiles, L.list, L.goff, L.gtotal, L.nb, sim->F, m.n(), sim->d_kb, kslice, s),
              "zip launch");
    }
    StageParams sp;
    fill_sim_params(sim, 0, mode, j, sp);
    HIP_TRY(launch_rk(kf32, sp, m.bt.d_tiles, L.list, L.nb, sim->d_coef, nullptr, s), "rk launch");
  }
  HIP_TRY(launch_increment(sim->d_step, s), "step increment");
  return LTS_OK;
}

lts_status lts_advance_unfused(lts_sim* sim, int64_t n_coarse_steps, int32_t mode, void* stream) {
  clear_error();
  if (!sim || !sim->U) return fail(LTS_EINVAL, "sim not bound");
  if (sim->batch) return fail(LTS_EINVAL, "sim is attached to a batch");
  if (mode != LTS_MODE_LTS && mode != LTS_MODE_GTS) return fail(LTS_EINVAL, "bad mode");
  if (sim->mode >= 0 && sim->mode != mode && sim->n > 0)
    return fail(LTS_EINVAL, "mode differs from the bound state's history; rebind first");
  hipStream_t s = (hipStream_t)stream;
  lts_status st = prepare_unfused(sim);
  if (st != LTS_OK) return st;
  sim->mode = mode;
  sim->poison = false;
  for (int64_t c = 0; c < n_coarse_steps; ++c) {
    if ((st = enqueue_unfused_step(sim, mode, s)) != LTS_OK) return st;
    sim->n += 1;
  }
  return LTS_OK;
}

lts_status lts_sim_current(lts_sim* sim, double* out, void* stream) {
  clear_error();
  if (!sim || !out || !sim->U) return fail(LTS_EINVAL, "NULL argument");
  Mesh& m = sim->mesh->m;
  StageParams sp;
  fill_sim_params(sim, 0, sim->mode < 0 ? LTS_MODE_LTS : sim->mode, 0, sp);
  HIP_TRY(launch_current(sp, m.bt.d_tiles, (int)m.blocks.size(), out, (hipStream_t)stream), "current launch");
  return LTS_OK;
}

lts_status lts_sim_restore(lts_sim* sim, const double* state, int64_t coarse_step, int32_t mode, void* stream) {
  clear_error();
  if (!sim || !state || !sim->U) return fail(LTS_EINVAL, "NULL argument or sim not bound");
  if (sim->batch) return fail(LTS_EINVAL, "sim is attached to a batch");
  if (coarse_step < 0) return fail(LTS_EINVAL, "coarse_step < 0");
  if (mode != LTS_MODE_LTS && mode != LTS_MODE_GTS) return fail(LTS_EINVAL, "bad mode");
  Mesh& m = sim->mesh->m;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_set_i64(sim->d_step, coarse_step, s), "set step");
  StageParams sp;
  fill_sim_params(sim, 0, mode, 0, sp);
  HIP_TRY(launch_restore(sp, m.bt.d_tiles, (int)m.blocks.size(), state, s), "restore launch");
  sim->n = coarse_step;
  sim->mode = mode;
  return LTS_OK;
}

int64_t lts_sim_coarse_step(const lts_sim* sim) { return sim ? sim->n : -1; }

void lts_sim_destroy(lts_sim* sim) {
  if (!sim) return;
  if (sim->batch) release_slot(sim->batch, sim, true);
  drop_graphs(sim);
  if (sim->cap_stream) (void)hipStreamDestroy(sim->cap_stream);
  if (sim->d_step) (void)hipFree(sim->d_step);
  if (sim->d_nonfinite) (void)hipFree(sim->d_nonfinite);
  for (void* p : sim->ualloc) (void)hipFree(p);
  if (sim->d_pad) (void)hipFree(sim->d_pad);
  if (sim->d_kb) (void)hipFree(sim->d_kb);
  if (sim->d_coef) (void)hipFree(sim->d_coef);
  if (sim->d_cscr) (void)hipFree(sim->d_cscr);
  delete sim;
}

lts_status lts_batch_advance(lts_sim* const* sims, int32_t n, int64_t n_coarse_steps, int32_t mode, void* stream) {
  clear_error();
  if (!sims || n <= 0) return fail(LTS_EINVAL, "no sims");
  if (n > kMaxBatch) return fail(LTS_EINVAL, "more sims than a batch holds");
  if (n_coarse_steps < 0) return fail(LTS_EINVAL, "n < 0");
  for (int i = 0; i < n; ++i)
    if (!sims[i]) return fail(LTS_EINVAL, "NULL sim");
  lts_batch* b = nullptr;
  lts_status st = lts_batch_create(sims[0]->eq, sims[0]->prec, sims[0]->tab, mode, n, &b);
  if (st != LTS_OK) return st;
  for (int i = 0; i < n && st == LTS_OK; ++i) st = lts_batch_attach(b, sims[i], n_coarse_steps);
  if (st == LTS_OK) {
    lts_batch_info info;
    lts_batch_query(b, &info);
    st = lts_batch_run(b, info.rounds_to_drain, 1, stream);
  }
  if (st != LTS_OK) {
    std::string msg = g_err;
    for (int i = 0; i < n; ++i)
      if (sims[i]->batch == b) release_slot(b, sims[i], true);
    lts_batch_destroy(b);
    return fail(st, msg);
  }
  lts_batch_destroy(b);
  return LTS_OK;
}

lts_status lts_norms(lts_mesh* mesh, int32_t nfields, const double* a, const double* b, double* out, void* stream) {
  clear_error();
  if (!mesh || !a || !out) return fail(LTS_EINVAL, "NULL argument");
  if (nfields <= 0 || nfields > 6) return fail(LTS_EINVAL, "bad nfields");
  lts_mesh_full* h = static_cast<lts_mesh_full*>(mesh);
  Mesh& m = mesh->m;
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = m.n();
  const size_t need = (size_t)(2 * nfields * N + 1) * sizeof(double);
  if (need > h->x.norm_cap) {
    if (h->x.d_norm) (void)hipFree(h->x.d_norm);
    h->x.d_norm = nullptr;
    h->x.norm_cap = 0;
    HIP_TRY(hipMalloc(&h->x.d_norm, need), "hipMalloc norms");
    h->x.norm_cap = need;
  }
  double* sq = h->x.d_norm;
  double* mx = sq + nfields * N;
  unsigned long long* bad = (unsigned long long*)(mx + nfields * N);
  HIP_TRY(hipMemsetAsync(bad, 0, 8, s), "memset");
  HIP_TRY(launch_norm_partials(a, b, nfields, N, (int)m.nn(), sq, mx, bad, s), "norm launch");
  std::vector<double> hs(2 * nfields * N + 1);
  HIP_TRY(hipMemcpyAsync(hs.data(), sq, need, hipMemcpyDeviceToHost, s), "norm copy");
  HIP_TRY(hipStreamSynchronize(s), "norm sync");
  double wsum = 0.0;
  std::vector<double> w(N);
  for (int64_t o = 0; o < N; ++o) {
    w[o] = std::ldexp(1.0, 3 * (m.L - m.lev[o]));
    wsum += w[o];
  }
  for (int f = 0; f < nfields; ++f) {
    double acc = 0.0, mxv = 0.0;
    for (int64_t o = 0; o < N; ++o) {
      acc += w[o] * hs[f * N + o];
      mxv = std::max(mxv, hs[nfields * N + f * N + o]);
    }
    out[f] = std::sqrt(acc / ((double)m.nn() * wsum));
    out[nfields + f] = mxv;
  }
  unsigned long long nb;
  std::memcpy(&nb, &hs[2 * nfields * N], 8);
  out[2 * nfields] = (double)nb;
  return nb ? fail(LTS_ENONFINITE, "non-finite values in the state") : LTS_OK;
}

// ---- remeshing (Sec. 3.2.2; at coarse-step boundaries) ------------------------------
namespace {
// wavelet indicators of a state on the device: per leaf, and per family (first leaf)
lts_status wavelet_indicators(Mesh& m, int F, const double* state, std::vector<double>& leaf_w,
                              std::vector<int64_t>& fam, std::vector<double>& fam_w, hipStream_t s) {
  fam = families(m);
  const int64_t N = m.n(), nf = (int64_t)fam.size();
  leaf_w.assign(N, 0.0);
  fam_w.assign(nf, 0.0);
  char* d = nullptr;
  const size_t bytes = (size_t)(N + 2 * nf + 1) * 8;
  HIP_TRY(hipMalloc(&d, bytes), "hipMalloc indicators");
  double* d_leaf = (double*)d;
  int64_t* d_fam = (int64_t*)(d + (size_t)N * 8);
  double* d_famw = (double*)(d + (size_t)(N + nf) * 8);
  hipError_t e = hipSuccess;
  if (nf) e = hipMemcpyAsync(d_fam, fam.data(), nf * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_wavelet(state, F, N, d_fam, nf, d_leaf, d_famw, s);
  if (e == hipSuccess) e = hipMemcpyAsync(leaf_w.data(), d_leaf, N * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && nf) e = hipMemcpyAsync(fam_w.data(), d_famw, nf * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "wavelet indicators");
  return LTS_OK;
}
}  // namespace

lts_status lts_remesh_indicators(lts_mesh* mesh, int32_t nfields, const double* state, double* leaf_ind,
                                 double* family_ind, void* stream) {
  clear_error();
  if (!mesh || !state || !leaf_ind || !family_ind) return fail(LTS_EINVAL, "NULL argument");
  if (nfields < 1 || nfields > 6) return fail(LTS_EINVAL, "bad nfields");
  Mesh& m = mesh->m;
  if (m.nodes != 5) return fail(LTS_EUNSUPPORTED, "remeshing is built for 5-node octants");
  std::vector<double> lw, fw;
  std::vector<int64_t> fam;
  lts_status st = wavelet_indicators(m, nfields, state, lw, fam, fw, (hipStream_t)stream);
  if (st != LTS_OK) return st;
  std::copy(lw.begin(), lw.end(), leaf_ind);
  std::fill(family_ind, family_ind + m.n(), -1.0);
  for (size_t q = 0; q < fam.size(); ++q) family_ind[fam[q]] = fw[q];
  return LTS_OK;
}

lts_status lts_remesh(lts_mesh* mesh, int32_t nfields, const double* state, double eps, int32_t l_min, int32_t l_max,
                      lts_mesh** out, void* stream) {
  clear_error();
  if (!mesh || !state || !out) return fail(LTS_EINVAL, "NULL argument");
  *out = nullptr;
  if (nfields < 1 || nfields > 6) return fail(LTS_EINVAL, "bad nfields");
  Mesh& m = mesh->m;
  if (m.nodes != 5) return fail(LTS_EUNSUPPORTED, "remeshing is built for 5-node octants");
  if (!(eps > 0.0) || l_min < 0 || l_min > l_max || l_max > m.L) return fail(LTS_EINVAL, "need eps > 0, 0 <= l_min <= l_max <= L");
  std::vector<double> lw, fw;
  std::vector<int64_t> fam;
  lts_status st = wavelet_indicators(m, nfields, state, lw, fam, fw, (hipStream_t)stream);
  if (st != LTS_OK) return st;
  std::vector<int32_t> leaves;
  remesh_leaves(m, lw, fam, fw, eps, l_min, l_max, leaves);
  lts_mesh_spec spec;
  std::memset(&spec, 0, sizeof(spec));
  spec.l_max = m.L;
  spec.l_min = 99;
  for (size_t i = 3; i < leaves.size(); i += 4) spec.l_min = std::min(spec.l_min, leaves[i]);
  spec.block_cap = m.cap;
  spec.n_leaves = (int64_t)leaves.size() / 4;
  spec.leaves = leaves.data();
  spec.boundary = m.periodic ? LTS_BOUNDARY_PERIODIC : LTS_BOUNDARY_OUTER;
  return lts_build_mesh(&spec, out);
}

lts_status lts_transfer(lts_mesh* from, lts_mesh* to, int32_t nfields, const double* state_from, double* state_to,
                        void* stream) {
  clear_error();
  if (!from || !to || !state_from || !state_to) return fail(LTS_EINVAL, "NULL argument");
  if (nfields < 1 || nfields > 6) return fail(LTS_EINVAL, "bad nfields");
  if (from->m.nodes != 5 || to->m.nodes != 5) return fail(LTS_EUNSUPPORTED, "remeshing is built for 5-node octants");
  std::vector<int32_t> rec;
  lts_status st = transfer_records(from->m, to->m, rec);
  if (st != LTS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  int32_t* d = nullptr;
  HIP_TRY(hipMalloc(&d, rec.size() * 4 + 4), "hipMalloc transfer records");
  hipError_t e = hipMemcpyAsync(d, rec.data(), rec.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_transfer(state_from, from->m.n(), state_to, to->m.n(), nfields, d, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "transfer");
  return LTS_OK;
}

lts_status lts_copy_probe(const void* src, void* dst, size_t nbytes, void* stream) {
  clear_error();
  if (!src || !dst) return fail(LTS_EINVAL, "NULL argument");
  if (nbytes % 32) return fail(LTS_EINVAL, "nbytes must be a multiple of 32");
  HIP_TRY(launch_copy(src, dst, nbytes, (hipStream_t)stream), "copy launch");
  return LTS_OK;
}

}  // extern "C"

// --------------------------------------------------------------------- batches
// Continuous batching: a table of up to `cap` simulations (one equation,
// precision, tableau and mode) advanced by rounds.  Round r runs, for every
// attached simulation, its substep (r - r0) mod 2^(lmax-lmin); each stage of a
// round is a ghost pre-pass and one launch per tile side over the union of the
// active tiles.  Simulations join and leave at round boundaries.
struct lts_batch {
  int eq = 0, prec = 0, tab = 0, mode = 0, F = 2, p = 4, cap = 0;
  int device = -1;
  double w[64], a[16], b[4];
  std::vector<lts_sim*> sims;   // per slot; nullptr = free
  std::vector<BatchSim> desc;   // host copy of the device table
  BatchSim* d_desc = nullptr;
  BatchSim* h_stage = nullptr;  // pinned staging buffer of table uploads
  hipEvent_t staged = nullptr;  // the last upload has read h_stage
  hipEvent_t done = nullptr;    // end of the last enqueued round
  bool staged_rec = false, done_rec = false;
  bool dirty = true;
  int nused = 0;                // table entries [0, nused) are passed to the kernels
  int64_t round = 0;            // next round to run
  int64_t* d_round = nullptr;   // device copy of `round`, read by the kernels
  int32_t* d_tab = nullptr;     // the round table [3][kMaxBatch + 1] (launch_batch_table)
  // one round captured as a graph (valid while the table and the shape stay)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t graph_gen = -1;
  // ghost tables of the attached sims (sim in slot k at entry desc[k].gbase)
  double* d_gscr = nullptr;
  size_t gscr_cap = 0;
};

namespace {

// Free the sim's slot.  A sim released before the end of its rounds must also
// leave the device table (upload = true); one that has used up its rounds is
// already inactive there, so the table (and a captured round) stays valid.
void release_slot(lts_batch* b, lts_sim* sim, bool upload) {
  const int k = sim->slot;
  if (k >= 0 && k < (int)b->sims.size() && b->sims[k] == sim) {
    b->sims[k] = nullptr;
    b->desc[k].rounds = 0;
    if (upload) b->dirty = true;
    sim->mesh->m.attached -= 1;
  }
  sim->batch = nullptr;
  sim->slot = -1;
  if (b->dirty) {   // the table is uploaded again: it can shrink
    int n = (int)b->sims.size();
    while (n > 0 && !b->sims[n - 1]) --n;
    b->nused = n;
  }
}

int64_t rounds_left(const lts_batch* b, const lts_sim* sim) { return sim->r0 + sim->rounds - b->round; }

// stage parameters shared by the batch (arrays and position come from the table)
void fill_batch_params(const lts_batch* b, int stage, StageParams& sp) {
  std::memset(&sp, 0, sizeof(sp));
  sp.ni = 4;   // batches hold 5-node meshes only
  sp.F = b->F;
  sp.p = b->p;
  sp.stage = stage;
  sp.mode = b->mode;
  for (int c = 0; c < 4; ++c)
    for (int i = 0; i < b->p; ++i) sp.w[c][i] = b->w[(c * b->p + stage) * b->p + i];
  for (int i = 0; i < b->p; ++i) sp.b[i] = b->b[i];
  set_kmask(sp);
}

void drop_batch_graph(lts_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

lts_status upload_table(lts_batch* b, hipStream_t s) {
  if (!b->dirty) return LTS_OK;
  drop_batch_graph(b);
  // ghost-table regions, in slot order
  int64_t ge = 0;
  for (int i = 0; i < b->nused; ++i) {
    b->desc[i].gbase = ge;
    if (b->sims[i]) ge += (int64_t)(b->sims[i]->mesh->m.ghosts.size() / 2);
  }
  const size_t need = (size_t)ge * b->F * 729 * sizeof(double);
  if (need > b->gscr_cap) {
    if (b->d_gscr) (void)hipFree(b->d_gscr);   // waits for the work that used it
    b->d_gscr = nullptr;
    b->gscr_cap = 0;
    HIP_TRY(hipMalloc(&b->d_gscr, need), "hipMalloc batch ghost scratch");
    b->gscr_cap = need;
  }
  if (b->nused > 0) {
    if (b->staged_rec) HIP_TRY(hipEventSynchronize(b->staged), "staging wait");
    std::memcpy(b->h_stage, b->desc.data(), b->nused * sizeof(BatchSim));
    HIP_TRY(hipMemcpyAsync(b->d_desc, b->h_stage, b->nused * sizeof(BatchSim), hipMemcpyHostToDevice, s),
            "table upload");
    HIP_TRY(hipEventRecord(b->staged, s), "event record");
    b->staged_rec = true;
  }
  b->dirty = false;
  return LTS_OK;
}

// the sim's coarse-step counter after `done` rounds of its batch run
lts_status finish_rounds(lts_batch* b, lts_sim* sim, int64_t done, hipStream_t s) {
  const int nsub = 1 << (sim->mesh->m.lmax - sim->mesh->m.lmin);
  sim->n = b->desc[sim->slot].n0 + done / nsub;
  HIP_TRY(launch_set_i64(sim->d_step, sim->n, s), "set step");
  release_slot(b, sim, done != sim->rounds);
  return LTS_OK;
}

// Active side-1 / side-2 tiles of round r (exact), or of any round (every
// attached sim at its lowest level: the bound a captured round is sized for).
void round_totals(const lts_batch* b, int64_t r, bool any_round, int64_t total[3]) {
  total[0] = total[1] = total[2] = 0;
  for (int i = 0; i < b->nused; ++i) {
    const lts_sim* sim = b->sims[i];
    if (!sim) continue;
    const BatchSim& d = b->desc[i];
    int lo = d.lmin;
    if (!any_round) {
      const int64_t rr = r - d.r0;
      if (rr < 0 || rr >= d.rounds) continue;
      const int j = (int)(rr & ((1 << (d.lmax - d.lmin)) - 1));
      lo = lowest_active_level(sim->mesh->m, b->mode, j);
    }
    total[0] += d.n_ge[0][lo];
    total[1] += d.n_ge[1][lo];
    total[2] += d.ghost_ge[lo];
  }
}

// The launches of one round: per stage the ghost pre-pass and the two tile
// sides, then the round counter.
lts_status enqueue_round(lts_batch* b, const int64_t total[3], hipStream_t s) {
  const bool kf32 = b->prec == LTS_FP32_RHS;
  // the round's table of cumulative active counts, once for all its launches
  HIP_TRY(launch_batch_table(b->d_desc, b->nused, b->mode, b->d_round, b->d_tab, s), "batch round table");
  LaunchShape bs = g_shape;
  bs.threads = g_shape.batch_threads;
  bs.max_wg = g_shape.batch_max_wg;
  for (int stg = 0; stg < b->p; ++stg) {
    StageParams sp;
    fill_batch_params(b, stg, sp);
    HIP_TRY(launch_ghost_pre_batch(b->F, kf32, sp, b->d_desc, b->nused, b->d_round, total[2], b->d_gscr, b->d_tab,
                                   bs.max_wg, s),
            "batch ghost pre-pass");
    for (int tt = 1; tt <= 2; ++tt)
      HIP_TRY(launch_fused_batch(tt, b->eq, kf32, sp, b->d_desc, b->nused, b->d_round, total[tt - 1], b->d_gscr,
                                 b->d_tab, bs, s),
              "batch launch");
  }
  HIP_TRY(launch_increment(b->d_round, s), "round increment");
  return LTS_OK;
}

}  // namespace

extern "C" {

lts_status lts_batch_create(int32_t equation, int32_t precision, int32_t tableau, int32_t mode, int32_t capacity,
                            lts_batch** out) {
  clear_error();
  if (!out) return fail(LTS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!equation_fields(equation)) return fail(LTS_EINVAL, "bad equation");
  if (equation == LTS_EQ_NLWAVE) return fail(LTS_EUNSUPPORTED, "the non-linear wave is not built for batched launches");
  if (precision != LTS_FP64 && precision != LTS_FP32_RHS) return fail(LTS_EINVAL, "bad precision");
  if (mode != LTS_MODE_LTS && mode != LTS_MODE_GTS) return fail(LTS_EINVAL, "bad mode");
  const int p = tableau_stages(tableau);
  if (!p) return fail(LTS_EINVAL, "bad tableau");
  if (capacity < 1 || capacity > kMaxBatch) return fail(LTS_EINVAL, "capacity must be in [1, 256]");
  lts_batch* b = new (std::nothrow) lts_batch();
  if (!b) return fail(LTS_ENOMEM, "host allocation");
  b->eq = equation;
  b->prec = precision;
  b->tab = tableau;
  b->mode = mode;
  b->F = equation_fields(equation);
  b->p = p;
  b->cap = capacity;
  coefficient_tables(tableau, b->w, b->a, b->b);
  b->sims.assign(capacity, nullptr);
  b->desc.assign(capacity, BatchSim{});
  hipError_t e = hipGetDevice(&b->device);
  if (e == hipSuccess) e = hipMalloc(&b->d_desc, capacity * sizeof(BatchSim));
  if (e == hipSuccess) e = hipHostMalloc(&b->h_stage, capacity * sizeof(BatchSim), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&b->d_round, sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&b->d_tab, 3 * (kMaxBatch + 1) * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(b->d_round, 0, sizeof(int64_t));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    lts_batch_destroy(b);
    return hip_fail(e, "batch create");
  }
  *out = b;
  return LTS_OK;
}

lts_status lts_batch_attach(lts_batch* b, lts_sim* sim, int64_t n_coarse_steps) {
  clear_error();
  if (!b || !sim) return fail(LTS_EINVAL, "NULL argument");
  if (!sim->U) return fail(LTS_EINVAL, "sim not bound");
  if (sim->batch) return fail(LTS_EINVAL, "sim is already attached to a batch");
  if (n_coarse_steps < 0) return fail(LTS_EINVAL, "n < 0");
  if (sim->eq != b->eq || sim->prec != b->prec || sim->tab != b->tab)
    return fail(LTS_EINVAL, "equation, precision and tableau must match the batch's");
  if (sim->mode >= 0 && sim->mode != b->mode && sim->n > 0)
    return fail(LTS_EINVAL, "mode differs from the bound state's history; rebind first");
  Mesh& m = sim->mesh->m;
  if (m.nodes != 5) return fail(LTS_EUNSUPPORTED, "7-node octants are not built for batched launches");
  if (m.ts[4].count() > 0)
    return fail(LTS_EUNSUPPORTED, "batched launches use tile sides 1 and 2 (lts_mesh_set_tile)");
  if (m.device != b->device) return fail(LTS_EINVAL, "sim and batch are on different devices");
  int k = 0;
  while (k < b->cap && b->sims[k]) ++k;
  if (k == b->cap) return fail(LTS_EINVAL, "batch is full");
  const int dl = m.lmax - m.lmin;
  BatchSim d;
  std::memset(&d, 0, sizeof(d));
  d.U = (double*)sim->U;
  d.K = sim->K;
  for (int t = 0; t < 2; ++t) {
    d.tiles[t] = m.ts[t + 1].d_tiles;
    d.slots[t] = m.ts[t + 1].d_slots;
    for (int l = 0; l <= LTS_MAX_LEVEL; ++l) d.n_ge[t][l] = (int32_t)m.ts[t + 1].n_ge[l];
  }
  d.ghosts = m.d_ghosts;
  for (int l = 0; l <= LTS_MAX_LEVEL; ++l) d.ghost_ge[l] = (int32_t)m.ghost_ge[l];
  d.N = m.n();
  d.r0 = b->round;
  d.rounds = n_coarse_steps << dl;
  d.n0 = sim->n;
  d.sigma = sim->prm.ko_sigma;
  d.lmin = m.lmin;
  d.lmax = m.lmax;
  sim->mode = b->mode;
  if (d.rounds == 0) return LTS_OK;   // nothing to do: not attached
  b->desc[k] = d;
  b->sims[k] = sim;
  b->nused = std::max(b->nused, k + 1);
  b->dirty = true;
  sim->batch = b;
  sim->slot = k;
  sim->r0 = d.r0;
  sim->rounds = d.rounds;
  m.attached += 1;
  return LTS_OK;
}

lts_status lts_batch_detach(lts_batch* b, lts_sim* sim, void* stream) {
  clear_error();
  if (!b || !sim) return fail(LTS_EINVAL, "NULL argument");
  if (sim->batch != b) return fail(LTS_EINVAL, "sim is not attached to this batch");
  const int64_t done = b->round - sim->r0;
  const int nsub = 1 << (sim->mesh->m.lmax - sim->mesh->m.lmin);
  if (done % nsub) return fail(LTS_EINVAL, "sim is inside a coarse step (detach at a coarse-step boundary)");
  return finish_rounds(b, sim, done, (hipStream_t)stream);
}

lts_status lts_batch_run(lts_batch* b, int64_t n_rounds, int32_t use_graph, void* stream) {
  clear_error();
  if (!b) return fail(LTS_EINVAL, "batch is NULL");
  if (n_rounds < 0) return fail(LTS_EINVAL, "n < 0");
  hipStream_t s = (hipStream_t)stream;
  lts_status st;
  for (int64_t k = 0; k < n_rounds; ++k) {
    if ((st = upload_table(b, s)) != LTS_OK) return st;
    if (use_graph) {
      if (b->exec && b->graph_gen != g_shape_gen) drop_batch_graph(b);
      if (!b->exec) {
        int64_t total[3];
        round_totals(b, 0, true, total);
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        st = enqueue_round(b, total, b->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (st != LTS_OK) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
        b->graph_gen = g_shape_gen;
      }
      HIP_TRY(hipGraphLaunch(b->exec, s), "graph launch");
    } else {
      int64_t total[3];
      round_totals(b, b->round, false, total);
      if ((st = enqueue_round(b, total, s)) != LTS_OK) return st;
    }
    b->round += 1;
    for (int i = 0; i < b->nused; ++i) {
      lts_sim* sim = b->sims[i];
      if (sim && rounds_left(b, sim) == 0 && (st = finish_rounds(b, sim, sim->rounds, s)) != LTS_OK) return st;
    }
  }
  HIP_TRY(hipEventRecord(b->done, s), "event record");
  b->done_rec = true;
  return LTS_OK;
}

lts_status lts_batch_query(const lts_batch* b, lts_batch_info* info) {
  clear_error();
  if (!b || !info) return fail(LTS_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->round = b->round;
  info->capacity = b->cap;
  for (int i = 0; i < b->nused; ++i) {
    const lts_sim* sim = b->sims[i];
    if (!sim) continue;
    info->attached += 1;
    info->rounds_to_drain = std::max(info->rounds_to_drain, rounds_left(b, sim));
  }
  return LTS_OK;
}

int64_t lts_sim_rounds_left(const lts_sim* sim) {
  if (!sim || !sim->batch) return 0;
  return rounds_left(sim->batch, sim);
}

void lts_batch_destroy(lts_batch* b) {
  if (!b) return;
  if (b->done_rec) (void)hipEventSynchronize(b->done);
  if (b->staged_rec) (void)hipEventSynchronize(b->staged);
  for (int i = 0; i < (int)b->sims.size(); ++i)
    if (b->sims[i]) release_slot(b, b->sims[i], true);
  drop_batch_graph(b);
  if (b->d_gscr) (void)hipFree(b->d_gscr);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_round) (void)hipFree(b->d_round);
  if (b->d_tab) (void)hipFree(b->d_tab);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  delete b;
}

}  // extern "C"
