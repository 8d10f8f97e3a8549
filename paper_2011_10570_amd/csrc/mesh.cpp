// Host mesh builder: refinement, balance, octree-to-block decomposition, tiles
// with their ghost-source slot tables, exports.
//
// Sec. 3.2.2 (refinement), Sec. 3.2.3 (2:1 balance; for 5-node octants extended
// to the reach of three ghost layers), Sec. 3.2.4 (o2o neighbour search),
// Sec. 3.2.5 + fig. oct_to_blocks (blocks = uniformly refined sub-trees).
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "lts_impl.h"

namespace lts {

namespace {

uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 20; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}

uint64_t key_of(int64_t x, int64_t y, int64_t z) {
  return spread3((uint64_t)x) | (spread3((uint64_t)y) << 1) | (spread3((uint64_t)z) << 2);
}

struct Leaf {
  int32_t x, y, z, l;
};

int64_t pmod(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}

int64_t point_dist(int64_t x, int64_t c, int64_t n) {
  int64_t d = pmod(x - c, n);
  return std::min(d, n - d);
}

// smallest / largest periodic distance from c to the closed interval [lo, hi]
int64_t dmin_axis(int64_t lo, int64_t hi, int64_t c, int64_t n) {
  int64_t best = INT64_MAX;
  for (int k = -1; k <= 1; ++k) {
    int64_t d = std::max<int64_t>(0, std::max(lo + k * n - c, c - (hi + k * n)));
    best = std::min(best, d);
  }
  return best;
}

int64_t dmax_axis(int64_t lo, int64_t hi, int64_t c, int64_t n) {
  int64_t anti = pmod(c + n / 2, n);
  for (int k = -1; k <= 1; ++k) {
    int64_t a = anti + k * n;
    if (lo <= a && a <= hi) return n / 2;
  }
  return std::max(point_dist(lo, c, n), point_dist(hi, c, n));
}

// The same distances on a bounded domain (no images).
int64_t dmin_axis_bounded(int64_t lo, int64_t hi, int64_t c) { return std::max<int64_t>(0, std::max(lo - c, c - hi)); }
int64_t dmax_axis_bounded(int64_t lo, int64_t hi, int64_t c) { return std::max(std::abs(lo - c), std::abs(hi - c)); }

bool refine_leaf(const lts_mesh_spec* spec, const Leaf& f, int L, bool periodic, int ni) {
  const int64_t n = (int64_t)ni << L;
  const int64_t s = 1ll << (L - f.l);
  const int64_t lo[3] = {(int64_t)ni * f.x, (int64_t)ni * f.y, (int64_t)ni * f.z};
  for (int ci = 0; ci < spec->n_criteria; ++ci) {
    const lts_criterion& c = spec->criteria[ci];
    int64_t dmin2 = 0, dmax2 = 0;
    for (int d = 0; d < 3; ++d) {
      int64_t a = periodic ? dmin_axis(lo[d], lo[d] + ni * s, c.center[d], n)
                           : dmin_axis_bounded(lo[d], lo[d] + ni * s, c.center[d]);
      dmin2 += a * a;
    }
    if (c.kind == LTS_CRIT_BALL) {
      if (c.r2[f.l] >= 0 && dmin2 < c.r2[f.l]) return true;
    } else {
      if (c.rhi2[f.l] < 0) continue;
      for (int d = 0; d < 3; ++d) {
        int64_t a = periodic ? dmax_axis(lo[d], lo[d] + ni * s, c.center[d], n)
                             : dmax_axis_bounded(lo[d], lo[d] + ni * s, c.center[d]);
        dmax2 += a * a;
      }
      if (c.rlo2[f.l] < dmax2 && dmin2 < c.rhi2[f.l]) return true;
    }
  }
  return false;
}

void push_children(std::vector<Leaf>& out, const Leaf& f, int L) {
  const int32_t h = 1 << (L - f.l - 1);
  for (int c = 0; c < 8; ++c)
    out.push_back({f.x + (c & 1) * h, f.y + ((c >> 1) & 1) * h, f.z + ((c >> 2) & 1) * h, f.l + 1});
}

void sort_leaves(std::vector<Leaf>& v) {
  std::sort(v.begin(), v.end(), [](const Leaf& a, const Leaf& b) {
    return key_of(a.x, a.y, a.z) < key_of(b.x, b.y, b.z);
  });
}

// Number of set cells of a periodic 3D indicator (prefix sums P, side n) in the
// closed integer box [lo, hi] per axis (may wrap or exceed the period).
struct Prefix {
  int64_t n = 0;
  bool periodic = true;   // false: cells beyond [0, n) do not exist
  std::vector<int32_t> P;  // (n+1)^3
  int64_t at(int64_t x, int64_t y, int64_t z) const { return P[(size_t)((z * (n + 1) + y) * (n + 1) + x)]; }
  int64_t box(int64_t x0, int64_t x1, int64_t y0, int64_t y1, int64_t z0, int64_t z1) const {
    return at(x1, y1, z1) - at(x0, y1, z1) - at(x1, y0, z1) - at(x1, y1, z0) + at(x0, y0, z1) + at(x0, y1, z0) +
           at(x1, y0, z0) - at(x0, y0, z0);
  }
  // split [lo, hi] into at most two half-open ranges inside [0, n)
  int ranges(int64_t lo, int64_t hi, int64_t r[2][2]) const {
    if (!periodic) {
      r[0][0] = std::max<int64_t>(lo, 0);
      r[0][1] = std::min<int64_t>(hi + 1, n);
      if (r[0][1] <= r[0][0]) { r[0][0] = 0; r[0][1] = 0; }
      return 1;
    }
    if (hi - lo + 1 >= n) {
      r[0][0] = 0; r[0][1] = n;
      return 1;
    }
    int64_t a = pmod(lo, n), b = a + (hi - lo);
    if (b < n) {
      r[0][0] = a; r[0][1] = b + 1;
      return 1;
    }
    r[0][0] = a; r[0][1] = n;
    r[1][0] = 0; r[1][1] = b - n + 1;
    return 2;
  }
  int64_t count(const int64_t lo[3], const int64_t hi[3]) const {
    int64_t rx[2][2], ry[2][2], rz[2][2];
    int nx = ranges(lo[0], hi[0], rx), ny = ranges(lo[1], hi[1], ry), nz = ranges(lo[2], hi[2], rz);
    int64_t c = 0;
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < ny; ++j)
        for (int k = 0; k < nz; ++k) c += box(rx[i][0], rx[i][1], ry[j][0], ry[j][1], rz[k][0], rz[k][1]);
    return c;
  }
};

// Balance: split a level-l leaf while a leaf of level >= l+2 has Chebyshev box
// distance <= 3 h_l from it (reach: 5-node octants) or touches it (2:1 balance:
// 7-node octants), with periodic images on a periodic domain.  For each l the
// test runs on the level-(l+2) cell grid: the leaf spans cells [A, A+4) per axis;
// the cells whose closed box meets its box grown by 3 h_l (= 3 cells) are
// [A-4, A+7], those whose closed box meets its own box [A-1, A+4].
lts_status balance(std::vector<Leaf>& leaves, int L, bool periodic, bool reach) {
  for (int pass = 0; pass < 64; ++pass) {
    int lo_lev = 99, hi_lev = -1;
    for (const Leaf& f : leaves) { lo_lev = std::min(lo_lev, f.l); hi_lev = std::max(hi_lev, f.l); }
    std::vector<char> split(leaves.size(), 0);
    bool any = false;
    for (int l = lo_lev; l + 2 <= hi_lev; ++l) {
      const int g = l + 2;
      const int64_t n = 1ll << g;
      Prefix pf;
      pf.n = n;
      pf.periodic = periodic;
      std::vector<uint8_t> ind((size_t)(n * n * n), 0);
      for (const Leaf& f : leaves) {
        if (f.l < g) continue;
        const int sh = L - g;
        ind[(size_t)(((f.z >> sh) * n + (f.y >> sh)) * n + (f.x >> sh))] = 1;
      }
      pf.P.assign((size_t)((n + 1) * (n + 1) * (n + 1)), 0);
      for (int64_t z = 0; z < n; ++z)
        for (int64_t y = 0; y < n; ++y) {
          int64_t row = 0;
          for (int64_t x = 0; x < n; ++x) {
            row += ind[(size_t)((z * n + y) * n + x)];
            const size_t o = (size_t)(((z + 1) * (n + 1) + (y + 1)) * (n + 1) + (x + 1));
            pf.P[o] = (int32_t)(row + pf.P[o - (n + 1)] + pf.P[o - (n + 1) * (n + 1)] -
                                pf.P[o - (n + 1) - (n + 1) * (n + 1)]);
          }
        }
      const int sh = L - g;
      for (size_t i = 0; i < leaves.size(); ++i) {
        const Leaf& f = leaves[i];
        if (f.l != l) continue;
        const int64_t A[3] = {f.x >> sh, f.y >> sh, f.z >> sh};
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
          lo[d] = A[d] - (reach ? 4 : 1);
          hi[d] = A[d] + (reach ? 7 : 4);
        }
        if (pf.count(lo, hi) > 0) { split[i] = 1; any = true; }
      }
    }
    if (!any) return LTS_OK;
    std::vector<Leaf> next;
    next.reserve(leaves.size() * 2);
    for (size_t i = 0; i < leaves.size(); ++i) {
      if (split[i]) push_children(next, leaves[i], L);
      else next.push_back(leaves[i]);
    }
    leaves.swap(next);
  }
  return fail(LTS_EINVAL, "balance did not converge");
}

}  // namespace

int Mesh::find(int level, int64_t cx, int64_t cy, int64_t cz) const {
  if (level < 0 || level > L) return -1;
  const int64_t n = 1ll << level;
  if (!periodic && (cx < 0 || cy < 0 || cz < 0 || cx >= n || cy >= n || cz >= n)) return -1;
  const int64_t s = 1ll << (L - level);
  const uint64_t k = key_of(pmod(cx, n) * s, pmod(cy, n) * s, pmod(cz, n) * s);
  auto it = std::lower_bound(key.begin(), key.end(), k);
  if (it == key.end() || *it != k) return -1;
  const int i = (int)(it - key.begin());
  return lev[i] == level ? i : -1;
}

lts_status build_mesh(const lts_mesh_spec* spec, Mesh& m) {
  if (!spec) return fail(LTS_EINVAL, "spec is NULL");
  const int L = spec->l_max;
  if (spec->l_min < 0 || L < spec->l_min || L > 10)
    return fail(LTS_EINVAL, "need 0 <= l_min <= l_max <= 10");
  if (spec->block_cap != 1 && spec->block_cap != 2 && spec->block_cap != 4)
    return fail(LTS_EINVAL, "block_cap must be 1, 2 or 4");
  if (spec->boundary != LTS_BOUNDARY_PERIODIC && spec->boundary != LTS_BOUNDARY_OUTER)
    return fail(LTS_EINVAL, "boundary must be LTS_BOUNDARY_PERIODIC or LTS_BOUNDARY_OUTER");
  const bool periodic = spec->boundary == LTS_BOUNDARY_PERIODIC;
  const int nodes = spec->nodes == 0 ? 5 : spec->nodes;
  if (nodes != 5 && nodes != 7) return fail(LTS_EINVAL, "nodes per octant side must be 5 or 7");
  std::vector<Leaf> leaves;
  if (spec->n_leaves > 0) {
    if (!spec->leaves) return fail(LTS_EINVAL, "leaves is NULL");
    const int64_t side = 1ll << L;
    int64_t vol = 0;
    for (int64_t i = 0; i < spec->n_leaves; ++i) {
      Leaf f{spec->leaves[4 * i], spec->leaves[4 * i + 1], spec->leaves[4 * i + 2], spec->leaves[4 * i + 3]};
      if (f.l < 0 || f.l > L) return fail(LTS_EINVAL, "leaf level out of range");
      const int64_t s = 1ll << (L - f.l);
      if (f.x < 0 || f.y < 0 || f.z < 0 || f.x + s > side || f.y + s > side || f.z + s > side ||
          f.x % s || f.y % s || f.z % s)
        return fail(LTS_EINVAL, "leaf anchor not aligned or outside the domain");
      vol += s * s * s;
      leaves.push_back(f);
    }
    sort_leaves(leaves);
    for (size_t i = 1; i < leaves.size(); ++i)
      if (key_of(leaves[i].x, leaves[i].y, leaves[i].z) == key_of(leaves[i - 1].x, leaves[i - 1].y, leaves[i - 1].z))
        return fail(LTS_EINVAL, "duplicate leaf anchor");
    if (vol != side * side * side) return fail(LTS_EINVAL, "leaves do not tile the domain");
    // overlap check: Morton-sorted non-overlapping leaves have disjoint key ranges
    for (size_t i = 0; i + 1 < leaves.size(); ++i) {
      const uint64_t k0 = key_of(leaves[i].x, leaves[i].y, leaves[i].z);
      const uint64_t span = 1ull << (3 * (L - leaves[i].l));
      if (k0 + span > key_of(leaves[i + 1].x, leaves[i + 1].y, leaves[i + 1].z))
        return fail(LTS_EINVAL, "leaves overlap");
    }
  } else {
    if (spec->n_criteria < 0 || (spec->n_criteria > 0 && !spec->criteria))
      return fail(LTS_EINVAL, "bad criteria");
    for (int ci = 0; ci < spec->n_criteria; ++ci) {
      const int k = spec->criteria[ci].kind;
      if (k != LTS_CRIT_BALL && k != LTS_CRIT_ANNULUS) return fail(LTS_EINVAL, "unknown criterion kind");
    }
    const int32_t s = 1 << (L - spec->l_min), n = 1 << spec->l_min;
    std::vector<Leaf> cur;
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) cur.push_back({x * s, y * s, z * s, spec->l_min});
    for (int l = spec->l_min; l < L && !cur.empty(); ++l) {
      std::vector<Leaf> next;
      for (const Leaf& f : cur) {
        if (refine_leaf(spec, f, L, periodic, nodes - 1)) push_children(next, f, L);
        else leaves.push_back(f);
      }
      cur.swap(next);
    }
    leaves.insert(leaves.end(), cur.begin(), cur.end());
  }
  lts_status st = balance(leaves, L, periodic, nodes == 5);
  if (st != LTS_OK) return st;
  sort_leaves(leaves);

  m.L = L;
  m.periodic = periodic;
  m.nodes = nodes;
  m.fine8.clear();
  m.fine_row.clear();
  m.cap = spec->block_cap;
  const size_t N = leaves.size();
  m.ax.resize(N); m.ay.resize(N); m.az.resize(N); m.lev.resize(N); m.key.resize(N);
  m.lmin = 99; m.lmax = -1;
  for (size_t i = 0; i < N; ++i) {
    m.ax[i] = leaves[i].x; m.ay[i] = leaves[i].y; m.az[i] = leaves[i].z; m.lev[i] = (int8_t)leaves[i].l;
    m.key[i] = key_of(leaves[i].x, leaves[i].y, leaves[i].z);
    m.lmin = std::min(m.lmin, leaves[i].l);
    m.lmax = std::max(m.lmax, leaves[i].l);
  }

  // ---- blocks: largest uniformly refined ancestor of every leaf (fig. oct_to_blocks)
  // cnt[l][i] = number of level-l leaves among the first i leaves
  std::vector<std::vector<int32_t>> cnt(L + 1, std::vector<int32_t>(N + 1, 0));
  for (size_t i = 0; i < N; ++i)
    for (int l = 0; l <= L; ++l) cnt[l][i + 1] = cnt[l][i] + (m.lev[i] == l ? 1 : 0);
  m.blocks.clear();
  m.block_of_leaf.assign(N, -1);
  for (size_t i = 0; i < N; ++i) {
    if (m.block_of_leaf[i] >= 0) continue;
    const int l = m.lev[i];
    int kstar = l;
    for (int k = l - 1; k >= 0; --k) {
      const int64_t span = 1ll << (L - k);
      const int64_t bx = (m.ax[i] / span) * span, by = (m.ay[i] / span) * span, bz = (m.az[i] / span) * span;
      const uint64_t k0 = key_of(bx, by, bz);
      const uint64_t k1 = k0 + (1ull << (3 * (L - k)));
      const int64_t lo = std::lower_bound(m.key.begin(), m.key.end(), k0) - m.key.begin();
      const int64_t hi = std::lower_bound(m.key.begin(), m.key.end(), k1) - m.key.begin();
      const int64_t want = 1ll << (3 * (l - k));
      if (hi - lo == want && cnt[l][hi] - cnt[l][lo] == want) kstar = k;
      else break;
    }
    const int mm = std::min(1 << (l - kstar), m.cap);
    const int64_t span = (int64_t)mm << (L - l);
    const int64_t bx = (m.ax[i] / span) * span, by = (m.ay[i] / span) * span, bz = (m.az[i] / span) * span;
    const int first = (int)(std::lower_bound(m.key.begin(), m.key.end(), key_of(bx, by, bz)) - m.key.begin());
    if (first != (int)i) return fail(LTS_EUNBALANCED, "block anchor is not its first leaf");
    const int bid = (int)m.blocks.size();
    m.blocks.push_back({first, mm, l, (int32_t)bx, (int32_t)by, (int32_t)bz});
    for (int j = 0; j < mm * mm * mm; ++j) {
      if (m.lev[first + j] != l) return fail(LTS_EUNBALANCED, "block is not uniform");
      m.block_of_leaf[first + j] = bid;
    }
  }
  st = build_block_tiles(m);
  if (st != LTS_OK) return st;
  return build_tiles(m, m.nodes == 5 ? 2 : 1);   // 7-node octants: side-1 tiles
}

namespace {

// Slot table entry of the level-l cell c (block-relative octant coordinates,
// may lie outside the block).
lts_status slot_entry(Mesh& m, const Block& B, int cx, int cy, int cz, int32_t out[2]) {
  if (cx >= 0 && cy >= 0 && cz >= 0 && cx < B.m && cy < B.m && cz < B.m) {
    out[0] = B.first + (int32_t)morton3(cx, cy, cz);
    out[1] = SRC_SAME;
    return LTS_OK;
  }
  const int l = B.level;
  const int64_t s = 1ll << (m.L - l);
  const int64_t gx = B.ax / s + cx, gy = B.ay / s + cy, gz = B.az / s + cz;
  if (!m.periodic) {
    const int64_t n = 1ll << l;
    if (gx < 0 || gy < 0 || gz < 0 || gx >= n || gy >= n || gz >= n) {
      out[0] = -1;   // beyond the outer faces: no source
      out[1] = SRC_NONE;
      return LTS_OK;
    }
  }
  int leaf = m.find(l, gx, gy, gz);
  if (leaf >= 0) {
    out[0] = leaf;
    out[1] = SRC_SAME;
    return LTS_OK;
  }
  const int64_t n = 1ll << l;
  const int64_t wx = pmod(gx, n), wy = pmod(gy, n), wz = pmod(gz, n);
  if (l > 0) {
    leaf = m.find(l - 1, wx >> 1, wy >> 1, wz >> 1);
    if (leaf >= 0) {
      const int beta = (int)((wx & 1) | ((wy & 1) << 1) | ((wz & 1) << 2));
      out[0] = leaf;
      out[1] = SRC_COARSE | (beta << 4);
      return LTS_OK;
    }
  }
  if (m.nodes == 7) {
    // the children next to the block must be leaves: per axis c = 1 below the
    // block, 0 above it, both where the cell is level with the block
    int32_t row[8];
    const int cc[3] = {cx, cy, cz};
    for (int c = 0; c < 8; ++c) {
      row[c] = m.find(l + 1, 2 * wx + (c & 1), 2 * wy + ((c >> 1) & 1), 2 * wz + ((c >> 2) & 1));
      bool needed = true;
      for (int d = 0; d < 3; ++d) {
        const int cd = (c >> d) & 1;
        if ((cc[d] < 0 && cd == 0) || (cc[d] >= B.m && cd == 1)) needed = false;
      }
      if (needed && row[c] < 0) return fail(LTS_EUNBALANCED, "ghost cell is neither same, coarser nor finer");
    }
    const uint64_t key = ((uint64_t)(l + 1) << 60) | key_of(wx, wy, wz);
    auto it = m.fine_row.find(key);
    int32_t r;
    if (it != m.fine_row.end()) {
      r = it->second;
    } else {
      r = (int32_t)(m.fine8.size() / 8);
      m.fine8.insert(m.fine8.end(), row, row + 8);
      m.fine_row.emplace(key, r);
    }
    out[0] = r;
    out[1] = SRC_FINE;
    return LTS_OK;
  }
  leaf = m.find(l + 1, 2 * wx, 2 * wy, 2 * wz);
  if (leaf < 0) return fail(LTS_EUNBALANCED, "ghost cell is neither same, coarser nor finer");
  for (int c = 1; c < 8; ++c) {
    const int f = m.find(l + 1, 2 * wx + (c & 1), 2 * wy + ((c >> 1) & 1), 2 * wz + ((c >> 2) & 1));
    if (f != leaf + c) return fail(LTS_EUNBALANCED, "ghost cell is not eight finer leaves");
  }
  out[0] = leaf;
  out[1] = SRC_FINE;
  return LTS_OK;
}

// A tile's slot table: (tt+2)^3 entries (leaf, kind | beta << 4 | cidx << 8) in slot
// order, followed by work lists (one int pair each): the same-level slots, the
// finer slots, the coarser slots, then the distinct coarser source leaves (cidx
// numbers them in order of first appearance).
lts_status add_tile(Mesh& m, int b, int tt, int ox, int oy, int oz, TileSet& ts) {
  const Block B = m.blocks[b];
  const int w = tt + 2;
  const int ns = w * w * w;
  std::vector<int32_t> tab(2 * ns);
  std::vector<int32_t> same, fine, coarse, cleaves;
  for (int sz = 0; sz < w; ++sz)
    for (int sy = 0; sy < w; ++sy)
      for (int sx = 0; sx < w; ++sx) {
        int32_t e[2];
        lts_status st = slot_entry(m, B, ox + sx - 1, oy + sy - 1, oz + sz - 1, e);
        if (st != LTS_OK) return st;
        const int si = sx + w * (sy + w * sz);
        const int kind = e[1] & 15;
        if (kind == SRC_COARSE) {
          int cidx = -1;
          for (size_t k = 0; k < cleaves.size(); ++k)
            if (cleaves[k] == e[0]) cidx = (int)k;
          if (cidx < 0) {
            cidx = (int)cleaves.size();
            cleaves.push_back(e[0]);
          }
          e[1] |= cidx << 8;
          coarse.push_back(si);
        } else if (kind == SRC_FINE) {
          fine.push_back(si);
        } else if (kind == SRC_SAME) {
          same.push_back(si);
        }
        tab[2 * si] = e[0];
        tab[2 * si + 1] = e[1];
      }
  const int32_t slot_off = (int32_t)(ts.slots.size() / 2);
  ts.slots.insert(ts.slots.end(), tab.begin(), tab.end());
  for (const auto* lst : {&same, &fine, &coarse, &cleaves})
    for (int32_t v : *lst) {
      ts.slots.push_back(v);
      ts.slots.push_back(0);
    }
  const int32_t counts = (int32_t)same.size() | ((int32_t)fine.size() << 8) | ((int32_t)coarse.size() << 16) |
                         ((int32_t)cleaves.size() << 24);
  const int32_t rec[8] = {B.first + (int32_t)morton3(ox, oy, oz), counts, B.level, B.m, tt,
                          ox | (oy << 8) | (oz << 16), slot_off, b};
  ts.tiles.insert(ts.tiles.end(), rec, rec + 8);
  return LTS_OK;
}

void finish_levels(TileSet& ts) {
  // sort tiles by level (finest first), stable in Morton order
  const int64_t T = ts.count();
  std::vector<int64_t> idx(T);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return ts.tiles[8 * a + TI_LEVEL] > ts.tiles[8 * b + TI_LEVEL];
  });
  std::vector<int32_t> t2(ts.tiles.size());
  for (int64_t i = 0; i < T; ++i) std::copy(&ts.tiles[8 * idx[i]], &ts.tiles[8 * idx[i]] + 8, &t2[8 * i]);
  ts.tiles.swap(t2);
  ts.n_ge.assign(LTS_MAX_LEVEL + 1, 0);
  for (int l = 0; l <= LTS_MAX_LEVEL; ++l) {
    int64_t c = 0;
    for (int64_t i = 0; i < T; ++i) c += ts.tiles[8 * i + TI_LEVEL] >= l ? 1 : 0;
    ts.n_ge[l] = c;
  }
  // Weighted partition of every launch prefix over the 8 XCDs (the paper's
  // weighted SFC partitioning, Sec. 3.6.4, applied to the chip's dies): cost of a
  // tile = 8 + half its finer slots (each finer point reads its own child leaf);
  // coarser slots read one precomputed ghost-table value and cost no more than
  // same-level ones.  (Weighting coarser slots and coarser leaves as well, as an
  // earlier model did, gave the XCDs unequal work: the wave_c2 step took 72.4
  // against 62.1 ms.)
  std::vector<double> pre(T + 1, 0.0);
  for (int64_t i = 0; i < T; ++i) {
    const int cnt = ts.tiles[8 * i + TI_COUNTS];
    const int nf = (cnt >> 8) & 255;
    pre[i + 1] = pre[i] + 8.0 + 0.5 * nf;
  }
  ts.xcd.assign(LTS_MAX_LEVEL + 1, std::vector<int32_t>(9, 0));
  for (int l = 0; l <= LTS_MAX_LEVEL; ++l) {
    const int64_t n = ts.n_ge[l];
    std::vector<int32_t>& b = ts.xcd[l];
    b[0] = 0;
    for (int x = 1; x < 8; ++x) {
      const double target = pre[n] * x / 8.0;
      int64_t k = std::lower_bound(pre.begin(), pre.begin() + n + 1, target) - pre.begin();
      if (k < b[x - 1]) k = b[x - 1];
      b[x] = (int32_t)std::min<int64_t>(k, n);
    }
    b[8] = (int32_t)n;
  }
}

}  // namespace

// The ghost table (see Mesh::ghosts) of the current tile sets; the second int of
// every entry of a tile's list of distinct coarser leaves becomes the leaf's
// ghost-table index.
static void build_ghosts(Mesh& m) {
  std::vector<int32_t> gid(m.n(), -1);
  std::vector<int32_t> leaves;
  for (int k : {1, 2, 4}) {
    TileSet& ts = m.ts[k];
    for (int64_t i = 0; i < ts.count(); ++i) {
      const int32_t* t = &ts.tiles[8 * i];
      const int cnt = t[TI_COUNTS], tt = t[TI_TT];
      const int ns = (tt + 2) * (tt + 2) * (tt + 2);
      const int ncl = (cnt >> 24) & 255;
      const int nent = ns + (cnt & 255) + ((cnt >> 8) & 255) + ((cnt >> 16) & 255) + ncl;
      for (int c = 0; c < ncl; ++c) {
        const int32_t leaf = ts.slots[2 * ((int64_t)t[TI_SLOT] + nent - ncl + c)];
        if (gid[leaf] < 0) {
          gid[leaf] = 0;
          leaves.push_back(leaf);
        }
      }
    }
  }
  // receiver level = coarser leaf level + 1; finest receivers first, then leaf order
  std::stable_sort(leaves.begin(), leaves.end(), [&](int32_t a, int32_t b) { return m.lev[a] > m.lev[b]; });
  for (size_t g = 0; g < leaves.size(); ++g) gid[leaves[g]] = (int32_t)g;
  // Half-node box of every entry that its receivers read: the union, over the
  // coarser cells of every block's padding, of (ni beta + nu) per axis with nu
  // over the padded points in the cell (every tiling's coarser reads lie in its
  // block's padding).  The pre-pass prolongates only inside the box.
  const int ni = m.ni(), gw = 2 * ni + 1;
  std::vector<int32_t> box(6 * leaves.size());
  for (size_t g = 0; g < leaves.size(); ++g)
    for (int d = 0; d < 3; ++d) {
      box[6 * g + 2 * d] = gw;
      box[6 * g + 2 * d + 1] = -1;
    }
  for (size_t b = 0; b < m.blocks.size(); ++b) {
    const int32_t* t = &m.bt.tiles[8 * b];
    const int mm = t[TI_M], w = mm + 2;
    // per receiver cell c (block-relative, -1..m) the range of nu of its padded points
    std::vector<int> nlo(w, 1 << 20), nhi(w, -1);
    for (int Q = -3; Q <= ni * mm + 3; ++Q) {
      const int c = cell_of(Q, mm, ni);
      nlo[c + 1] = std::min(nlo[c + 1], Q - ni * c);
      nhi[c + 1] = std::max(nhi[c + 1], Q - ni * c);
    }
    const int32_t* sl = &m.bt.slots[2 * (size_t)t[TI_SLOT]];
    for (int sz = 0; sz < w; ++sz)
      for (int sy = 0; sy < w; ++sy)
        for (int sx = 0; sx < w; ++sx) {
          const int si = sx + w * (sy + w * sz);
          const int kb = sl[2 * si + 1];
          if ((kb & 15) != SRC_COARSE) continue;
          const int g = gid[sl[2 * si]];
          const int beta = (kb >> 4) & 7;
          const int s3[3] = {sx, sy, sz};
          for (int d = 0; d < 3; ++d) {
            const int o = ni * ((beta >> d) & 1);
            box[6 * g + 2 * d] = std::min(box[6 * g + 2 * d], o + nlo[s3[d]]);
            box[6 * g + 2 * d + 1] = std::max(box[6 * g + 2 * d + 1], o + nhi[s3[d]]);
          }
        }
  }
  m.ghosts.clear();
  for (size_t g = 0; g < leaves.size(); ++g) {
    m.ghosts.push_back(leaves[g]);
    // receiver level (5 bits) | box (4 bits per bound: x lo, x hi, y lo, y hi, z lo, z hi)
    int32_t rec = m.lev[leaves[g]] + 1;
    for (int d = 0; d < 3; ++d) {
      int lo = box[6 * g + 2 * d], hi = box[6 * g + 2 * d + 1];
      if (hi < lo) {   // no block reads the entry (not expected): the whole grid
        lo = 0;
        hi = gw - 1;
      }
      rec |= (lo << (5 + 8 * d)) | (hi << (9 + 8 * d));
    }
    m.ghosts.push_back(rec);
  }
  m.ghost_of_leaf = gid;
  m.ghost_ge.assign(LTS_MAX_LEVEL + 1, 0);
  for (int l = 0; l <= LTS_MAX_LEVEL; ++l) {
    int64_t c = 0;
    for (size_t g = 0; g < leaves.size(); ++g) c += (m.ghosts[2 * g + 1] & 31) >= l ? 1 : 0;
    m.ghost_ge[l] = c;
  }
  for (int k : {1, 2, 4}) {
    TileSet& ts = m.ts[k];
    for (int64_t i = 0; i < ts.count(); ++i) {
      const int32_t* t = &ts.tiles[8 * i];
      const int cnt = t[TI_COUNTS], tt = t[TI_TT];
      const int ns = (tt + 2) * (tt + 2) * (tt + 2);
      const int ncl = (cnt >> 24) & 255;
      const int nent = ns + (cnt & 255) + ((cnt >> 8) & 255) + ((cnt >> 16) & 255) + ncl;
      for (int c = 0; c < ncl; ++c) {
        const int64_t e = 2 * ((int64_t)t[TI_SLOT] + nent - ncl + c);
        ts.slots[e + 1] = gid[ts.slots[e]];
      }
      // in the slot table itself a coarser slot names its ghost-table entry
      for (int q = 0; q < ns; ++q) {
        const int64_t e = 2 * ((int64_t)t[TI_SLOT] + q);
        if ((ts.slots[e + 1] & 15) == SRC_COARSE) ts.slots[e] = gid[ts.slots[e]];
      }
    }
  }
}

// Tiles of the fused kernels for maximum tile side t (1, 2 or 4): a block of side
// m is cut into tiles of side min(m, t).  ts[k] holds the side-k tiles, each set
// ordered finest level first.  Side-4 tiles (whole 4^3 blocks) are streamed plane
// by plane.  Coarser ghosts of every side come from the ghost-table pre-pass.
lts_status build_tiles(Mesh& m, int t) {
  if (t != 1 && t != 2 && t != 4) return fail(LTS_EINVAL, "tile side must be 1, 2 or 4");
  for (int k = 1; k <= 4; ++k) {
    m.ts[k].tiles.clear();
    m.ts[k].slots.clear();
  }
  for (size_t b = 0; b < m.blocks.size(); ++b) {
    const Block& B = m.blocks[b];
    const int tt = std::min(B.m, t);
    for (int oz = 0; oz < B.m; oz += tt)
      for (int oy = 0; oy < B.m; oy += tt)
        for (int ox = 0; ox < B.m; ox += tt) {
          lts_status st = add_tile(m, (int)b, tt, ox, oy, oz, m.ts[tt]);
          if (st != LTS_OK) return st;
        }
  }
  for (int k : {1, 2, 4}) finish_levels(m.ts[k]);
  build_ghosts(m);
  m.tile = t;
  return LTS_OK;
}

lts_status build_block_tiles(Mesh& m) {
  TileSet& ts = m.bt;
  ts.tiles.clear();
  ts.slots.clear();
  for (size_t b = 0; b < m.blocks.size(); ++b) {
    lts_status st = add_tile(m, (int)b, m.blocks[b].m, 0, 0, 0, ts);
    if (st != LTS_OK) return st;
  }
  // block tiles stay in block order (no level sort): tile b is block b
  return LTS_OK;
}

void unzip_map_block(const Mesh& m, int b, int32_t* out) {
  const TileSet& ts = m.bt;
  const int32_t* t = &ts.tiles[8 * b];
  const int mm = t[TI_M];
  const int ni = m.ni();
  const int P = ni * mm + 7;
  const int32_t* slots = &ts.slots[2 * (size_t)t[TI_SLOT]];
  size_t r = 0;
  for (int qz = 0; qz < P; ++qz)
    for (int qy = 0; qy < P; ++qy)
      for (int qx = 0; qx < P; ++qx, ++r) {
        Loc L = locate(qx, qy, qz, 0, 0, 0, mm, mm, ni);
        const int32_t leaf = slots[2 * L.slot], kb = slots[2 * L.slot + 1];
        const int kind = kb & 15, beta = (kb >> 4) & 7;
        const int sx = L.slot % (mm + 2), sy = (L.slot / (mm + 2)) % (mm + 2), sz = L.slot / ((mm + 2) * (mm + 2));
        const bool inside = sx >= 1 && sx <= mm && sy >= 1 && sy <= mm && sz >= 1 && sz <= mm;
        int32_t* o = out + 5 * r;
        if (inside) {
          o[0] = leaf; o[1] = SRC_OWN;
          for (int d = 0; d < 3; ++d) o[2 + d] = 2 * L.nu[d];
        } else if (kind == SRC_SAME) {
          o[0] = leaf; o[1] = SRC_SAME;
          for (int d = 0; d < 3; ++d) o[2 + d] = 2 * L.nu[d];
        } else if (kind == SRC_NONE) {
          o[0] = -1; o[1] = SRC_NONE;
          for (int d = 0; d < 3; ++d) o[2 + d] = 2 * L.nu[d];
        } else if (kind == SRC_FINE) {
          int c[3];
          if (ni == 4) {
            for (int d = 0; d < 3; ++d) c[d] = L.nu[d] >> 1 < 1 ? L.nu[d] >> 1 : 1;
            o[0] = leaf + c[0] + 2 * c[1] + 4 * c[2];
          } else {
            for (int d = 0; d < 3; ++d) c[d] = fine_child6(L.nu[d], (L.below >> d) & 1);
            o[0] = m.fine8[8 * (size_t)leaf + c[0] + 2 * c[1] + 4 * c[2]];
          }
          o[1] = SRC_FINE;
          for (int d = 0; d < 3; ++d) o[2 + d] = 2 * (2 * L.nu[d] - ni * c[d]);
        } else {
          o[0] = leaf; o[1] = SRC_COARSE;
          for (int d = 0; d < 3; ++d) o[2 + d] = ni * ((beta >> d) & 1) + L.nu[d];
        }
      }
}

}  // namespace lts
