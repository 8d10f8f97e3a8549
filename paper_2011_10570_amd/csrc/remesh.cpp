// Remeshing at a coarse-step boundary (Sec. 3.2.2: the octree follows the
// wavelet criterion; remeshing is a global operation when every block is
// synchronised in time, Sec. 5): complete sibling families, the refine /
// coarsen decisions from the wavelet indicators, and the records of the
// intergrid transfer.
//
// Decisions: a leaf of level < l_max splits where its indicator exceeds eps; a
// complete family of 8 same-level siblings (level > l_min, none splitting)
// merges where the indicator of its parent is below eps / 4 (so a merged parent
// does not split again at the next remesh).  The new leaves are then closed
// under the ghost-reach balance by build_mesh.
#include <algorithm>
#include <vector>

#include "lts_impl.h"

namespace lts {

std::vector<int64_t> families(const Mesh& m) {
  std::vector<int64_t> out;
  const int64_t N = m.n();
  for (int64_t i = 0; i + 8 <= N; ++i) {
    const int l = m.lev[i];
    if (l == 0) continue;
    const int32_t s = 1 << (m.L - l);
    if ((m.ax[i] % (2 * s)) || (m.ay[i] % (2 * s)) || (m.az[i] % (2 * s))) continue;
    bool ok = true;
    for (int c = 0; c < 8 && ok; ++c)
      ok = m.lev[i + c] == l && m.ax[i + c] == m.ax[i] + (c & 1) * s && m.ay[i + c] == m.ay[i] + ((c >> 1) & 1) * s &&
           m.az[i + c] == m.az[i] + ((c >> 2) & 1) * s;
    if (ok) out.push_back(i);
  }
  return out;
}

void remesh_leaves(const Mesh& m, const std::vector<double>& leaf_w, const std::vector<int64_t>& fam,
                   const std::vector<double>& fam_w, double eps, int l_min, int l_max, std::vector<int32_t>& out) {
  const int64_t N = m.n();
  std::vector<char> split(N, 0), merge(N, 0);
  for (int64_t i = 0; i < N; ++i) split[i] = m.lev[i] < l_max && leaf_w[i] > eps;
  for (size_t q = 0; q < fam.size(); ++q) {
    const int64_t f = fam[q];
    if (m.lev[f] <= l_min || !(fam_w[q] < eps / 4)) continue;
    bool any = false;
    for (int c = 0; c < 8; ++c) any |= split[f + c] != 0;
    if (!any)
      for (int c = 0; c < 8; ++c) merge[f + c] = 1;
  }
  out.clear();
  for (int64_t i = 0; i < N; ++i) {
    const int l = m.lev[i];
    if (split[i]) {
      const int32_t h = 1 << (m.L - l - 1);
      for (int c = 0; c < 8; ++c) {
        const int32_t r[4] = {m.ax[i] + (c & 1) * h, m.ay[i] + ((c >> 1) & 1) * h, m.az[i] + ((c >> 2) & 1) * h, l + 1};
        out.insert(out.end(), r, r + 4);
      }
    } else if (merge[i]) {
      // the first leaf of a merged family stands for the parent
      const int32_t s2 = 2 << (m.L - l);
      if (m.ax[i] % s2 == 0 && m.ay[i] % s2 == 0 && m.az[i] % s2 == 0 && (i + 7 < N) && merge[i + 7]) {
        const int32_t r[4] = {m.ax[i], m.ay[i], m.az[i], l - 1};
        out.insert(out.end(), r, r + 4);
      }
    } else {
      const int32_t r[4] = {m.ax[i], m.ay[i], m.az[i], l};
      out.insert(out.end(), r, r + 4);
    }
  }
}

lts_status transfer_records(const Mesh& from, const Mesh& to, std::vector<int32_t>& rec) {
  if (from.L != to.L || from.periodic != to.periodic) return fail(LTS_EINVAL, "meshes of different domains");
  rec.assign(6 * (size_t)to.n(), 0);
  for (int64_t q = 0; q < to.n(); ++q) {
    const int l = to.lev[q];
    // the old leaf holding the new leaf's anchor cell: last key <= the anchor's
    const uint64_t k = to.key[q];
    int64_t o = (int64_t)(std::upper_bound(from.key.begin(), from.key.end(), k) - from.key.begin()) - 1;
    if (o < 0) return fail(LTS_EINVAL, "a new leaf lies outside the old octree");
    const int lo = from.lev[o];
    int32_t* r = &rec[6 * q];
    r[0] = (int32_t)o;
    if (lo <= l) {
      const int32_t s_new = 1 << (to.L - l);
      const int32_t so = 1 << (from.L - lo);
      // the old leaf must contain the new one
      if (to.ax[q] < from.ax[o] || to.ax[q] >= from.ax[o] + so || to.ay[q] < from.ay[o] || to.ay[q] >= from.ay[o] + so ||
          to.az[q] < from.az[o] || to.az[q] >= from.az[o] + so)
        return fail(LTS_EINVAL, "a new leaf is not inside an old leaf");
      r[1] = 0;
      r[2] = 4 * (to.ax[q] - from.ax[o]) / s_new;
      r[3] = 4 * (to.ay[q] - from.ay[o]) / s_new;
      r[4] = 4 * (to.az[q] - from.az[o]) / s_new;
      r[5] = l - lo;
    } else {
      if (lo != l + 1 || o + 8 > from.n()) return fail(LTS_EINVAL, "a new leaf merges leaves more than one level finer");
      for (int c = 0; c < 8; ++c) {
        const int32_t h = 1 << (from.L - lo);
        if (from.lev[o + c] != lo || from.ax[o + c] != to.ax[q] + (c & 1) * h ||
            from.ay[o + c] != to.ay[q] + ((c >> 1) & 1) * h || from.az[o + c] != to.az[q] + ((c >> 2) & 1) * h)
          return fail(LTS_EINVAL, "a new leaf is not the union of 8 old siblings");
      }
      r[1] = 1;
    }
  }
  return LTS_OK;
}

}  // namespace lts
