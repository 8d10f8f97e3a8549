// Host/device helpers shared by the mesh builder's exports and the HIP kernels.
//
// Point location inside a tile's padded region (Sec. 3.3, fig. unzip).  Octants
// have ni + 1 nodes per side (ni = 4, or 6 for 7^3 nodes).  A tile is a cube of
// tt^3 octants at offset o (octants) inside a block of m^3 octants at level l.
// Padded tile point q in [0, ni tt + 7)^3 has block-relative node coordinate
// Q = ni o + q - 3 in [-3, ni m + 3].  Per axis the receiver-level cell is
//   -1 if Q < 0,   min(Q / ni, m-1) if 0 <= Q <= ni m,   m if Q > ni m,
// and nu = Q - ni cell in [0, ni]: the block's closed box is cut along its own
// octant grid, outside it cells are half-open.  The cell is looked up in the
// tile's slot table of (tt+2)^3 entries (cells o-1 .. o+tt per axis).  A slot
// holds one same-level leaf (node nu), leaves one level finer, or one octant
// (child bits beta) of a leaf one level coarser (position (ni beta + nu)/2 in its
// node units, interpolated when odd).  Finer leaves: with ni = 4 all 8 children
// are leaves (ghost-reach balance) and the slot names the first; the point reads
// child c = min(nu>>1, 1), fine node 2(nu - 2c).  With ni = 6 (2:1 balance) only
// the children next to the block need be leaves: the slot names a row of the
// mesh's fine table (8 child leaves, -1 where a child is refined further) and
// the point reads child c = 1 if nu > 3, 0 if nu < 3, and on the mid-plane
// nu = 3 the child next to the block (1 below it, 0 above), fine node
// 2(nu - 3c).
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define LTS_HD __host__ __device__ inline
#else
#define LTS_HD inline
#endif

namespace lts {

enum { SRC_OWN = 0, SRC_SAME = 1, SRC_FINE = 2, SRC_COARSE = 3, SRC_NONE = 4 };

// tile record: int32[8]; TI_COUNTS packs the lengths of the tile's work lists:
// same-level slots | finer slots << 8 | coarser slots << 16 | coarser leaves << 24
enum { TI_FIRST = 0, TI_COUNTS = 1, TI_LEVEL = 2, TI_M = 3, TI_TT = 4, TI_OFF = 5, TI_SLOT = 6, TI_BLOCK = 7 };
// slot record: int32[2] = leaf, kind | beta << 4 | cidx << 8 (cidx: index of a
// coarser source leaf in the tile's list of distinct coarser leaves).  In the
// tile sets of the fused kernels a coarser slot's first int is the coarser
// leaf's ghost-table entry instead (the tile's list keeps (leaf, entry) pairs).

LTS_HD uint32_t part1by2(uint32_t v) {
  uint32_t r = 0;
  for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
  return r;
}

LTS_HD uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}

// Result of locating one padded point: slot index and node offset inside the
// slot's cell (0..ni).
struct Loc {
  int slot;
  int nu[3];
  int below;   // bit d: the cell lies below the block along axis d
};

LTS_HD int cell_of(int Q, int m, int ni = 4) {
  if (Q < 0) return -1;
  if (Q > ni * m) return m;
  const int c = ni == 4 ? Q >> 2 : Q / ni;
  return c < m - 1 ? c : m - 1;
}

// Child of a finer slot along one axis for ni = 6 (see above): below = the cell
// lies below the block along this axis.
LTS_HD int fine_child6(int nu, bool below) { return nu > 3 ? 1 : (nu < 3 ? 0 : (below ? 1 : 0)); }

LTS_HD Loc locate(int qx, int qy, int qz, int ox, int oy, int oz, int tt, int m, int ni = 4) {
  const int q[3] = {qx, qy, qz};
  const int o[3] = {ox, oy, oz};
  Loc r;
  int s[3];
  r.below = 0;
  for (int d = 0; d < 3; ++d) {
    const int Q = ni * o[d] + q[d] - 3;
    r.below |= (Q < 0 ? 1 : 0) << d;
    const int cell = cell_of(Q, m, ni);
    r.nu[d] = Q - ni * cell;
    s[d] = cell - o[d] + 1;
  }
  const int w = tt + 2;
  r.slot = s[0] + w * (s[1] + w * s[2]);
  return r;
}

}  // namespace lts
