// Internal declarations of the library (not part of the C ABI).
#pragma once
#include <stdint.h>

#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lts.h"
#include "lts_common.h"

namespace lts {

// Error plumbing: thread-local message, returned status.
lts_status fail(lts_status st, const std::string& msg);
void clear_error();

struct Block {
  int32_t first, m, level, ax, ay, az;
};

// One set of tiles of the fused kernels (all tiles of side tt) or of the
// standalone block kernels (one tile per block, tt = m).
struct TileSet {
  std::vector<int32_t> tiles;   // [T][8]
  std::vector<int32_t> slots;   // [S][2]
  // LTS: tiles are sorted by level (finest first); n_ge[l] = tiles with level >= l
  std::vector<int64_t> n_ge;    // size LTS_MAX_LEVEL + 1
  // per lowest active level l: the prefix [0, n_ge[l]) cut into 8 contiguous
  // ranges of equal estimated cost (one per XCD): xcd[l][0..8]
  std::vector<std::vector<int32_t>> xcd;
  int32_t* d_tiles = nullptr;
  int32_t* d_slots = nullptr;
  int64_t count() const { return (int64_t)tiles.size() / 8; }
};

struct Mesh {
  int L = 0, lmin = 0, lmax = 0, cap = 4;
  bool periodic = true;               // false: bounded by the outer faces
  int nodes = 5;                      // nodes per octant side (5 or 7)
  // 7-node meshes: a finer slot names a row of 8 child leaves (-1: refined
  // further), one row per distinct finer ghost cell (key: level, cell)
  std::vector<int32_t> fine8;
  std::unordered_map<uint64_t, int32_t> fine_row;
  int32_t* d_fine8 = nullptr;
  std::vector<int32_t> ax, ay, az;
  std::vector<int8_t> lev;
  std::vector<uint64_t> key;          // Morton key of the anchor (sorted)
  std::vector<Block> blocks;
  std::vector<int32_t> block_of_leaf;
  int tile = 2;
  TileSet ts[5];                      // ts[t]: tiles of side t (1, 2, 4)
  // Ghost table: every leaf that is a coarser source of some fused tile, with the
  // level of its receivers (its own level + 1), ordered by receiver level
  // (finest first); ghost_ge[l] = entries with receiver level >= l.  The
  // prolongation pre-pass writes entry g's stage state on its (2 ni + 1)^3
  // half-node grid (inside the box its receivers read) to scratch g; a tile's
  // list of distinct coarser leaves holds (leaf, g).
  std::vector<int32_t> ghosts;        // [E][2] = leaf, receiver level | read box << 5
  std::vector<int64_t> ghost_ge;
  std::vector<int32_t> ghost_of_leaf; // [N]: the leaf's ghost-table entry, -1 if none
  int32_t* d_ghosts = nullptr;
  int32_t* d_ghost_of_leaf = nullptr;
  int32_t* d_leafxyz = nullptr;      // [N][4] leaf anchors and levels (positions of the non-linear wave)
  TileSet bt;                         // one tile per block (standalone kernels)
  bool uploaded = false;
  int device = -1;
  int attached = 0;                   // sims of this mesh attached to batches
  int64_t tables_gen = 0;             // bumped whenever the tile tables are rebuilt
  // scratch for the standalone kernels' block lists
  int32_t* d_list = nullptr;
  int64_t* d_off = nullptr;
  size_t list_cap = 0;

  int64_t n() const { return (int64_t)lev.size(); }
  int ni() const { return nodes - 1; }
  int64_t nn() const { return (int64_t)nodes * nodes * nodes; }   // nodes per octant
  int find(int level, int64_t cx, int64_t cy, int64_t cz) const;
};

lts_status build_mesh(const lts_mesh_spec* spec, Mesh& m);
lts_status build_tiles(Mesh& m, int t);
lts_status build_block_tiles(Mesh& m);
void unzip_map_block(const Mesh& m, int b, int32_t* out);  // [(ni m+7)^3][5]

// Remeshing (remesh.cpp): complete same-level sibling families (first leaf), the
// new leaf list [n][4] from the wavelet indicators, and the intergrid transfer
// records [N_to][6] (see launch_transfer).
std::vector<int64_t> families(const Mesh& m);
void remesh_leaves(const Mesh& m, const std::vector<double>& leaf_w, const std::vector<int64_t>& fam,
                   const std::vector<double>& fam_w, double eps, int l_min, int l_max, std::vector<int32_t>& out);
lts_status transfer_records(const Mesh& from, const Mesh& to, std::vector<int32_t>& rec);

// Exact-rational coefficient tables: w[case][s][i] (4 x p x p), a[p][p], b[p].
int tableau_stages(int tableau);
bool coefficient_tables(int tableau, double* w, double* a, double* b);

}  // namespace lts

struct lts_mesh {
  lts::Mesh m;
};
