// Host-side plan geometry: configuration checks, k-shells, triangle selection,
// bin labels and the contraction tile lists.  Pure C++ (no HIP), so the
// host-only queries of the C ABI work without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "bispec.h"

namespace bispec {

struct Tri {
  int32_t a1, a2, a3;
};

struct ShellGeometry {
  int32_t n_g = 0, n_s = 0;
  int32_t n_est = 0;             // estimator grid G (shell fields, triple sums)
  double box_l = 0, w = 0, beta = 0;
  // integer |m|^2 bounds: shell n (1-based) holds lo2[n-1] <= |m|^2 < hi2[n-1]
  std::vector<int64_t> lo2, hi2;
  // largest |m_y| (and |m_z|) of a mode below hi2 of shell n: floor(sqrt(hi2-1))
  std::vector<int32_t> rad;
  std::vector<int64_t> counts;   // modes per shell over the whole lattice
  std::vector<double> mean_k;    // mean |k| per shell (k units)
  // Legendre order of the weight L_ell(k_z/|k|) on each shell's field (empty: none)
  std::vector<int32_t> ell;
};

struct Selection {
  std::vector<Tri> tri;          // ascending (a1,a2,a3)
  std::vector<double> k1_mu_t;   // [n_tri][3]
};

// Order-4 bins (Section 4's polyspectrum with p = 4): a1 >= a2 >= a3 >= a4 >= 1,
// a2 + a3 + a4 >= a1.
struct Quad {
  int32_t a1, a2, a3, a4;
};
int select_quads(const bispec_config& cfg, const ShellGeometry& g, std::vector<Quad>& q, std::string& err);

// The order-4 contraction T = sum_x P_(a1,a2) P_(a3,a4) as a GEMM of row pairs
// (a1, a2) against column pairs (a3, a4), K = voxels: row blocks and column
// blocks of 16 pairs, 16 x 16 tiles holding at least one selected bin; tiles
// dealt to wavefronts (<= kSlotTiles each, kSlotsPerWg per work group), so a
// tile's partial sums sit at slot = wg * kTilesPerWg + wave * kSlotTiles + k.
struct QuadTiling {
  std::vector<int32_t> pair_ij;   // pair p: (i | j << 16), 0-based shells; entry n_pairs: the zero pair
  std::vector<int32_t> rb_pairs;  // [n_rb][16] pair indices (n_pairs = padding)
  std::vector<int32_t> cb_pairs;  // [n_cb][16]
  std::vector<int32_t> tiles;     // [n_tiles][4]: slot, row block, column block, 0
  std::vector<int32_t> wave_t0;   // [n_wg * kSlotsPerWg + 1]: tiles of wavefront w are [wave_t0[w], wave_t0[w+1])
  std::vector<int32_t> slot_of;   // per bin: slot * 256 + element (16 x 16 accumulator layout)
  int32_t n_pairs = 0, n_wg = 0;
};
void build_quad_tiles(const std::vector<Quad>& q, int n_shells, QuadTiling& qt);

// Validates cfg (everything except memory).  Returns a bispec_status.
int validate(const bispec_config& cfg, std::string& err);
int build_shells(const bispec_config& cfg, ShellGeometry& g, std::string& err);
int select_triangles(const bispec_config& cfg, const ShellGeometry& g, Selection& s, std::string& err);

// Grid sizes the FFT kernels are built for: 2^a, 3*2^a, 5*2^a with 2^a >= 8, <= 1024.
bool grid_size_supported(int n);

// ---- estimator-grid classes ------------------------------------------------
//
// The G^3-point triple sum of one triangle (a1, a2, a3) picks exactly its
// closed mode triples once no sum of three mode components can reach +-G,
// i.e. G > R_a1 + R_a2 + R_a3 with R_n the largest component of a mode of
// shell n (the aliasing argument of Section 2.2, eq. 3FT, applied per
// triangle); a shell field is held on G points when G > 2 R_a1.  So each
// triangle can be summed on the smallest supported grid above its own bound.
// The selected triangles are split into classes of one grid each; a class
// evaluates the shell fields of its shell range on its grid and contracts its
// triangles there.  Classes trade voxels of the contraction against extra
// shell transforms and launches; the partition minimises a cost model of the
// three (calibrated on the kernels' measured rates), by dynamic programming
// over the supported sizes up to the plan's estimator grid.
struct GridClassSpec {
  int32_t g = 0;              // grid of the class (points per side)
  int32_t s_lo = 0;           // first shell of the class's fields (0-based)
  int32_t n_s = 0;            // shells s_lo .. s_lo + n_s - 1
  std::vector<int32_t> tri;   // indices of its triangles in the selection, ascending
};
// Smallest grid (supported, >= 8) on which triangle t's sum is exact.
int triangle_min_grid(const ShellGeometry& g, const Tri& t);
// one_grid: a single class on g.n_est over every shell (also when n_est is forced).
void choose_grid_classes(const ShellGeometry& g, const Selection& s, bool one_grid,
                         std::vector<GridClassSpec>& out);

// FFT radix schedule of a length (product of 8,4,2,3,5); empty if unsupported.
std::vector<int> fft_radices(int n);

// ---- contraction work decomposition -------------------------------------
//
// The triple sums T(i,j,l) = sum_x F_i F_j F_l for the selected triangles are
// grouped as a GEMM whose rows are shell pairs (i >= j) and whose columns are
// single shells l: row (i,j) x column l contributes to triangle (i,j,l) when
// l <= j.  Rows are packed in blocks of kRows pairs; each row block meets the
// columns it needs in consecutive blocks of kCols shells.  A tile is one
// (row block, column block) product; every selected triangle lies in exactly
// one tile.
constexpr int kRows = 32;
constexpr int kCols = 32;

struct RowBlock {
  int16_t i[kRows];
  int16_t j[kRows];   // 0 = padding row
};

struct Tile {
  int32_t rb;     // row block
  int32_t col0;   // first column shell (1-based)
};

// A task is at most kMaxTilesPerTask tiles handled together over a voxel range
// by one work group of the vector kernels.  A row block's tiles stay in one
// task when they fit, so its pair products are formed once.
constexpr int kMaxTilesPerTask = 8;

struct TilePlan {
  std::vector<RowBlock> rows;
  std::vector<Tile> tiles;       // task-major
  std::vector<int32_t> task_off; // task q owns tiles [task_off[q], task_off[q+1])
  int64_t useful = 0;            // selected triangles
  int64_t slots = 0;             // tiles * kRows * kCols
};

void build_tiles(const Selection& s, int max_tiles_per_task, TilePlan& tp);

// Tiling of the MFMA kernel (v_mfma_f32_16x16x32_bf16): a row block holds
// kMRows shell pairs, a column tile kMCols consecutive shells.  Column tiles
// are taken in windows of kMaxColTiles; within a window, pairs are grouped by
// the span of column tiles their selected l fall in, so each row block meets
// the column tiles of one span as whole rectangles.  A slot (one wavefront of
// the kernel) holds n_rb row blocks of one span and the n <= kMaxColTiles
// column tiles they meet, with n_rb <= slot_row_blocks(n) so that
// n * n_rb <= kSlotTiles accumulator tiles; a work group has kSlotsPerWg
// slots.  A pair whose l reach several windows appears once per window
// (never for <= 128 shells).
constexpr int kMRows = 16;
constexpr int kMCols = 16;
constexpr int kMTileElems = kMRows * kMCols;  // partial sums per tile
struct MRowBlock {
  int16_t i[kMRows];
  int16_t j[kMRows];   // 0 = padding row
};
constexpr int kMaxColTiles = 8;
constexpr int kSlotTiles = 16;
constexpr int kMaxRbPerSlot = 8;
constexpr int kSlotsPerWg = 12;
constexpr int kRbPerWg = kMaxRbPerSlot * kSlotsPerWg;
constexpr int kTilesPerWg = kSlotTiles * kSlotsPerWg;
inline constexpr int slot_row_blocks(int n_cols) {
  return n_cols <= 2 ? 8 : n_cols == 3 ? 5 : n_cols == 4 ? 4 : n_cols == 5 ? 3 : 2;
}

struct SlotCols {
  int32_t n;                      // column tiles of this slot (0 = idle slot)
  int32_t n_rb;                   // row blocks of this slot
  int32_t col0[kMaxColTiles];     // first shell (1-based) of each column tile
};

struct WgRows {
  int32_t s_lo, s_n;   // shells staged by the work group: s_lo .. s_lo + s_n - 1 (0-based)
};

struct MfmaTiling {
  std::vector<MRowBlock> rows;    // kRbPerWg per work group (kMaxRbPerSlot per slot)
  std::vector<SlotCols> cols;     // kSlotsPerWg per work group
  std::vector<WgRows> wg_rows;    // one per work group
  // triangle t sits in partial slot slot_of[t] = tile * kMTileElems + element
  std::vector<int32_t> slot_of;
  int32_t n_wg = 0;
  int64_t tiles = 0;              // non-empty (row block, column tile) products
  int32_t max_s = 0;              // largest s_n
};

// max_cols (1..kMaxColTiles): the column-tile window, i.e. the most column
// tiles one slot may hold (a tile-shape parameter of the autotuner; narrower
// windows give more, shorter slots whose row operands stream).
void build_mfma_tiles(const Selection& s, int n_shells, MfmaTiling& mt, int max_cols = kMaxColTiles);

// ---- adjoint field build on the matrix cores ------------------------------
// G_n(x) = sum_j F_j(x) H_(n,j)(x),  H_(n,j)(x) = sum_l W[(n,j), l] F_l(x), where
// W[(n,j), l] sums gB_t norm_t over the terms (t; j, l) of d(F_a1 F_a2 F_a3)/dF_n
// (j the larger of the other two shells).  Rows (n, j) of one n, ordered by
// their last l, are cut into row blocks of at most kAdjRows rows (the cut with
// the fewest K tiles); a row block meets nkt K tiles of kAdjK consecutive shells l from
// an 8-aligned first shell (0-based shells 8 l8 + 32 kt .. 8 l8 + 32 kt + 31,
// so the tiles end at most 31 shells past the block's last l).  A K tile's
// weights sit in the MFMA row-operand layout: slot (tile, lane, i) holds row
// lane % 16, K index 8 (lane / 16) + i.
constexpr int kAdjRows = 16;
constexpr int kAdjK = 32;
constexpr int kAdjWaves = 8;        // wavefronts per work group of the kernel
struct AdjRowBlock {
  int16_t j[kAdjRows];  // 1-based j of each row, 0 = padding row
  int32_t w_tile;       // first K tile of the block in the weight buffer
  int16_t l8, nkt;      // K tile kt (0 .. nkt - 1) starts at 0-based shell 8 l8 + kAdjK kt
};
struct AdjN {
  int32_t n;            // 1-based output shell
  int32_t rb0, rb1;     // its row blocks
};
struct AdjWave {
  int32_t e0, e1;       // the AdjN entries of one wavefront
};
// Row blocks, weight-slot lists (CSR: slot q = tile * 512 + lane * 8 + i lists
// the triangles whose terms fall on it; a triangle with two equal shells is
// listed twice where its two terms coincide) and the assignment of every
// output shell 1..n_s to one wavefront of n_wg * kAdjWaves.
struct AdjTables {
  std::vector<AdjRowBlock> rbs;
  std::vector<AdjN> ns;
  std::vector<AdjWave> waves;
  std::vector<int32_t> off, tri;
  long long n_tiles = 0;
  int n_wg = 1;
};
// s: triangles on shells 1..n_s; tri_id[k]: the index reported for triangle k
void build_adjoint_tables(const Selection& s, const std::vector<int32_t>& tri_id, int n_s, AdjTables& at);

}  // namespace bispec
