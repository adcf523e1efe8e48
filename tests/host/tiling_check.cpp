// Host check of the contraction work decomposition (geometry.cpp): for a
// configuration given on the command line, every selected triangle (on one grid, and in each estimator-grid class) must map to
// exactly one accumulator element of the split-bf16 tiling, that element must
// decode back to the triangle's (a1, a2, a3), its shells must lie in the staged
// row range of its work group, and the vector-kernel tiling must cover every
// triangle once.  Prints "ok" or the first violation; exit status 0 / 1.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <tuple>
#include <string>

#include "geometry.h"

using namespace bispec;

// The checks for one selection on shells 1..n_shells (a grid class, renumbered).
static int check_selection(const Selection& s, int n_shells, const char* what) {
  MfmaTiling mt;
  build_mfma_tiles(s, n_shells, mt);
  const long long cap = (long long)mt.n_wg * kTilesPerWg * kMTileElems;
  std::set<int> seen;
  for (size_t t = 0; t < s.tri.size(); ++t) {
    const int v = mt.slot_of[t];
    if (v < 0 || v >= cap) { std::printf("triangle %zu: element %d out of range\n", t, v); { std::printf("  in %s\n", what); return 1; } }
    if (!seen.insert(v).second) { std::printf("triangle %zu: element %d used twice\n", t, v); { std::printf("  in %s\n", what); return 1; } }
    const int tile = v / kMTileElems, el = v % kMTileElems;
    const int w = tile / kTilesPerWg, loc = tile % kTilesPerWg;
    const int slot = loc / kSlotTiles, k = loc % kSlotTiles;
    const SlotCols& sc = mt.cols[(size_t)w * kSlotsPerWg + slot];
    if (sc.n < 1 || sc.n > kMaxColTiles || sc.n_rb < 1 || sc.n_rb > slot_row_blocks(sc.n)) {
      std::printf("triangle %zu: bad slot shape (%d, %d)\n", t, sc.n, sc.n_rb);
      { std::printf("  in %s\n", what); return 1; }
    }
    const int q = k / sc.n, ct = k % sc.n;
    if (q >= sc.n_rb) { std::printf("triangle %zu: row block beyond the slot\n", t); { std::printf("  in %s\n", what); return 1; } }
    // accumulator element -> (row, column) of the 16 x 16 tile (MFMA output layout)
    const int lane = el % 64, vv = el / 64;
    const int row = 4 * (lane >> 4) + vv, col = lane % 16;
    const MRowBlock& rb = mt.rows[(size_t)w * kRbPerWg + slot * kMaxRbPerSlot + q];
    const int i = rb.i[row], j = rb.j[row], l = sc.col0[ct] + col;
    if (i != s.tri[t].a1 || j != s.tri[t].a2 || l != s.tri[t].a3) {
      std::printf("triangle %zu (%d,%d,%d) decodes to (%d,%d,%d)\n", t, s.tri[t].a1, s.tri[t].a2, s.tri[t].a3, i, j, l);
      { std::printf("  in %s\n", what); return 1; }
    }
    const WgRows& wr = mt.wg_rows[w];
    for (int sh : {i, j, l})
      if (sh - 1 < wr.s_lo || sh - 1 >= wr.s_lo + wr.s_n) {
        std::printf("triangle %zu: shell %d outside the staged rows of work group %d\n", t, sh, w);
        { std::printf("  in %s\n", what); return 1; }
      }
    if (wr.s_n > mt.max_s) { std::printf("work group %d stages more rows than max_s\n", w); { std::printf("  in %s\n", what); return 1; } }
  }
  // vector kernels: every triangle in exactly one tile element
  TilePlan tp;
  build_tiles(s, kMaxTilesPerTask, tp);
  std::set<std::tuple<int, int, int>> cov;
  for (const Tile& tl : tp.tiles) {
    const RowBlock& rb = tp.rows[tl.rb];
    for (int r = 0; r < kRows; ++r) {
      if (!rb.j[r]) continue;
      for (int cc = 0; cc < kCols; ++cc) {
        const int l = tl.col0 + cc;
        if (l >= 1 && l <= rb.j[r]) cov.insert({rb.i[r], rb.j[r], l});
      }
    }
  }
  for (const Tri& t : s.tri)
    if (!cov.count({t.a1, t.a2, t.a3})) { std::printf("vector tiling misses (%d,%d,%d)\n", t.a1, t.a2, t.a3); { std::printf("  in %s\n", what); return 1; } }
  // the highest busy slot position of work group 0 (replicas need it below 12 / rep)
  int top = -1;
  for (int k = 0; k < kSlotsPerWg; ++k)
    if (mt.cols[k].n > 0 && mt.cols[k].n_rb > 0) top = k;
  std::printf("%s: n_tri=%zu work_groups=%d tiles=%lld max_s=%d top_slot=%d rows0=%d\n", what, s.tri.size(), mt.n_wg,
              (long long)mt.tiles, mt.max_s, top, mt.wg_rows[0].s_n);
  return 0;
}

int main(int argc, char** argv) {
  if (argc < 6) {
    std::printf("usage: tiling_check n_g n_shells box_l dk tri_mode [k1 ...]\n");
    return 2;
  }
  bispec_config c{};
  c.n_g = std::atoi(argv[1]);
  c.n_shells = std::atoi(argv[2]);
  c.box_l = std::atof(argv[3]);
  c.dk = std::atof(argv[4]);
  c.tri_mode = std::atoi(argv[5]);
  int k1[64];
  c.n_k1 = 0;
  for (int q = 6; q < argc && c.n_k1 < 64; ++q) k1[c.n_k1++] = std::atoi(argv[q]);
  c.k1_shells = k1;
  c.n_mu = c.n_t = 10;
  std::string err;
  ShellGeometry g;
  Selection s;
  if (validate(c, err) || build_shells(c, g, err) || select_triangles(c, g, s, err)) {
    std::printf("config error: %s\n", err.c_str());
    return 1;
  }
  // the whole selection on one grid, then each estimator-grid class (shells renumbered from its first)
  if (check_selection(s, c.n_shells, "one grid")) return 1;
  std::vector<GridClassSpec> cls;
  choose_grid_classes(g, s, false, cls);
  for (size_t k = 0; k < cls.size(); ++k) {
    Selection cs;
    for (int32_t t : cls[k].tri)
      cs.tri.push_back({s.tri[t].a1 - cls[k].s_lo, s.tri[t].a2 - cls[k].s_lo, s.tri[t].a3 - cls[k].s_lo});
    char what[64];
    std::snprintf(what, sizeof what, "class %zu (G=%d)", k, cls[k].g);
    if (check_selection(cs, cls[k].n_s, what)) return 1;
  }
  std::printf("ok\n");
  return 0;
}
