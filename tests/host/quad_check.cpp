// Host check of the order-4 pair tiling (geometry.cpp, build_quad_tiles): for
// a configuration on the command line, every selected quadruple maps to one
// accumulator element of one tile, the element decodes (tile -> row block and
// column block -> lane row and column -> pairs) back to (a1, a2) and (a3, a4),
// no element is used twice, every wavefront holds at most kSlotTiles tiles and
// every tile's slot belongs to its wavefront.  Prints "ok" or the first
// violation; exit status 0 / 1.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <vector>

#include "geometry.h"

using namespace bispec;

int main(int argc, char** argv) {
  if (argc < 6) {
    std::printf("usage: quad_check n_g n_shells box_l dk tri_mode [k1 ...]\n");
    return 2;
  }
  bispec_config c{};
  c.n_g = std::atoi(argv[1]);
  c.n_shells = std::atoi(argv[2]);
  c.box_l = std::atof(argv[3]);
  c.dk = std::atof(argv[4]);
  c.tri_mode = std::atoi(argv[5]);
  c.order = 4;
  int k1[64];
  c.n_k1 = 0;
  for (int q = 6; q < argc && c.n_k1 < 64; ++q) k1[c.n_k1++] = std::atoi(argv[q]);
  c.k1_shells = k1;
  std::string err;
  ShellGeometry g;
  std::vector<Quad> q;
  if (validate(c, err) || build_shells(c, g, err) || select_quads(c, g, q, err)) {
    std::printf("config error: %s\n", err.c_str());
    return 1;
  }
  QuadTiling qt;
  build_quad_tiles(q, g.n_s, qt);
  const int waves = qt.n_wg * kSlotsPerWg;
  if ((int)qt.wave_t0.size() != waves + 1) { std::printf("wave table size\n"); return 1; }
  const int n_tiles = (int)qt.tiles.size() / 4;
  for (int w = 0; w < waves; ++w) {
    const int t0 = qt.wave_t0[w], t1 = qt.wave_t0[w + 1];
    if (t1 < t0 || t1 - t0 > kSlotTiles) { std::printf("wavefront %d holds %d tiles\n", w, t1 - t0); return 1; }
    for (int t = t0; t < t1; ++t) {
      const int slot = qt.tiles[4 * t];
      if (slot != (w / kSlotsPerWg) * kTilesPerWg + (w % kSlotsPerWg) * kSlotTiles + (t - t0)) {
        std::printf("tile %d: slot %d not its wavefront's\n", t, slot);
        return 1;
      }
    }
  }
  if (qt.wave_t0[waves] != n_tiles) { std::printf("tiles not all dealt\n"); return 1; }
  std::set<int> seen;
  for (size_t t = 0; t < q.size(); ++t) {
    const int e = qt.slot_of[t];
    if (e < 0 || e >= qt.n_wg * kTilesPerWg * kMTileElems || !seen.insert(e).second) {
      std::printf("bin %zu: element %d out of range or used twice\n", t, e);
      return 1;
    }
    const int slot = e / kMTileElems, el = e % kMTileElems, lane = el % 64, v = el / 64;
    const int r = 4 * (lane >> 4) + v, col = lane % 16;
    int tile = -1;
    for (int k = 0; k < n_tiles; ++k)
      if (qt.tiles[4 * k] == slot) tile = k;
    if (tile < 0) { std::printf("bin %zu: slot %d holds no tile\n", t, slot); return 1; }
    const int pr = qt.rb_pairs[qt.tiles[4 * tile + 1] * 16 + r], pc = qt.cb_pairs[qt.tiles[4 * tile + 2] * 16 + col];
    if (pr >= qt.n_pairs || pc >= qt.n_pairs) { std::printf("bin %zu decodes to a padding pair\n", t); return 1; }
    const int i = (qt.pair_ij[pr] & 0xffff) + 1, j = (qt.pair_ij[pr] >> 16) + 1;
    const int k = (qt.pair_ij[pc] & 0xffff) + 1, l = (qt.pair_ij[pc] >> 16) + 1;
    if (i != q[t].a1 || j != q[t].a2 || k != q[t].a3 || l != q[t].a4) {
      std::printf("bin %zu (%d,%d,%d,%d) decodes to (%d,%d,%d,%d)\n", t, q[t].a1, q[t].a2, q[t].a3, q[t].a4, i, j, k, l);
      return 1;
    }
  }
  std::printf("ok n_quad=%zu pairs=%d tiles=%d work_groups=%d\n", q.size(), qt.n_pairs, n_tiles, qt.n_wg);
  return 0;
}
