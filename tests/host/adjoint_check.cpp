// Host check of the matrix-core adjoint tables (geometry.cpp,
// build_adjoint_tables): for a configuration given on the command line, per
// grid class, every output shell belongs to exactly one wavefront, every row
// block's K tiles cover its rows' shells, every weight slot lies inside the
// weight buffer, and the adjoint fields rebuilt from the tables the way the
// kernel indexes them (rows x K tiles x lane / element slots, padding rows and
// shells beyond n_s read as zero) equal the direct sum over the terms
// G_n = sum_t c_t d(F_a1 F_a2 F_a3)/dF_n, for random weights and field values.
// Prints "ok" or the first violation; exit status 0 / 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "geometry.h"

using namespace bispec;

int main(int argc, char** argv) {
  if (argc < 6) {
    std::printf("usage: adjoint_check n_g n_shells box_l dk tri_mode [k1 ...]\n");
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
  std::vector<GridClassSpec> cls;
  choose_grid_classes(g, s, false, cls);
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> cw(s.tri.size());
  for (double& x : cw) x = U(rng);
  constexpr int kVox = 3;
  for (size_t ci = 0; ci < cls.size(); ++ci) {
    const GridClassSpec& k = cls[ci];
    Selection cs;
    for (int32_t t : k.tri) cs.tri.push_back({s.tri[t].a1 - k.s_lo, s.tri[t].a2 - k.s_lo, s.tri[t].a3 - k.s_lo});
    AdjTables at;
    build_adjoint_tables(cs, k.tri, k.n_s, at);
    const int ns = k.n_s;
    // every shell in exactly one wavefront
    std::vector<int> seen(ns + 1, 0);
    if ((int)at.waves.size() != at.n_wg * kAdjWaves) { std::printf("class %zu: wave table size\n", ci); return 1; }
    for (const AdjWave& w : at.waves)
      for (int e = w.e0; e < w.e1; ++e) {
        const int n = at.ns[e].n;
        if (n < 1 || n > ns || seen[n]++) { std::printf("class %zu: shell %d assigned twice or out of range\n", ci, n); return 1; }
      }
    for (int n = 1; n <= ns; ++n)
      if (!seen[n]) { std::printf("class %zu: shell %d has no wavefront\n", ci, n); return 1; }
    if ((long long)at.off.size() != at.n_tiles * 512 + 1) { std::printf("class %zu: slot table size\n", ci); return 1; }
    // weights per slot
    std::vector<double> W(at.n_tiles * 512, 0.0);
    for (long long q = 0; q < at.n_tiles * 512; ++q)
      for (int e = at.off[q]; e < at.off[q + 1]; ++e) W[q] += cw[at.tri[e]];
    // random field values on a few voxels, shells 0..ns-1
    std::vector<double> F((size_t)ns * kVox);
    for (double& x : F) x = U(rng);
    std::vector<double> ref((size_t)(ns + 1) * kVox, 0.0), emu((size_t)(ns + 1) * kVox, 0.0);
    for (size_t q = 0; q < cs.tri.size(); ++q) {
      const Tri& t = cs.tri[q];
      const double w = cw[k.tri[q]];
      for (int v = 0; v < kVox; ++v) {
        const double f1 = F[(t.a1 - 1) * kVox + v], f2 = F[(t.a2 - 1) * kVox + v], f3 = F[(t.a3 - 1) * kVox + v];
        ref[t.a1 * kVox + v] += w * f2 * f3;
        ref[t.a2 * kVox + v] += w * f1 * f3;
        ref[t.a3 * kVox + v] += w * f1 * f2;
      }
    }
    for (const AdjN& nn : at.ns)
      for (int r = nn.rb0; r < nn.rb1; ++r) {
        const AdjRowBlock& rb = at.rbs[r];
        if (rb.w_tile < 0 || rb.w_tile + rb.nkt > at.n_tiles || rb.nkt < 1) {
          std::printf("class %zu: row block %d tiles out of range\n", ci, r);
          return 1;
        }
        // the tiles end within 31 shells past the last (the zero padding the kernel stages)
        if (rb.l8 < 0 || 8 * rb.l8 + kAdjK * rb.nkt > ns + 31) {
          std::printf("class %zu: row block %d tiles reach past the padded shells\n", ci, r);
          return 1;
        }
        for (int row = 0; row < kAdjRows; ++row) {
          const int j = rb.j[row];
          for (int v = 0; v < kVox; ++v) {
            double h = 0.0;
            for (int kt = 0; kt < rb.nkt; ++kt)
              for (int kk = 0; kk < kAdjK; ++kk) {
                const int l = 8 * rb.l8 + kt * kAdjK + kk;   // 0-based shell
                const int lane = row + 16 * (kk / 8), i = kk % 8;
                const double w = W[(size_t)(rb.w_tile + kt) * 512 + lane * 8 + i];
                if (l >= ns) {
                  if (w != 0.0) { std::printf("class %zu: weight beyond the shells\n", ci); return 1; }
                  continue;
                }
                h += w * F[l * kVox + v];
              }
            if (j == 0) {
              if (h != 0.0) { std::printf("class %zu: padding row with weights\n", ci); return 1; }
              continue;
            }
            emu[nn.n * kVox + v] += F[(j - 1) * kVox + v] * h;
          }
        }
      }
    for (int n = 1; n <= ns; ++n)
      for (int v = 0; v < kVox; ++v) {
        const double a = ref[n * kVox + v], b = emu[n * kVox + v];
        if (std::fabs(a - b) > 1e-9 * (1.0 + std::fabs(a))) {
          std::printf("class %zu: G_%d differs: direct %.12g tables %.12g\n", ci, n, a, b);
          return 1;
        }
      }
  }
  std::printf("ok\n");
  return 0;
}
