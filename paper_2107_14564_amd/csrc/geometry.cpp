// Plan geometry on the host (see geometry.h).  Compiled without floating-point
// contraction so the double-precision shell and grid rules evaluate exactly as
// written in bispec.h.
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>

namespace bispec {

static int fail(std::string& err, int code, const char* msg) {
  err = msg;
  return code;
}

std::vector<int> fft_radices(int n) {
  std::vector<int> r;
  if (n < 2) return r;
  while (n % 8 == 0 && n > 8) { r.push_back(8); n /= 8; }
  for (int p : {8, 4, 2, 3, 5})
    while (n % p == 0) { r.push_back(p); n /= p; }
  if (n != 1) r.clear();
  return r;
}

bool grid_size_supported(int n) {
  if (n < 8 || n > 1024) return false;
  int m = n;
  while (m > 1 && m % 2 == 0) m /= 2;
  return (m == 1 || m == 3 || m == 5) && n / m >= 8;
}

int validate(const bispec_config& c, std::string& err) {
  if (!grid_size_supported(c.n_g))
    return fail(err, BISPEC_EINVAL, "n_g must be 2^a, 3*2^a or 5*2^a with 2^a >= 8, at most 1024");
  if (c.n_est != 0 && !grid_size_supported(c.n_est))
    return fail(err, BISPEC_EINVAL, "n_est must be 0 or a supported grid size");
  if (!(c.box_l > 0) || !std::isfinite(c.box_l)) return fail(err, BISPEC_EINVAL, "box_l must be > 0");
  if (!(c.dk >= 1.0) || !std::isfinite(c.dk)) return fail(err, BISPEC_EINVAL, "dk (shell width in k_f) must be >= 1");
  if (c.n_shells < 1 || c.n_shells > 1024) return fail(err, BISPEC_EINVAL, "n_shells must be in [1, 1024]");
  if (!std::isfinite(c.rsd_beta)) return fail(err, BISPEC_EINVAL, "rsd_beta must be finite");
  if (c.precision != BISPEC_PREC_SPLITBF16 && c.precision != BISPEC_PREC_FP32)
    return fail(err, BISPEC_EINVAL, "unknown precision");
  if (c.order != 0 && c.order != 3 && c.order != 4) return fail(err, BISPEC_EINVAL, "order must be 0, 3 or 4");
  // eq. 3FT and Section 4: all shell modes below 2 pi N_g / (p L)  <=>  (n_s + 1/2) w <= N_g / p
  const int p = c.order == 4 ? 4 : 3;
  if ((c.n_shells + 0.5) * c.dk * p > (double)c.n_g)
    return fail(err, BISPEC_ECUTOFF, p == 4 ? "shells reach k >= 2 pi N_g/(4L): need (n_shells + 1/2) dk <= n_g/4"
                                            : "shells reach k >= 2 pi N_g/(3L): need (n_shells + 1/2) dk <= n_g/3");
  if (c.order == 4 && c.tri_mode == BISPEC_TRI_MUT_GRID)
    return fail(err, BISPEC_EINVAL, "order 4 takes the ALL, K1SET or LIST selections");
  if (c.ell != 0 && c.ell != 2 && c.ell != 4) return fail(err, BISPEC_EINVAL, "ell must be 0, 2 or 4");
  if (c.ell != 0 && c.order == 4) return fail(err, BISPEC_EINVAL, "multipoles are defined for the bispectrum only");
  if (c.ell != 0 && (c.flags & BISPEC_FLAG_GRAD))
    return fail(err, BISPEC_EINVAL, "BISPEC_FLAG_GRAD is not available for multipoles (ell > 0)");
  switch (c.tri_mode) {
    case BISPEC_TRI_ALL: break;
    case BISPEC_TRI_K1SET:
    case BISPEC_TRI_MUT_GRID:
      if (c.n_k1 < 1 || !c.k1_shells) return fail(err, BISPEC_EINVAL, "k1_shells required");
      for (int q = 0; q < c.n_k1; ++q)
        if (c.k1_shells[q] < 1 || c.k1_shells[q] > c.n_shells) return fail(err, BISPEC_EINVAL, "k1 shell out of range");
      if (c.tri_mode == BISPEC_TRI_MUT_GRID && (c.n_mu < 2 || c.n_t < 2 || c.n_mu > 4096 || c.n_t > 4096))
        return fail(err, BISPEC_EINVAL, "n_mu and n_t must be in [2, 4096]");
      break;
    case BISPEC_TRI_LIST:
      if (c.n_list < 1 || !c.list) return fail(err, BISPEC_EINVAL, "list required");
      break;
    default: return fail(err, BISPEC_EINVAL, "unknown tri_mode");
  }
  if (c.flags & ~(uint32_t)(BISPEC_FLAG_GRAD | BISPEC_FLAG_STAGE_TIMING | BISPEC_FLAG_AUTOTUNE | BISPEC_FLAG_NO_WORKSPACE |
                            BISPEC_FLAG_ONE_GRID))
    return fail(err, BISPEC_EINVAL, "unknown flag bits");
  return BISPEC_OK;
}

// smallest integer q >= 0 with 4 q >= (2n-1)^2 w^2 (the exact rule of bispec.h)
static int64_t edge_m2(int64_t two_n_pm1, double w) {
  const double rhs = (double)(two_n_pm1 * two_n_pm1) * (w * w);
  int64_t q = (int64_t)std::floor(rhs / 4.0) - 2;
  if (q < 0) q = 0;
  while (!(4.0 * (double)q >= rhs)) ++q;
  return q;
}

int build_shells(const bispec_config& c, ShellGeometry& g, std::string& err) {
  int st = validate(c, err);
  if (st) return st;
  g.n_g = c.n_g;
  g.n_s = c.n_shells;
  g.box_l = c.box_l;
  g.w = c.dk;
  g.beta = c.rsd_beta;
  g.lo2.resize(g.n_s);
  g.hi2.resize(g.n_s);
  g.rad.resize(g.n_s);
  for (int n = 1; n <= g.n_s; ++n) {
    g.lo2[n - 1] = edge_m2(2 * n - 1, g.w);
    g.hi2[n - 1] = edge_m2(2 * n + 1, g.w);
    int64_t r = (int64_t)std::floor(std::sqrt((double)(g.hi2[n - 1] - 1)));
    while (r * r > g.hi2[n - 1] - 1) --r;
    while ((r + 1) * (r + 1) <= g.hi2[n - 1] - 1) ++r;
    g.rad[n - 1] = (int32_t)r;
  }
  // estimator grid: the triple sums over G^3 points are exact when no sum of
  // three mode components can reach +-G, i.e. G > 3 max|m_i| (Section 2.2);
  // four for the order-4 sums
  const int R = g.rad[g.n_s - 1];
  const int need = (c.order == 4 ? 4 : 3) * R + 1;
  if (c.n_est != 0) {
    if (c.n_est < need || c.n_est > c.n_g)
      return fail(err, BISPEC_EINVAL, "n_est must satisfy p max|m_i| < n_est <= n_g (p = 3, or 4 for order 4)");
    g.n_est = c.n_est;
  } else {
    g.n_est = c.n_g;
    for (int q = need; q <= c.n_g; ++q)
      if (grid_size_supported(q)) { g.n_est = q; break; }
  }
  // mode counts and mean |m| over the full lattice ball
  const int64_t top = g.hi2[g.n_s - 1];
  std::vector<double> sum(g.n_s, 0.0);
  g.counts.assign(g.n_s, 0);
  // shell lookup by |m|^2
  std::vector<int32_t> shell_of(top, 0);
  for (int n = 1; n <= g.n_s; ++n)
    for (int64_t q = g.lo2[n - 1]; q < g.hi2[n - 1]; ++q) shell_of[q] = n;
  for (int x = -R; x <= R; ++x)
    for (int y = -R; y <= R; ++y)
      for (int z = -R; z <= R; ++z) {
        int64_t q = (int64_t)x * x + (int64_t)y * y + (int64_t)z * z;
        if (q >= top || q == 0) continue;
        int n = shell_of[q];
        if (!n) continue;
        g.counts[n - 1] += 1;
        sum[n - 1] += std::sqrt((double)q);
      }
  const double kf = 2.0 * M_PI / g.box_l;
  g.mean_k.resize(g.n_s);
  for (int n = 0; n < g.n_s; ++n) {
    if (g.counts[n] == 0) return fail(err, BISPEC_EINVAL, "empty shell");
    g.mean_k[n] = kf * (sum[n] / (double)g.counts[n]);
  }
  return BISPEC_OK;
}

static std::vector<double> linspace_half_one(int n) {
  // numpy.linspace(0.5, 1.0, n): start + i*step, last point exactly 1.0
  std::vector<double> v(n);
  const double step = (1.0 - 0.5) / (double)(n - 1);
  for (int i = 0; i < n; ++i) v[i] = (double)i * step + 0.5;
  v[n - 1] = 1.0;
  return v;
}

int select_triangles(const bispec_config& c, const ShellGeometry& g, Selection& s, std::string& err) {
  std::set<std::tuple<int, int, int>> pick;
  const int ns = g.n_s;
  auto closable = [](int a1, int a2, int a3) { return a1 >= a2 && a2 >= a3 && a3 >= 1 && a2 + a3 >= a1; };
  if (c.tri_mode == BISPEC_TRI_ALL || c.tri_mode == BISPEC_TRI_K1SET) {
    std::vector<char> use(ns + 1, c.tri_mode == BISPEC_TRI_ALL);
    if (c.tri_mode == BISPEC_TRI_K1SET)
      for (int q = 0; q < c.n_k1; ++q) use[c.k1_shells[q]] = 1;
    for (int a1 = 1; a1 <= ns; ++a1) {
      if (!use[a1]) continue;
      for (int a2 = 1; a2 <= a1; ++a2)
        for (int a3 = 1; a3 <= a2; ++a3)
          if (a2 + a3 >= a1) pick.insert({a1, a2, a3});
    }
  } else if (c.tri_mode == BISPEC_TRI_MUT_GRID) {
    const std::vector<double> mus = linspace_half_one(c.n_mu), ts = linspace_half_one(c.n_t);
    for (int q = 0; q < c.n_k1; ++q) {
      const int a1 = c.k1_shells[q];
      for (double t : ts)
        for (double mu : mus) {
          if (t * mu < 0.5 - 1e-12) continue;
          int a2 = (int)std::floor(t * a1 + 0.5);
          a2 = std::min(std::max(a2, 1), a1);
          double r = 1.0 + t * t - 2.0 * mu * t;
          if (r < 0.0) r = 0.0;
          int a3 = (int)std::floor(a1 * std::sqrt(r) + 0.5);
          a3 = std::min(std::max(a3, 1), a2);
          if (closable(a1, a2, a3)) pick.insert({a1, a2, a3});
        }
    }
  } else {  // LIST
    for (int64_t r = 0; r < c.n_list; ++r) {
      int a1 = c.list[3 * r], a2 = c.list[3 * r + 1], a3 = c.list[3 * r + 2];
      if (a1 > ns || !closable(a1, a2, a3)) return fail(err, BISPEC_EINVAL, "list row is not a closable triple within n_shells");
      if (!pick.insert({a1, a2, a3}).second) return fail(err, BISPEC_EINVAL, "duplicate list row");
    }
  }
  if (pick.empty()) return fail(err, BISPEC_EINVAL, "no triangle selected");
  s.tri.clear();
  s.k1_mu_t.clear();
  for (auto& p : pick) {
    Tri t{std::get<0>(p), std::get<1>(p), std::get<2>(p)};
    s.tri.push_back(t);
    const double k1 = g.mean_k[t.a1 - 1], k2 = g.mean_k[t.a2 - 1], k3 = g.mean_k[t.a3 - 1];
    // eq. shape
    s.k1_mu_t.push_back(k1);
    s.k1_mu_t.push_back(0.5 * (k1 / k2 + k2 / k1 - (k3 / k1) * (k3 / k2)));
    s.k1_mu_t.push_back(k2 / k1);
  }
  return BISPEC_OK;
}

int select_quads(const bispec_config& c, const ShellGeometry& g, std::vector<Quad>& q, std::string& err) {
  std::set<std::tuple<int, int, int, int>> pick;
  const int ns = g.n_s;
  auto closable = [](int a1, int a2, int a3, int a4) {
    return a1 >= a2 && a2 >= a3 && a3 >= a4 && a4 >= 1 && a2 + a3 + a4 >= a1;
  };
  if (c.tri_mode == BISPEC_TRI_ALL || c.tri_mode == BISPEC_TRI_K1SET) {
    std::vector<char> use(ns + 1, c.tri_mode == BISPEC_TRI_ALL);
    if (c.tri_mode == BISPEC_TRI_K1SET)
      for (int k = 0; k < c.n_k1; ++k) use[c.k1_shells[k]] = 1;
    for (int a1 = 1; a1 <= ns; ++a1) {
      if (!use[a1]) continue;
      for (int a2 = 1; a2 <= a1; ++a2)
        for (int a3 = 1; a3 <= a2; ++a3)
          for (int a4 = 1; a4 <= a3; ++a4)
            if (a2 + a3 + a4 >= a1) pick.insert({a1, a2, a3, a4});
    }
  } else if (c.tri_mode == BISPEC_TRI_LIST) {
    for (int64_t r = 0; r < c.n_list; ++r) {
      const int a1 = c.list[4 * r], a2 = c.list[4 * r + 1], a3 = c.list[4 * r + 2], a4 = c.list[4 * r + 3];
      if (a1 > ns || !closable(a1, a2, a3, a4))
        return fail(err, BISPEC_EINVAL, "list row is not a closable quadruple within n_shells");
      if (!pick.insert({a1, a2, a3, a4}).second) return fail(err, BISPEC_EINVAL, "duplicate list row");
    }
  } else {
    return fail(err, BISPEC_EINVAL, "order 4 takes the ALL, K1SET or LIST selections");
  }
  if (pick.empty()) return fail(err, BISPEC_EINVAL, "no quadruple selected");
  q.clear();
  for (auto& p : pick) q.push_back({std::get<0>(p), std::get<1>(p), std::get<2>(p), std::get<3>(p)});
  return BISPEC_OK;
}

void build_quad_tiles(const std::vector<Quad>& q, int n_shells, QuadTiling& qt) {
  (void)n_shells;
  // row pairs ordered by a2 then a1, column pairs by a3 then a4: bins (a2 >= a3)
  // then fill one side of the tile grid's diagonal
  std::map<std::pair<int, int>, int> rkey, ckey, pid;
  for (const Quad& b : q) {
    rkey[{b.a2, b.a1}] = 0;
    ckey[{b.a3, b.a4}] = 0;
    pid[{b.a1, b.a2}] = 0;
    pid[{b.a3, b.a4}] = 0;
  }
  qt.pair_ij.clear();
  for (auto& kv : pid) {
    kv.second = (int)qt.pair_ij.size();
    qt.pair_ij.push_back((kv.first.first - 1) | ((kv.first.second - 1) << 16));
  }
  qt.n_pairs = (int32_t)qt.pair_ij.size();
  qt.pair_ij.push_back(-1);  // the zero pair (the kernels map it to the zero row)
  auto blocks = [&](std::map<std::pair<int, int>, int>& keys, bool rows, std::vector<int32_t>& out) {
    int k = 0;
    out.clear();
    for (auto& kv : keys) {
      kv.second = k++;
      const std::pair<int, int> ij = rows ? std::make_pair(kv.first.second, kv.first.first) : kv.first;
      out.push_back(pid.at(ij));
    }
    while (out.size() % 16) out.push_back(qt.n_pairs);
  };
  blocks(rkey, true, qt.rb_pairs);
  blocks(ckey, false, qt.cb_pairs);
  // tiles with a selected bin, dealt to wavefronts in order
  std::map<std::pair<int, int>, std::vector<int>> tile_bins;
  for (size_t t = 0; t < q.size(); ++t) {
    const int r = rkey.at({q[t].a2, q[t].a1}), cc = ckey.at({q[t].a3, q[t].a4});
    tile_bins[{r / 16, cc / 16}].push_back((int)t);
  }
  const int n_tiles = (int)tile_bins.size();
  const int n_waves = (n_tiles + kSlotTiles - 1) / kSlotTiles;
  qt.n_wg = std::max(1, (n_waves + kSlotsPerWg - 1) / kSlotsPerWg);
  // spread the tiles evenly over every wavefront of the work groups
  const int waves_total = qt.n_wg * kSlotsPerWg;
  qt.wave_t0.assign(waves_total + 1, 0);
  qt.tiles.clear();
  qt.slot_of.assign(q.size(), -1);
  auto it = tile_bins.begin();
  for (int w = 0; w < waves_total; ++w) {
    const int take = n_tiles / waves_total + (w < n_tiles % waves_total ? 1 : 0);
    const int wg = w / kSlotsPerWg, wave = w % kSlotsPerWg;
    qt.wave_t0[w] = (int32_t)(qt.tiles.size() / 4);
    for (int k = 0; k < take; ++k, ++it) {
      const int slot = wg * kTilesPerWg + wave * kSlotTiles + k;
      qt.tiles.insert(qt.tiles.end(), {slot, it->first.first, it->first.second, 0});
      for (int t : it->second) {
        const int r = rkey.at({q[t].a2, q[t].a1}) % 16, cc = ckey.at({q[t].a3, q[t].a4}) % 16;
        const int lane = cc + 16 * (r >> 2), v = r & 3;
        qt.slot_of[t] = slot * kMTileElems + v * 64 + lane;
      }
    }
  }
  qt.wave_t0[waves_total] = (int32_t)(qt.tiles.size() / 4);
}

void build_tiles(const Selection& s, int max_tiles_per_task, TilePlan& tp) {
  // pairs (i, j) with their selected l values
  std::map<std::pair<int, int>, std::vector<int>> pl;
  for (const Tri& t : s.tri) pl[{t.a1, t.a2}].push_back(t.a3);
  struct P { int i, j, lo, hi; };
  std::vector<P> pairs;
  for (auto& kv : pl) {
    auto mm = std::minmax_element(kv.second.begin(), kv.second.end());
    pairs.push_back({kv.first.first, kv.first.second, *mm.first, *mm.second});
  }
  // rows with similar column ranges share a block: order by (hi, lo, i, j)
  std::sort(pairs.begin(), pairs.end(), [](const P& a, const P& b) {
    if (a.hi != b.hi) return a.hi < b.hi;
    if (a.lo != b.lo) return a.lo < b.lo;
    if (a.i != b.i) return a.i < b.i;
    return a.j < b.j;
  });
  tp.rows.clear();
  tp.tiles.clear();
  tp.task_off.clear();
  std::vector<std::vector<Tile>> per_rb;
  for (size_t p0 = 0; p0 < pairs.size(); p0 += kRows) {
    RowBlock rb{};
    int lo = 1 << 30, hi = 0;
    for (int r = 0; r < kRows; ++r) {
      if (p0 + r < pairs.size()) {
        rb.i[r] = (int16_t)pairs[p0 + r].i;
        rb.j[r] = (int16_t)pairs[p0 + r].j;
        lo = std::min(lo, pairs[p0 + r].lo);
        hi = std::max(hi, pairs[p0 + r].hi);
      } else {
        rb.i[r] = 0;
        rb.j[r] = 0;
      }
    }
    const int id = (int)tp.rows.size();
    tp.rows.push_back(rb);
    std::vector<Tile> ts;
    for (int c0 = lo; c0 <= hi; c0 += kCols) {
      // keep the tile only if some selected (i, j, l) falls in it
      bool any = false;
      for (int r = 0; r < kRows && !any; ++r) {
        if (!rb.j[r]) continue;
        for (int l : pl[{rb.i[r], rb.j[r]}])
          if (l >= c0 && l < c0 + kCols) { any = true; break; }
      }
      if (any) ts.push_back({id, c0});
    }
    per_rb.push_back(ts);
  }
  // tasks: consecutive row blocks; a row block with more than max_tiles_per_task
  // tiles is split across tasks (its products are then formed once per task)
  tp.task_off.push_back(0);
  int in_task = 0;
  for (auto& ts : per_rb) {
    if (in_task > 0 && in_task + (int)ts.size() > max_tiles_per_task) {
      tp.task_off.push_back((int32_t)tp.tiles.size());
      in_task = 0;
    }
    for (auto& t : ts) {
      if (in_task == max_tiles_per_task) {
        tp.task_off.push_back((int32_t)tp.tiles.size());
        in_task = 0;
      }
      tp.tiles.push_back(t);
      ++in_task;
    }
  }
  if ((int)tp.tiles.size() > tp.task_off.back()) tp.task_off.push_back((int32_t)tp.tiles.size());
  tp.useful = (int64_t)s.tri.size();
  tp.slots = (int64_t)tp.tiles.size() * kRows * kCols;
}

int triangle_min_grid(const ShellGeometry& g, const Tri& t) {
  const int r1 = g.rad[t.a1 - 1], r2 = g.rad[t.a2 - 1], r3 = g.rad[t.a3 - 1];
  const int need = std::max(r1 + r2 + r3, 2 * std::max(r1, std::max(r2, r3))) + 1;
  for (int q = std::max(8, need); q <= 1024; ++q)
    if (grid_size_supported(q)) return q;
  return 0;
}

void choose_grid_classes(const ShellGeometry& g, const Selection& s, bool one_grid,
                         std::vector<GridClassSpec>& out) {
  out.clear();
  const int n_tri = (int)s.tri.size();
  if (one_grid) {
    GridClassSpec c;
    c.g = g.n_est;
    c.s_lo = 0;
    c.n_s = g.n_s;
    c.tri.resize(n_tri);
    for (int t = 0; t < n_tri; ++t) c.tri[t] = t;
    out.push_back(std::move(c));
    return;
  }
  // candidate grids: the supported sizes up to the plan's estimator grid
  std::vector<int> sizes;
  for (int q = 8; q <= g.n_est; ++q)
    if (grid_size_supported(q)) sizes.push_back(q);
  const int K = (int)sizes.size();
  std::vector<std::vector<int32_t>> bucket(K);
  for (int t = 0; t < n_tri; ++t) {
    const int q = std::min(triangle_min_grid(g, s.tri[t]), g.n_est);
    const int b = (int)(std::lower_bound(sizes.begin(), sizes.end(), q) - sizes.begin());
    bucket[std::min(b, K - 1)].push_back(t);
  }
  // cost of one class (seconds): shell transforms ~ shells x G^3, contraction
  // ~ (triangles x G^3 for the matrix unit, distinct (a1, a2) pairs x G^3 for
  // the pair products), plus a fixed cost per class (launches, tails)
  constexpr double kFft = 2.16e-12, kTri = 4.5e-15, kPair = 1.8e-13, kFixed = 4e-5;
  auto cls_cost = [&](int g3i, long long n_t, long long n_p, int n_sh) {
    const double g3 = (double)g3i * g3i * g3i;
    return n_t ? kFft * n_sh * g3 + kTri * (double)n_t * g3 + kPair * (double)n_p * g3 + kFixed : 0.0;
  };
  // best[j + 1]: cheapest cover of buckets 0..j; a class spans buckets i+1..j on grid sizes[j]
  std::vector<double> best(K + 1, 1e300);
  std::vector<int> from(K + 1, -1);
  best[0] = 0.0;
  for (int i = -1; i < K - 1; ++i) {
    if (best[i + 1] >= 1e299) continue;
    std::set<long long> pairs;
    long long n_t = 0;
    int lo = 1 << 30, hi = -1;
    for (int j = i + 1; j < K; ++j) {
      for (int32_t t : bucket[j]) {
        const Tri& q = s.tri[t];
        pairs.insert((long long)q.a1 * 4096 + q.a2);
        lo = std::min(lo, q.a3 - 1);
        hi = std::max(hi, q.a1 - 1);
        ++n_t;
      }
      const double c = best[i + 1] + cls_cost(sizes[j], n_t, (long long)pairs.size(), hi - lo + 1);
      if (c < best[j + 1]) {
        best[j + 1] = c;
        from[j + 1] = i;
      }
    }
  }
  std::vector<std::pair<int, int>> spans;  // (i, j): buckets i+1..j
  for (int j = K - 1; j >= 0;) {
    const int i = from[j + 1];
    spans.push_back({i, j});
    j = i;
  }
  std::reverse(spans.begin(), spans.end());
  for (auto& sp : spans) {
    GridClassSpec c;
    c.g = sizes[sp.second];
    int lo = 1 << 30, hi = -1;
    for (int b = sp.first + 1; b <= sp.second; ++b)
      for (int32_t t : bucket[b]) {
        c.tri.push_back(t);
        lo = std::min(lo, s.tri[t].a3 - 1);
        hi = std::max(hi, s.tri[t].a1 - 1);
      }
    if (c.tri.empty()) continue;
    std::sort(c.tri.begin(), c.tri.end());
    c.s_lo = lo;
    c.n_s = hi - lo + 1;
    out.push_back(std::move(c));
  }
}

void build_mfma_tiles(const Selection& s, int n_shells, MfmaTiling& mt, int max_cols) {
  max_cols = std::max(1, std::min(max_cols, kMaxColTiles));
  std::map<std::pair<int, int>, std::vector<int>> pl;
  for (const Tri& t : s.tri) pl[{t.a1, t.a2}].push_back(t.a3);
  struct P { int i, j, lo, hi; };
  // (window, first block, last block) -> pairs with selected l in that window
  std::map<std::tuple<int, int, int>, std::vector<P>> groups;
  for (auto& kv : pl) {
    std::map<int, std::pair<int, int>> per_window;  // window -> (min l, max l)
    for (int l : kv.second) {
      const int wdw = ((l - 1) / kMCols) / max_cols;
      auto it = per_window.find(wdw);
      if (it == per_window.end()) per_window[wdw] = {l, l};
      else it->second = {std::min(it->second.first, l), std::max(it->second.second, l)};
    }
    for (auto& pw : per_window) {
      const int lo = pw.second.first, hi = pw.second.second;
      groups[{pw.first, (lo - 1) / kMCols, (hi - 1) / kMCols}].push_back({kv.first.first, kv.first.second, lo, hi});
    }
  }
  std::map<std::pair<int, int>, std::vector<P>> spans;  // (first, last column block) -> pairs
  for (auto& g : groups) spans[{std::get<1>(g.first), std::get<2>(g.first)}] = g.second;
  // slots: row blocks of one span + the non-empty column tiles they meet
  struct Slot { MRowBlock rb[kMaxRbPerSlot]; SlotCols sc; };
  auto col_used = [&](const MRowBlock& rb, int col0) {
    for (int r = 0; r < kMRows; ++r) {
      if (!rb.j[r]) continue;
      for (int l : pl[{rb.i[r], rb.j[r]}])
        if (l >= col0 && l < col0 + kMCols) return true;
    }
    return false;
  };
  std::vector<Slot> slots;
  for (auto& sp : spans) {
    auto& ps = sp.second;
    std::sort(ps.begin(), ps.end(), [](const P& a, const P& b) {
      if (a.hi != b.hi) return a.hi < b.hi;
      if (a.lo != b.lo) return a.lo < b.lo;
      if (a.i != b.i) return a.i < b.i;
      return a.j < b.j;
    });
    std::vector<MRowBlock> rbs((ps.size() + kMRows - 1) / kMRows, MRowBlock{});
    for (size_t k = 0; k < ps.size(); ++k) {
      rbs[k / kMRows].i[k % kMRows] = (int16_t)ps[k].i;
      rbs[k / kMRows].j[k % kMRows] = (int16_t)ps[k].j;
    }
    const int n_blocks = sp.first.second - sp.first.first + 1;
    const int per_slot = slot_row_blocks(n_blocks);
    for (size_t b0 = 0; b0 < rbs.size(); b0 += per_slot) {
      Slot sl{};
      sl.sc.n_rb = (int32_t)std::min<size_t>(per_slot, rbs.size() - b0);
      for (int q = 0; q < sl.sc.n_rb; ++q) sl.rb[q] = rbs[b0 + q];
      sl.sc.n = 0;
      for (int c = sp.first.first; c <= sp.first.second; ++c) {
        const int col0 = c * kMCols + 1;
        bool any = false;
        for (int q = 0; q < sl.sc.n_rb && !any; ++q) any = col_used(sl.rb[q], col0);
        if (any) sl.sc.col0[sl.sc.n++] = col0;
      }
      slots.push_back(sl);
    }
  }
  // Fewer work groups per voxel range: every work group of a range stages its
  // rows of every voxel block, so a group is worth saving.  While the slots
  // need one group more than a tighter packing would, merge two slots whose
  // column sets together span at most kMaxColTiles tiles into one slot shape
  // the kernel runs (its row blocks then also meet the other's column tiles:
  // those tiles are computed and never read), fewest wasted tiles first; keep
  // the merges only if they remove a group.
  {
    auto groups_of = [](size_t n) { return (n + kSlotsPerWg - 1) / kSlotsPerWg; };
    auto tiles_of = [](const Slot& sl) { return sl.sc.n * sl.sc.n_rb; };
    auto merge = [&](const Slot& a, const Slot& b, Slot& m) {
      std::set<int> cols(a.sc.col0, a.sc.col0 + a.sc.n);
      cols.insert(b.sc.col0, b.sc.col0 + b.sc.n);
      const int nt = (int)cols.size(), nrb = a.sc.n_rb + b.sc.n_rb;
      if (nt > kMaxColTiles || nrb > kMaxRbPerSlot || nrb > slot_row_blocks(nt) || nt * nrb > kSlotTiles) return false;
      m = Slot{};
      m.sc.n = nt;
      m.sc.n_rb = nrb;
      int k = 0;
      for (int c : cols) m.sc.col0[k++] = c;
      for (int q = 0; q < a.sc.n_rb; ++q) m.rb[q] = a.rb[q];
      for (int q = 0; q < b.sc.n_rb; ++q) m.rb[a.sc.n_rb + q] = b.rb[q];
      return true;
    };
    const size_t g0 = groups_of(slots.size());
    if (g0 > 1) {
      std::vector<Slot> work = slots;
      const size_t want = (g0 - 1) * kSlotsPerWg;
      while (work.size() > want) {
        int bi = -1, bj = -1, best = 1 << 30;
        Slot bm{};
        for (size_t i = 0; i < work.size(); ++i)
          for (size_t j = i + 1; j < work.size(); ++j) {
            Slot m{};
            if (!merge(work[i], work[j], m)) continue;
            const int waste = tiles_of(m) - tiles_of(work[i]) - tiles_of(work[j]);
            if (waste < best) {
              best = waste;
              bi = (int)i;
              bj = (int)j;
              bm = m;
            }
          }
        if (bi < 0) break;
        work[bi] = bm;
        work.erase(work.begin() + bj);
      }
      if (work.size() <= want) slots.swap(work);
    }
  }
  // LDS bank conflicts of the row reads: LDS has 128 banks of 4 bytes and
  // serves a 16-byte read for lanes 0-31, then 32-63; lanes 0-31 hold the 16
  // pairs of one row block at two voxel octets.  The kernel keeps each octet
  // of the fp32 rows in a plane of its own (32 bytes per row, planes an odd
  // number of 16-byte bank groups apart), so two distinct shells of a block
  // collide when they differ by a multiple of 16; equal shells share the
  // read.  Within each slot, swap pairs between its row blocks while that
  // lowers the summed worst collision count of the blocks (the slot's column
  // tiles do not change).
  {
    auto block_cost = [](const MRowBlock& rb) {
      int c = 0;
      for (int f = 0; f < 2; ++f) {
        int mult[16] = {0};
        int seen[kMRows], n_seen = 0;
        for (int r = 0; r < kMRows; ++r) {
          if (!rb.j[r]) continue;
          const int sh = f ? rb.j[r] : rb.i[r];
          bool dup = false;
          for (int k = 0; k < n_seen; ++k) dup = dup || seen[k] == sh;
          if (dup) continue;
          seen[n_seen++] = sh;
          ++mult[sh & 15];
        }
        int m = 0;
        for (int b = 0; b < 16; ++b) m = std::max(m, mult[b]);
        c += std::max(0, m - 1);
      }
      return c;
    };
    for (Slot& sl : slots) {
      if (sl.sc.n_rb < 2) continue;
      for (int pass = 0; pass < 6; ++pass) {
        bool improved = false;
        for (int q0 = 0; q0 < sl.sc.n_rb; ++q0)
          for (int q1 = q0 + 1; q1 < sl.sc.n_rb; ++q1)
            for (int a = 0; a < kMRows; ++a)
              for (int b = 0; b < kMRows; ++b) {
                MRowBlock &x = sl.rb[q0], &y = sl.rb[q1];
                const int before = block_cost(x) + block_cost(y);
                std::swap(x.i[a], y.i[b]);
                std::swap(x.j[a], y.j[b]);
                if (block_cost(x) + block_cost(y) < before) {
                  improved = true;
                } else {
                  std::swap(x.i[a], y.i[b]);
                  std::swap(x.j[a], y.j[b]);
                }
              }
        if (!improved) break;
      }
    }
  }
  // Cost-balanced placement: per 32 voxels a slot costs 3 NT n_rb MFMAs (16
  // cycles each) and n_rb row-operand formations (~32 VALU instructions of 4
  // cycles each); the matrix unit and the vector ALU of a SIMD overlap only in
  // part, so a SIMD's time is close to the sum over its waves, and a work
  // group's time that of its busiest SIMD.  Waves q, q + 4, q + 8 of a group
  // share SIMD q % 4: slots go longest first to the least-loaded (group,
  // SIMD) bin with room, which evens out the SIMDs of every group and so the
  // groups too (groups that share a voxel range then advance together and
  // re-read each chunk from L2).
  {
    auto cost = [](const Slot& sl) { return sl.sc.n_rb * (48 * sl.sc.n + 128); };
    std::vector<Slot> real;
    for (const Slot& sl : slots)
      if (sl.sc.n) real.push_back(sl);
    std::stable_sort(real.begin(), real.end(), [&](const Slot& a, const Slot& b) { return cost(a) > cost(b); });
    constexpr int kSimds = 4, kPerSimd = kSlotsPerWg / kSimds;
    static_assert(kSlotsPerWg % kSimds == 0, "slots per work group must fill the SIMDs evenly");
    const int n_wg = std::max<int>(1, (int)((real.size() + kSlotsPerWg - 1) / kSlotsPerWg));
    const int n_bins = n_wg * kSimds;
    std::vector<std::vector<Slot>> bin(n_bins);
    std::vector<long> load(n_bins, 0);
    for (const Slot& sl : real) {
      int best = -1;
      for (int b = 0; b < n_bins; ++b)
        if ((int)bin[b].size() < kPerSimd && (best < 0 || load[b] < load[best])) best = b;
      bin[best].push_back(sl);
      load[best] += cost(sl);
    }
    // then swaps of slots between bins while they lower the sum over groups
    // of the busiest SIMD's load (the time the groups of one range take)
    for (auto& bv : bin) bv.resize(kPerSimd, Slot{});  // idle slots pad the bins
    auto bin_load = [&](int b) {
      long t = 0;
      for (const Slot& sl : bin[b]) t += sl.sc.n ? cost(sl) : 0;
      return t;
    };
    auto wg_time = [&](int w) {
      long m = 0;
      for (int q = 0; q < kSimds; ++q) m = std::max(m, bin_load(w * kSimds + q));
      return m;
    };
    for (int pass = 0; pass < 8; ++pass) {
      bool improved = false;
      for (int b0 = 0; b0 < n_bins; ++b0)
        for (int b1 = b0 + 1; b1 < n_bins; ++b1)
          for (int k0 = 0; k0 < kPerSimd; ++k0)
            for (int k1 = 0; k1 < kPerSimd; ++k1) {
              const int w0 = b0 / kSimds, w1 = b1 / kSimds;
              const long before = wg_time(w0) + (w1 != w0 ? wg_time(w1) : 0);
              std::swap(bin[b0][k0], bin[b1][k1]);
              const long after = wg_time(w0) + (w1 != w0 ? wg_time(w1) : 0);
              if (after < before) improved = true;
              else std::swap(bin[b0][k0], bin[b1][k1]);
            }
      if (!improved) break;
    }
    // compact placement: busy slots first in each bin, and within a group the
    // SIMDs (interchangeable) ordered by busy slots, so a group with few busy
    // slots uses the lowest positions (which lets the kernel replicate it)
    for (auto& bv : bin)
      std::stable_partition(bv.begin(), bv.end(), [](const Slot& sl) { return sl.sc.n != 0; });
    auto busy = [](const std::vector<Slot>& bv) {
      int k = 0;
      for (const Slot& sl : bv) k += sl.sc.n != 0;
      return k;
    };
    for (int w = 0; w < n_wg; ++w)
      std::stable_sort(bin.begin() + w * kSimds, bin.begin() + (w + 1) * kSimds,
                       [&](const std::vector<Slot>& a, const std::vector<Slot>& b) { return busy(a) > busy(b); });
    slots.assign((size_t)n_wg * kSlotsPerWg, Slot{});
    for (int b = 0; b < n_bins; ++b) {
      const int w = b / kSimds, q = b % kSimds;
      for (size_t k = 0; k < bin[b].size(); ++k) slots[(size_t)w * kSlotsPerWg + q + kSimds * k] = bin[b][k];
    }
  }
  mt.n_wg = (int32_t)(slots.size() / kSlotsPerWg);
  // LDS bank conflicts of the row reads: the 16 lanes served together are
  // the 16 rows of one block (same voxel octet), so the order of the pairs
  // within a block does not matter and is left as built.
  mt.rows.assign((size_t)mt.n_wg * kRbPerWg, MRowBlock{});
  mt.cols.assign((size_t)mt.n_wg * kSlotsPerWg, SlotCols{});
  mt.wg_rows.assign(mt.n_wg, WgRows{});
  mt.tiles = 0;
  mt.max_s = 0;
  std::map<std::tuple<int, int, int>, int32_t> where;
  for (int w = 0; w < mt.n_wg; ++w) {
    int s_lo = 1 << 30, s_hi = -1;
    for (int sidx = 0; sidx < kSlotsPerWg; ++sidx) {
      const Slot& sl = slots[(size_t)w * kSlotsPerWg + sidx];
      mt.cols[(size_t)w * kSlotsPerWg + sidx] = sl.sc;
      mt.tiles += (int64_t)sl.sc.n * sl.sc.n_rb;
      for (int t = 0; t < sl.sc.n; ++t) {
        s_lo = std::min(s_lo, sl.sc.col0[t] - 1);
        s_hi = std::max(s_hi, std::min(sl.sc.col0[t] - 1 + kMCols - 1, n_shells - 1));
      }
      for (int q = 0; q < sl.sc.n_rb; ++q) {
        mt.rows[(size_t)w * kRbPerWg + sidx * kMaxRbPerSlot + q] = sl.rb[q];
        for (int r = 0; r < kMRows; ++r) {
          const int i = sl.rb[q].i[r], j = sl.rb[q].j[r];
          if (!j) continue;
          s_lo = std::min(s_lo, std::min(i, j) - 1);
          s_hi = std::max(s_hi, std::max(i, j) - 1);
          // element of the 16x16 accumulator: row r, column c -> (v, lane)
          for (int t = 0; t < sl.sc.n; ++t)
            for (int l : pl[{i, j}]) {
              const int c = l - sl.sc.col0[t];
              if (c < 0 || c >= kMCols) continue;
              const int lane = c + 16 * (r >> 2), v = r & 3;
              const int tile = w * kTilesPerWg + sidx * kSlotTiles + q * sl.sc.n + t;
              where[{i, j, l}] = tile * kMTileElems + v * 64 + lane;
            }
        }
      }
    }
    WgRows& wr = mt.wg_rows[w];
    if (s_hi < 0) { s_lo = 0; s_hi = -1; }
    wr.s_lo = s_lo;
    wr.s_n = s_hi - s_lo + 1;
    mt.max_s = std::max(mt.max_s, wr.s_n);
  }
  mt.slot_of.resize(s.tri.size());
  for (size_t t = 0; t < s.tri.size(); ++t) mt.slot_of[t] = where.at({s.tri[t].a1, s.tri[t].a2, s.tri[t].a3});
}

void build_adjoint_tables(const Selection& sel, const std::vector<int32_t>& tri_global, int n_s, AdjTables& at) {
  // (n, j) -> l -> triangles
  std::vector<std::map<int, std::map<int, std::vector<int32_t>>>> rows(n_s + 1);
  for (size_t k = 0; k < sel.tri.size(); ++k) {
    const Tri& q = sel.tri[k];
    const int32_t t = tri_global[k];
    rows[q.a1][q.a2][q.a3].push_back(t);
    rows[q.a2][q.a1][q.a3].push_back(t);
    rows[q.a3][q.a1][q.a2].push_back(t);
  }
  std::vector<std::vector<int32_t>> slot_tris;  // per slot (tile * 512 + lane * 8 + i)
  std::vector<long long> cost(n_s + 1, 0);
  at.rbs.clear();
  std::vector<std::pair<int32_t, int32_t>> n_rb(n_s + 1, {0, 0});
  for (int n = 1; n <= n_s; ++n) {
    struct R { int j, lmin, lmax; };
    std::vector<R> rr;
    for (auto& jr : rows[n]) rr.push_back({jr.first, jr.second.begin()->first, jr.second.rbegin()->first});
    std::sort(rr.begin(), rr.end(), [](const R& a, const R& b) {
      return a.lmax != b.lmax ? a.lmax < b.lmax : (a.lmin != b.lmin ? a.lmin < b.lmin : a.j < b.j);
    });
    // rows in that order cut into consecutive blocks of <= kAdjRows rows: the
    // cut with the fewest K tiles (plus 2/5 of a tile per block for its
    // epilogue), by dynamic programming over the cut points
    auto tiles_of = [](int lo, int hi) { return (hi - 1 - (lo - 1) / 8 * 8) / kAdjK + 1; };
    const int nr = (int)rr.size();
    std::vector<double> best(nr + 1, 1e300);
    std::vector<int> cut(nr + 1, 0);
    best[0] = 0.0;
    for (int e = 1; e <= nr; ++e) {
      int lo = 1 << 30, hi = 0;
      for (int s = e - 1; s >= 0 && s >= e - kAdjRows; --s) {
        lo = std::min(lo, rr[s].lmin);
        hi = std::max(hi, rr[s].lmax);
        const double c = best[s] + tiles_of(lo, hi) + 0.4;
        if (c < best[e]) {
          best[e] = c;
          cut[e] = s;
        }
      }
    }
    std::vector<std::pair<int, int>> blocks;   // [first, end) rows
    for (int e = nr; e > 0; e = cut[e]) blocks.push_back({cut[e], e});
    std::reverse(blocks.begin(), blocks.end());
    n_rb[n].first = (int32_t)at.rbs.size();
    for (const auto& bl : blocks) {
      const size_t r0 = (size_t)bl.first;
      const int nrows = bl.second - bl.first;
      AdjRowBlock rb{};
      int lmin = 1 << 30, lmax = 0;
      for (int r = 0; r < kAdjRows; ++r) {
        if (r < nrows) {
          rb.j[r] = (int16_t)rr[r0 + r].j;
          lmin = std::min(lmin, rr[r0 + r].lmin);
          lmax = std::max(lmax, rr[r0 + r].lmax);
        } else {
          rb.j[r] = 0;
        }
      }
      rb.l8 = (int16_t)((lmin - 1) / 8);
      rb.nkt = (int16_t)((lmax - 1 - 8 * rb.l8) / kAdjK + 1);
      rb.w_tile = (int32_t)at.n_tiles;
      at.n_tiles += rb.nkt;
      slot_tris.resize((size_t)at.n_tiles * 512);
      for (int r = 0; r < nrows; ++r) {
        const int j = rr[r0 + r].j;
        for (auto& lt : rows[n][j]) {
          const int k = (lt.first - 1) - 8 * rb.l8;   // K index within the block's tiles
          const int tile = rb.w_tile + k / kAdjK, kk = k % kAdjK;
          const int lane = r + 16 * (kk / 8), i = kk % 8;
          auto& v = slot_tris[(size_t)tile * 512 + lane * 8 + i];
          v.insert(v.end(), lt.second.begin(), lt.second.end());
        }
      }
      cost[n] += 3LL * 8 * rb.nkt + 12;   // MFMAs per chunk, plus the row block's own work
      at.rbs.push_back(rb);
    }
    n_rb[n].second = (int32_t)at.rbs.size();
  }
  at.off.assign(1, 0);
  at.tri.clear();
  for (auto& v : slot_tris) {
    at.tri.insert(at.tri.end(), v.begin(), v.end());
    at.off.push_back((int32_t)at.tri.size());
  }
  // shells to wavefronts: longest first onto the least-loaded of n_wg * kAdjWaves
  long long total = 0, biggest = 0;
  for (int n = 1; n <= n_s; ++n) {
    total += cost[n] + 4;
    biggest = std::max(biggest, cost[n] + 4);
  }
  const long long per_wave = std::max(biggest, (long long)(3 * 8 * 12));
  at.n_wg = (int)std::min<long long>(32, std::max<long long>(1, (total + per_wave * kAdjWaves - 1) / (per_wave * kAdjWaves)));
  const int n_bins = at.n_wg * kAdjWaves;
  std::vector<std::vector<int>> bin(n_bins);
  std::vector<long long> load(n_bins, 0);
  std::vector<int> order;
  for (int n = 1; n <= n_s; ++n) order.push_back(n);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  for (int n : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    bin[k].push_back(n);
    load[k] += cost[n] + 4;
  }
  at.ns.clear();
  at.waves.assign(n_bins, AdjWave{0, 0});
  for (int k = 0; k < n_bins; ++k) {
    std::sort(bin[k].begin(), bin[k].end());
    at.waves[k].e0 = (int32_t)at.ns.size();
    for (int n : bin[k]) at.ns.push_back(AdjN{n, n_rb[n].first, n_rb[n].second});
    at.waves[k].e1 = (int32_t)at.ns.size();
  }
}

}  // namespace bispec
