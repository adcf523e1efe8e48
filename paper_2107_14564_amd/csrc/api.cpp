// C ABI of the estimator (bispec.h): plan construction, memory management,
// the N_tri computation at plan time and the asynchronous run.
//
// A plan splits its triangles into estimator-grid classes (geometry.h,
// choose_grid_classes): class c evaluates the shell fields of its shell range
// on its own grid G_c and contracts its triangles there.  The forward
// transform runs once at N_g; the shell passes run per class; one grouped
// split-bf16 launch contracts every class; a reduction per class writes B in
// the plan's triangle order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bispec.h"
#include "geometry.h"
#include "kernels.h"

using namespace bispec;

// Static run scratch of bispec_run_noalloc: one copy per device, held by every
// GPU the library runs on until the process ends.  Host code never uses this
// name as an address: the per-device address comes from hipGetSymbolAddress.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return set_err(BISPEC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;   // false: a view of memory owned elsewhere (a batch's shared workspace)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned) {
    o.p = nullptr;
    o.bytes = 0;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    owned = true;
  }
  void view(const DevBuf& o) {
    release();
    p = o.p;
    bytes = o.bytes;
    owned = false;
  }
  void view(const DevBuf& o, size_t offset, size_t n) {
    release();
    p = static_cast<unsigned char*>(o.p) + offset;
    bytes = n;
    owned = false;
  }
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

hipError_t dalloc(DevBuf& b, size_t bytes) {
  b.release();
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e == hipSuccess) b.bytes = bytes;
  return e;
}

template <typename T> hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  hipError_t e = dalloc(b, v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// voxel ranges of the MFMA kernel: 256 (a multiple of 8, so all work groups of
// a range share an XCD; groups * 256 work groups fill whole rounds of the 256
// CUs at one work group per CU), fewer for small grids (>= 4 chunks per range)
int n_krange_mfma_for(long long n_vox) {
  const long long cap = std::max(8LL, (n_vox / (64 * 4)) / 8 * 8);
  return (int)std::min(256LL, cap);
}

int n_krange_for(long long groups, long long n_vox) {
  long long k = (1024 + groups - 1) / groups;
  k = ((k + 7) / 8) * 8;
  long long cap = std::max(8LL, (n_vox / 64) / 8 * 8);
  if (k > cap) k = cap;
  if (k < 8) k = 8;
  return (int)k;
}

// candidates of the autotuner: voxel-range counts (multiples of 8) and
// column-tile windows of the MFMA tiling
constexpr int kTuneRanges[] = {64, 128, 256, 512};
constexpr int kTuneCols[] = {8, 4};

std::vector<float2> twiddles32(int m) {
  std::vector<float2> t(m);
  for (int k = 0; k < m; ++k) {
    const double ang = 2.0 * M_PI * (double)k / (double)m;
    t[k] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
  }
  return t;
}

std::vector<double2> twiddles64(int m) {
  std::vector<double2> t(m);
  for (int k = 0; k < m; ++k) {
    const double ang = 2.0 * M_PI * (double)k / (double)m;
    t[k] = make_double2(std::cos(ang), -std::sin(ang));
  }
  return t;
}

// Byte sizes of a plan (sums or maxima over its grid classes).
struct Sizes {
  long long n_tri = 0;
  size_t spec = 0;                              // half spectrum at N_g
  size_t fields32 = 0;                          // every class's float32 fields (resident together)
  size_t a1_32 = 0, a2_32 = 0;                  // largest class's pass intermediates (and the gradient's ball)
  size_t fields64 = 0, a1_64 = 0, a2_64 = 0;    // largest class's float64 unit shells (plan time)
  size_t partial_vec = 0, partial_mfma = 0;     // every class's partials
  size_t grad = 0, tables = 0;
  bool own_workspace = true;   // false: BISPEC_FLAG_NO_WORKSPACE (runs use the static scratch)
  size_t workspace() const { return spec + fields32 + a1_32 + a2_32 + partial_vec + partial_mfma; }
  size_t run_total() const { return (own_workspace ? workspace() : 0) + grad + tables; }
  // planning: the float64 unit shells and their pass buffers exist before the run workspace
  size_t plan_temp() const { return fields64 + a1_64 + a2_64 + n_tri * sizeof(double); }
  size_t plan_peak() const { return std::max(plan_temp() + tables + partial_vec + partial_mfma, run_total()); }
};

// One estimator-grid class: its shells, triangles, tilings, pass tables and
// the offsets of its buffers inside the plan's.
struct GridClass {
  GridClassSpec spec;          // grid, shell range, triangles (plan indices)
  ShellGeometry geo;           // its shells only (n_s = spec.n_s, n_est = spec.g)
  Selection sel;               // its triangles with shells renumbered 1 .. n_s
  TilePlan tiles;              // tasks of <= kMaxTilesPerTask tiles (vector kernels)
  MfmaTiling mfma;             // span-grouped row blocks (MFMA kernel)
  ShellPassPlan pass32;
  long long n_vox = 0, n_tri = 0;
  // voxel-slab streaming: the grid in slabs of slab_x x-planes (the last may
  // be shorter); fields, second-pass intermediates and partials hold one slab
  int slab_x = 0, n_slab = 1;
  long long slab_vox = 0;      // voxels of a full slab (n_vox when the grid is one slab)
  size_t fields32 = 0, fields64 = 0, partial_vec = 0, partial_mfma = 0;
  int n_krange_vec = 8, n_krange_mfma = 8;
  int n_krange_mfma_cap = 8;   // its MFMA partials hold this many ranges
  int max_cols = kMaxColTiles; // column-tile window of its MFMA tiling (a tuned tile shape)
  int tiles_cap = 1;           // its MFMA partials hold this many tiles (times replicas) per range
  int rep = 1;                 // replicas of the one-work-group slot set (split-bf16)
  int tile_stride = 0;         // tiles per voxel range of its MFMA partials
  float tuned_ms = 0.f;        // autotuner: time of the chosen shape (0 = not tuned)
  int tune_source = 0;         // 0 default, 1 timed at plan time, 2 from the tuning cache
  long long f_off = 0;         // element offset of its fields in the plan's F (and G)
  long long pv_off = 0, pm_off = 0;   // element offsets of its vector and MFMA partials
  long long n_terms = 0;
  // adjoint field build on the matrix cores (BISPEC_FLAG_GRAD, split-bf16 plans)
  long long adj_tiles = 0;
  int adj_wg = 0, adj_krange = 8;
  DevBuf tri_index, rows, tile_list, task_off, mfma_rows, mfma_cols, mfma_wgrows, mfma_slot, tri_out, shells,
      x_tiles, y_off, z_off, tw32, g_terms, g_term_off, g_w, adj_rbs, adj_ns, adj_waves, adj_off, adj_tri, adj_W,
      ws_slab;                 // streamed plans: launch groups of a full slab and of the last slab
  WsGroup ws_slab_host[2];
  // x-planes of slab k and its voxels
  int slab_planes(int k) const { return (int)std::min<long long>(slab_x, (long long)spec.g - (long long)k * slab_x); }
  long long slab_voxels(int k) const { return (long long)slab_planes(k) * spec.g * spec.g; }
};

// A class's own geometry: shells s_lo .. s_lo + n_s - 1 of g, renumbered from 1.
ShellGeometry class_geometry(const ShellGeometry& g, const GridClassSpec& c) {
  ShellGeometry h;
  h.n_g = g.n_g;
  h.n_s = c.n_s;
  h.n_est = c.g;
  h.box_l = g.box_l;
  h.w = g.w;
  h.beta = g.beta;
  h.lo2.assign(g.lo2.begin() + c.s_lo, g.lo2.begin() + c.s_lo + c.n_s);
  h.hi2.assign(g.hi2.begin() + c.s_lo, g.hi2.begin() + c.s_lo + c.n_s);
  h.rad.assign(g.rad.begin() + c.s_lo, g.rad.begin() + c.s_lo + c.n_s);
  h.counts.assign(g.counts.begin() + c.s_lo, g.counts.begin() + c.s_lo + c.n_s);
  h.mean_k.assign(g.mean_k.begin() + c.s_lo, g.mean_k.begin() + c.s_lo + c.n_s);
  return h;
}

}  // namespace

struct bispec_plan_s;

struct ManyLane;

// A batch: heterogeneous plans on up to kMaxLanes concurrent lanes (a private
// stream and a run workspace each; a lane runs its members back to back),
// forked from and joined back into the caller's stream, optionally replayed
// from a captured HIP graph.
struct bispec_many_s {
  std::vector<bispec_plan_s*> plans;
  std::vector<int64_t> d_off, b_off;   // prefix sums of N_g^3 and n_tri
  std::vector<int> lane_of;            // member -> lane
  std::vector<ManyLane*> lanes;
  hipEvent_t ev_fork = nullptr;
  hipStream_t cap_stream = nullptr;    // private stream the graph is captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const float* g_delta = nullptr;      // pointers baked into the graph
  double* g_B = nullptr;
  // every member's fields and MFMA partials stay resident (members view them
  // at offsets), so one grouped launch contracts all split-bf16 members
  DevBuf F_all, pm_all, ws_groups;
  std::vector<size_t> f_at, pm_at;     // byte offsets of member i's pieces
  int ws_n = 0, ws_blocks = 0;
  size_t ws_lds = 0;
  // one grouped reduction of every split member's classes after the contraction
  DevBuf red_groups;
  int red_n = 0, red_blocks = 0;
  // cohorts: runs of m >= 2 consecutive identical split-bf16 members (the
  // realisations of one configuration) whose forward transforms and shell
  // passes run as one launch each (grid y = member), with a spectrum
  // and pass intermediates per member; units are the cohorts and the members
  // outside any, in member order, each run on one lane
  struct Unit {
    int i0 = 0, m = 1;                 // members i0 .. i0 + m - 1
    DevBuf spec, a1, a2;               // m > 1: per member, at m times the strides below
    size_t spec_b = 0, a1_b = 0, a2_b = 0;
  };
  std::vector<std::unique_ptr<Unit>> units;
  std::vector<int> unit_lane;
  ~bispec_many_s();
};

struct bispec_plan_s {
  bispec_config cfg{};
  ShellGeometry geo;
  Selection sel;
  std::vector<GridClass> cls;  // grid classes, grids ascending
  ShellPassPlan pass_ball;     // one pseudo-shell covering every shell mode at n_g (last inverse of grad)
  Sizes sz;
  std::vector<int64_t> ntri;
  int precision = BISPEC_PREC_SPLITBF16;
  int slabs = 1;               // x-slabs per grid class (1: whole grids resident)
  bool ran = false;
  bool in_batch = false;       // owned by a bispec_many_t (workspace shared)
  int device = 0;
  // grouped split-bf16 launch over the classes
  std::vector<WsGroup> ws_host;
  int ws_blocks = 0;
  size_t ws_lds = 0;
  // order 4 (the fourth-order polyspectrum): bins, pair tiling and its tables
  bool quad = false;
  std::vector<Quad> quads;
  QuadTiling qt;
  int n_krange4 = 8;
  DevBuf q_pairs, q_rb, q_cb, q_tiles, q_wave, q_slot;
  // grouped matrix-core adjoint build over the classes (GRAD, split-bf16)
  bool adj_mfma = false;
  int adj_groups_n = 0, adj_blocks = 0, adj_max_s = 0;
  // device memory
  DevBuf spec, F, a1, a2, partial, partial_mfma, norm, tw32, ws_groups, adj_groups;
  // gradient workspace (BISPEC_FLAG_GRAD)
  DevBuf G, ball_shells, ball_x, ball_y, ball_z;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  ~bispec_plan_s() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

// Order-4 plans: one grid class over every shell on the estimator grid
// (G > 4 max|m_i|), the quadruples and their pair tiling.
int build_host_quad(const bispec_config* cfg, bispec_plan_s& p) {
  std::string err;
  if (cfg->precision != BISPEC_PREC_SPLITBF16)
    return set_err(BISPEC_EINVAL, "order-4 plans contract in split-bf16 only");
  if (cfg->flags & (BISPEC_FLAG_GRAD | BISPEC_FLAG_NO_WORKSPACE | BISPEC_FLAG_AUTOTUNE))
    return set_err(BISPEC_EINVAL, "order-4 plans take no GRAD, NO_WORKSPACE or AUTOTUNE flag");
  int st = select_quads(*cfg, p.geo, p.quads, err);
  if (st) return set_err(st, err);
  build_quad_tiles(p.quads, p.geo.n_s, p.qt);
  if (p.qt.n_pairs > kMaxQuadPairs)
    return set_err(BISPEC_EINVAL, "order-4 plans stage at most 496 shell pairs (all bins of 31 shells)");
  p.quad = true;
  const long long n = p.geo.n_g;
  Sizes& s = p.sz;
  s.n_tri = (long long)p.quads.size();
  s.spec = (size_t)n * n * (size_t)spec_row(n) * sizeof(float2);
  p.cls.clear();
  p.cls.emplace_back();
  GridClass& c = p.cls.back();
  c.spec.g = p.geo.n_est;
  c.spec.s_lo = 0;
  c.spec.n_s = p.geo.n_s;
  c.geo = class_geometry(p.geo, c.spec);
  const long long g = c.spec.g;
  plan_shell_passes(c.geo, (int)g, false, c.pass32);
  ShellPassPlan p64;
  plan_shell_passes(c.geo, (int)g, true, p64);
  c.n_vox = g * g * g;
  c.fields32 = (size_t)blocked_elems(c.n_vox, c.geo.n_s) * sizeof(float);
  c.fields64 = (size_t)blocked_elems(c.n_vox, c.geo.n_s) * sizeof(double);
  c.f_off = 0;
  s.fields32 = (c.fields32 + 255) / 256 * 256;
  s.a1_32 = (size_t)c.pass32.a1_elems * sizeof(float2);
  s.a2_32 = (size_t)c.pass32.a2_elems * sizeof(float2);
  s.fields64 = c.fields64;
  s.a1_64 = (size_t)p64.a1_elems * sizeof(double2);
  s.a2_64 = (size_t)p64.a2_elems * sizeof(double2);
  p.n_krange4 = n_krange_mfma_for(c.n_vox);
  s.partial_mfma = (size_t)p.n_krange4 * p.qt.n_wg * kTilesPerWg * kMTileElems * sizeof(double);
  s.partial_vec = 0;
  s.tables = p.qt.pair_ij.size() * 4 + p.qt.rb_pairs.size() * 4 + p.qt.cb_pairs.size() * 4 + p.qt.tiles.size() * 4 +
             p.qt.slot_of.size() * 4 + c.pass32.x_tiles.size() * sizeof(int4) + (size_t)s.n_tri * 16 +
             (size_t)(n + g) * 16 + 4096 * 4;
  s.own_workspace = true;
  p.precision = cfg->precision;
  return BISPEC_OK;
}

// slabs > 1: every grid class streams its fields in that many x-slabs (at
// least one plane each): the run buffers then hold one slab.
int build_host(const bispec_config* cfg, bispec_plan_s& p, int slabs = 1) {
  if (!cfg) return set_err(BISPEC_EINVAL, "null config");
  p.slabs = std::max(1, slabs);
  if (p.slabs > 1 && (cfg->flags & BISPEC_FLAG_GRAD))
    return set_err(BISPEC_EINVAL, "BISPEC_FLAG_GRAD needs the whole fields resident (no slab streaming)");
  std::string err;
  p.cfg = *cfg;
  p.cfg.k1_shells = nullptr;
  p.cfg.list = nullptr;
  int st = build_shells(*cfg, p.geo, err);
  if (st) return set_err(st, err);
  if (p.geo.n_s > 256) return set_err(BISPEC_EINVAL, "n_shells > 256 is not supported by the contraction kernels");
  if (cfg->precision == BISPEC_PREC_SPLITBF16 && p.geo.n_s > kMaxSplitShells)
    return set_err(BISPEC_EINVAL, "split-bf16 contraction supports n_shells <= 128");
  if ((cfg->flags & BISPEC_FLAG_NO_WORKSPACE) && (cfg->flags & (BISPEC_FLAG_GRAD | BISPEC_FLAG_AUTOTUNE)))
    return set_err(BISPEC_EINVAL, "BISPEC_FLAG_NO_WORKSPACE excludes BISPEC_FLAG_GRAD and BISPEC_FLAG_AUTOTUNE");
  if (cfg->order == 4) return build_host_quad(cfg, p);
  st = select_triangles(*cfg, p.geo, p.sel, err);
  if (st) return set_err(st, err);
  const long long n = p.geo.n_g;
  Sizes& s = p.sz;
  s.n_tri = (long long)p.sel.tri.size();
  s.spec = (size_t)n * n * (size_t)spec_row(n) * sizeof(float2);
  std::vector<GridClassSpec> specs;
  choose_grid_classes(p.geo, p.sel, cfg->n_est != 0 || (cfg->flags & BISPEC_FLAG_ONE_GRID), specs);
  p.cls.clear();
  p.cls.reserve(specs.size());
  for (GridClassSpec& spc : specs) {
    p.cls.emplace_back();
    GridClass& c = p.cls.back();
    c.spec = std::move(spc);
    c.geo = class_geometry(p.geo, c.spec);
    int first_off = 0;
    if (cfg->ell) {
      // multipoles: weighted copies of the class's shells after its own
      // (fields n_s .. 2 n_s - 1 carry L_ell(mu)), the first side of every
      // triangle on them (Section 3.1 with the weight on shell a1)
      const int ns = c.geo.n_s;
      if (2 * ns > (cfg->precision == BISPEC_PREC_SPLITBF16 ? kMaxSplitShells : 256))
        return set_err(BISPEC_EINVAL, "multipoles: a grid class spans more than 64 shells (split-bf16) or 128 (fp32)");
      auto twice = [ns](auto& v) {
        const auto head = v;
        v.insert(v.end(), head.begin(), head.begin() + ns);
      };
      twice(c.geo.lo2);
      twice(c.geo.hi2);
      twice(c.geo.rad);
      twice(c.geo.counts);
      twice(c.geo.mean_k);
      c.geo.ell.assign(ns, 0);
      c.geo.ell.resize(2 * (size_t)ns, cfg->ell);
      c.geo.n_s = 2 * ns;
      first_off = ns;
    }
    c.sel.tri.reserve(c.spec.tri.size());
    for (int32_t t : c.spec.tri) {
      const Tri& q = p.sel.tri[t];
      c.sel.tri.push_back({q.a1 - c.spec.s_lo + first_off, q.a2 - c.spec.s_lo, q.a3 - c.spec.s_lo});
    }
    build_tiles(c.sel, kMaxTilesPerTask, c.tiles);
    build_mfma_tiles(c.sel, c.geo.n_s, c.mfma);
    const long long g = c.spec.g;
    c.n_vox = g * g * g;
    c.slab_x = (int)std::max<long long>(1, (g + p.slabs - 1) / p.slabs);
    c.n_slab = (int)((g + c.slab_x - 1) / c.slab_x);
    c.slab_vox = (long long)c.slab_x * g * g;
    plan_shell_passes(c.geo, (int)g, false, c.pass32, c.slab_x);
    ShellPassPlan p64;
    plan_shell_passes(c.geo, (int)g, true, p64, c.slab_x);
    c.n_tri = (long long)c.sel.tri.size();
    c.fields32 = (size_t)blocked_elems(c.slab_vox, c.geo.n_s) * sizeof(float);
    c.fields64 = (size_t)blocked_elems(c.slab_vox, c.geo.n_s) * sizeof(double);
    const long long ntasks = (long long)c.tiles.task_off.size() - 1;
    c.n_krange_vec = n_krange_for(ntasks, c.slab_vox);
    c.n_krange_mfma = n_krange_mfma_for(c.slab_vox);
    c.n_krange_mfma_cap = c.n_krange_mfma;
    if (cfg->flags & BISPEC_FLAG_AUTOTUNE)
      for (int k : kTuneRanges)
        if (k <= std::max(8LL, (c.slab_vox / (64 * 4)) / 8 * 8)) c.n_krange_mfma_cap = std::max(c.n_krange_mfma_cap, k);
    c.partial_vec = (size_t)c.n_krange_vec * c.n_tri * sizeof(double);
    c.rep = ws_max_rep(c.mfma);
    c.tile_stride = ws_tile_stride(c.mfma);
    c.tiles_cap = c.rep * c.tile_stride;
    if (cfg->flags & BISPEC_FLAG_AUTOTUNE)
      for (int mc : kTuneCols) {
        MfmaTiling alt;
        build_mfma_tiles(c.sel, c.geo.n_s, alt, mc);
        c.tiles_cap = std::max(c.tiles_cap, ws_max_rep(alt) * ws_tile_stride(alt));
      }
    c.partial_mfma = (size_t)c.n_krange_mfma_cap * c.tiles_cap * kMTileElems * sizeof(double);
    // offsets: fields and partials of the classes back to back (256-byte aligned pieces)
    c.f_off = (long long)(s.fields32 / sizeof(float));
    s.fields32 += (c.fields32 + 255) / 256 * 256;
    c.pv_off = (long long)(s.partial_vec / sizeof(double));
    s.partial_vec += (c.partial_vec + 255) / 256 * 256;
    c.pm_off = (long long)(s.partial_mfma / sizeof(double));
    s.partial_mfma += (c.partial_mfma + 255) / 256 * 256;
    s.a1_32 = std::max(s.a1_32, (size_t)c.pass32.a1_elems * sizeof(float2));
    s.a2_32 = std::max(s.a2_32, (size_t)c.pass32.a2_elems * sizeof(float2));
    s.fields64 = std::max(s.fields64, c.fields64);
    s.a1_64 = std::max(s.a1_64, (size_t)p64.a1_elems * sizeof(double2));
    s.a2_64 = std::max(s.a2_64, (size_t)p64.a2_elems * sizeof(double2));
    s.tables += (size_t)c.geo.n_s * c.geo.n_s * c.geo.n_s * sizeof(int32_t) + c.tiles.rows.size() * sizeof(RowBlock) +
                c.tiles.tiles.size() * sizeof(Tile) + c.mfma.rows.size() * sizeof(MRowBlock) +
                c.mfma.cols.size() * sizeof(SlotCols) + c.mfma.wg_rows.size() * sizeof(WgRows) +
                c.mfma.slot_of.size() * sizeof(int32_t) * 2 + c.pass32.x_tiles.size() * sizeof(int4) +
                (size_t)g * 16 + 4096 * 4;
  }
  if (cfg->flags & BISPEC_FLAG_GRAD) {
    // the gathered spectrum S lives on the modes of shells 1..n_s: one pseudo-shell at n_g
    ShellGeometry ball;
    ball.n_g = p.geo.n_g;
    ball.n_est = p.geo.n_g;
    ball.n_s = 1;
    ball.lo2 = {p.geo.lo2[0]};
    ball.hi2 = {p.geo.hi2[p.geo.n_s - 1]};
    ball.rad = {p.geo.rad[p.geo.n_s - 1]};
    plan_shell_passes(ball, (int)n, false, p.pass_ball);
    s.a1_32 = std::max(s.a1_32, (size_t)p.pass_ball.a1_elems * sizeof(float2));
    s.a2_32 = std::max(s.a2_32, (size_t)p.pass_ball.a2_elems * sizeof(float2));
    s.grad = s.fields32 + (size_t)3 * s.n_tri * (sizeof(int4) + sizeof(double));
  }
  s.tables += (size_t)s.n_tri * 8 + (size_t)n * 16;
  s.own_workspace = !(cfg->flags & BISPEC_FLAG_NO_WORKSPACE);
  p.precision = cfg->precision;
  return BISPEC_OK;
}

// Voxel ranges of a batch member's classes: at most cap (a multiple of 8), so
// that the batch's one grouped launch has a few thousand work groups and
// small partials; recomputes the MFMA partial sizes and offsets.
void cap_mfma_ranges(bispec_plan_s& p, int cap) {
  p.sz.partial_mfma = 0;
  for (GridClass& c : p.cls) {
    c.n_krange_mfma = std::max(8, std::min(c.n_krange_mfma, cap));
    c.n_krange_mfma_cap = std::max(8, std::min(c.n_krange_mfma_cap, cap));
    c.partial_mfma = (size_t)c.n_krange_mfma_cap * c.tiles_cap * kMTileElems * sizeof(double);
    c.pm_off = (long long)(p.sz.partial_mfma / sizeof(double));
    p.sz.partial_mfma += (c.partial_mfma + 255) / 256 * 256;
  }
}

// Voxel ranges of a class's split-bf16 partials (work-group ranges times replicas).
int mfma_ranges(const GridClass& c) { return c.rep * c.n_krange_mfma; }

// The launch group of a class for n_krange work-group ranges.
WsGroup class_group(const GridClass& c, int n_krange) {
  WsGroup w;
  w.f_off = c.f_off;
  w.p_off = c.pm_off;
  w.rows = c.mfma_rows.as<MRowBlock>();
  w.cols = c.mfma_cols.as<SlotCols>();
  w.wg_rows = c.mfma_wgrows.as<WgRows>();
  w.n_vox = c.slab_vox;
  w.n_wg = c.mfma.n_wg;
  w.n_s = c.geo.n_s;
  w.max_s = c.mfma.max_s;
  w.n_krange = n_krange;
  w.rep = c.rep;
  w.tile_stride = c.tile_stride;
  w.block0 = 0;
  return w;
}

// The grouped split-bf16 launch over the plan's classes, for the classes'
// current voxel-range counts; blocks of the costliest groups first.
void build_ws_groups(bispec_plan_s& p) {
  p.ws_host.clear();
  std::vector<int> order;
  for (int k = 0; k < (int)p.cls.size(); ++k)
    if (p.cls[k].n_tri > 0) order.push_back(k);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const GridClass &x = p.cls[a], &y = p.cls[b];
    return (double)x.n_vox / x.n_krange_mfma > (double)y.n_vox / y.n_krange_mfma;
  });
  int block = 0;
  p.ws_lds = 0;
  for (int k : order) {
    GridClass& c = p.cls[k];
    WsGroup w = class_group(c, c.n_krange_mfma);
    w.block0 = block;
    block += w.n_wg * w.n_krange;
    p.ws_lds = std::max(p.ws_lds, bf16x3_lds_bytes(w.max_s, w.rep));
    p.ws_host.push_back(w);
  }
  p.ws_blocks = block;
}

// Append a plan's class groups to a batch table, its fields and partials at
// element offsets f_base (floats) and p_base (doubles) of the batch buffers.
void append_ws_groups(bispec_plan_s& p, long long f_base, long long p_base, std::vector<WsGroup>& out) {
  for (const WsGroup& g : p.ws_host) {
    WsGroup w = g;
    w.f_off += f_base;
    w.p_off += p_base;
    out.push_back(w);
  }
}

ContractArgs contract_args(GridClass& c, double* partial_base) {
  ContractArgs a;
  a.rows = c.rows.as<RowBlock>();
  a.tiles = c.tile_list.as<Tile>();
  a.task_off = c.task_off.as<int32_t>();
  a.n_tasks = (int)c.tiles.task_off.size() - 1;
  a.tri_index = c.tri_index.as<int32_t>();
  a.n_s = c.geo.n_s;
  a.n_vox = c.slab_vox;
  a.n_krange = c.n_krange_vec;
  a.partial = partial_base + c.pv_off;
  a.n_tri = c.n_tri;
  return a;
}

Quad4Args quad_args(bispec_plan_s& p, double* partial) {
  Quad4Args a;
  a.pair_ij = p.q_pairs.as<int32_t>();
  a.rb_pairs = p.q_rb.as<int32_t>();
  a.cb_pairs = p.q_cb.as<int32_t>();
  a.tiles = p.q_tiles.as<int4>();
  a.wave_t0 = p.q_wave.as<int32_t>();
  a.n_pairs = p.qt.n_pairs;
  a.n_s = p.geo.n_s;
  a.n_wg = p.qt.n_wg;
  a.n_krange = p.n_krange4;
  a.n_vox = p.cls[0].n_vox;
  a.partial = partial;
  return a;
}

ShellLaunch shell_launch(const ShellPassPlan& pp, const DevBuf& shells, const DevBuf& xt, const DevBuf& yo,
                         const DevBuf& zo, int n_s, int spec_n) {
  ShellLaunch L;
  L.n_shells = n_s;
  L.spec_n = spec_n;
  L.shells = shells.as<ShellDev>();
  L.x_tiles = xt.as<int4>();
  L.n_x_tiles = (long long)pp.x_tiles.size();
  L.y_off = yo.as<long long>();
  L.n_y_blocks = pp.y_off.back();
  L.z_off = zo.as<long long>();
  L.n_z_blocks = pp.z_off.back();
  return L;
}

ShellLaunch class_launch(const bispec_plan_s& p, const GridClass& c) {
  return shell_launch(c.pass32, c.shells, c.x_tiles, c.y_off, c.z_off, c.geo.n_s, p.geo.n_g);
}

// The y and z passes of slab k of a class (x-planes k slab_x .. + slab_planes(k)).
ShellLaunch slab_of(ShellLaunch L, const GridClass& c, int k) {
  L.x0 = k * c.slab_x;
  L.x_end = L.x0 + c.slab_planes(k);
  L.n_lines = (long long)c.slab_planes(k) * c.spec.g;
  return L;
}

size_t max_bytes_env() {
  const char* s = std::getenv("BISPEC_MAX_BYTES");
  if (!s || !*s) return 0;
  return (size_t)std::strtoull(s, nullptr, 10);
}

// N_tri from the float64 unit shells (eqs. 2FT, Ntri2) on the GPU, class by
// class on the class grids: N_tri = G_c^-3 sum_y I_a1 I_a2 I_a3.
int compute_ntri(bispec_plan_s& p, hipStream_t st) {
  DevBuf I, a1, a2, sums;
  HIP_TRY(dalloc(I, p.sz.fields64));
  HIP_TRY(dalloc(a1, p.sz.a1_64));
  HIP_TRY(dalloc(a2, p.sz.a2_64));
  HIP_TRY(dalloc(sums, (size_t)p.sz.n_tri * sizeof(double)));
  // per-class pass tables stay alive until the stream has drained
  std::vector<DevBuf> keep;
  keep.reserve(p.cls.size() * 5);
  std::vector<double> denom(p.sz.n_tri, 1.0);
  for (GridClass& c : p.cls) {
    const int g = c.spec.g;
    ShellPassPlan pp;
    plan_shell_passes(c.geo, g, true, pp, c.slab_x);   // A2 and the y/z blocks of one slab (a2_64 is that size)
    DevBuf shells, xt, yo, zo, tw;
    HIP_TRY(upload(shells, pp.shells, st));
    HIP_TRY(upload(xt, pp.x_tiles, st));
    HIP_TRY(upload(yo, pp.y_off, st));
    HIP_TRY(upload(zo, pp.z_off, st));
    HIP_TRY(upload(tw, twiddles64(g), st));
    ShellLaunch L = shell_launch(pp, shells, xt, yo, zo, c.geo.n_s, p.geo.n_g);
    if (c.n_slab == 1) {
      HIP_TRY(launch_unit_shells(a1.as<double2>(), a2.as<double2>(), I.as<double>(), L, g, tw.as<double2>(), st));
      HIP_TRY(launch_contract_fp64(I.as<double>(), contract_args(c, p.partial.as<double>()), st));
      HIP_TRY(launch_reduce(p.partial.as<double>() + c.pv_off, c.n_krange_vec, c.n_tri, c.n_tri, nullptr, nullptr,
                            c.tri_out.as<int32_t>(), sums.as<double>(), st));
    } else {
      // streamed: the x pass once, then per x-slab the y and z passes, the
      // contraction of the slab's voxels and its sums added in slab order
      HIP_TRY(launch_inv_x_unit_f64(a1.as<double2>(), L, g, tw.as<double2>(), st));
      for (int k = 0; k < c.n_slab; ++k) {
        const ShellLaunch Lk = slab_of(L, c, k);
        HIP_TRY(launch_inv_y_f64(a1.as<double2>(), a2.as<double2>(), Lk, g, tw.as<double2>(), st));
        HIP_TRY(launch_c2r_f64(a2.as<double2>(), I.as<double>(), Lk, g, tw.as<double2>(), st));
        ContractArgs ca = contract_args(c, p.partial.as<double>());
        ca.n_vox = c.slab_voxels(k);
        HIP_TRY(launch_contract_fp64(I.as<double>(), ca, st));
        HIP_TRY(launch_reduce(p.partial.as<double>() + c.pv_off, c.n_krange_vec, c.n_tri, c.n_tri, nullptr, nullptr,
                              c.tri_out.as<int32_t>(), sums.as<double>(), st, k > 0));
      }
    }
    for (int32_t t : c.spec.tri) denom[t] = (double)c.n_vox;
    keep.push_back(std::move(shells));
    keep.push_back(std::move(xt));
    keep.push_back(std::move(yo));
    keep.push_back(std::move(zo));
    keep.push_back(std::move(tw));
  }
  std::vector<double> h(p.sz.n_tri);
  HIP_TRY(hipMemcpyAsync(h.data(), sums.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  p.ntri.resize(p.sz.n_tri);
  // the float64 grid sum of a count of n carries a rounding error of about
  // 1e-13 n at G = 1024 (unit fields of ~1e6 modes, strong cancellation):
  // accept |v - round(v)| <= 1e-3 + 4e-12 |v|, far below 1/2 for any count
  double worst = 0.0;
  long long worst_t = -1;
  for (long long t = 0; t < p.sz.n_tri; ++t) {
    const double v = h[t] / denom[t];
    const double r = std::nearbyint(v);
    const double excess = std::fabs(v - r) - (1e-3 + 4e-12 * std::fabs(v));
    if (worst_t < 0 || excess > worst) {
      worst = excess;
      worst_t = t;
    }
    p.ntri[t] = (int64_t)r;
  }
  if (worst > 0.0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "N_tri sum of triangle %lld is %.6f beyond its rounding tolerance from an integer",
                  worst_t, worst);
    return set_err(BISPEC_EPREC, buf);
  }
  return BISPEC_OK;
}

// N_quad from the float64 unit shells (eq. 2FT) on the estimator grid:
// N_quad = G^-3 sum_y I_a1 I_a2 I_a3 I_a4, rounded and checked.
int compute_nquad(bispec_plan_s& p, hipStream_t st) {
  GridClass& c = p.cls[0];
  const int g = c.spec.g;
  DevBuf I, a1, a2, sums, shells, xt, yo, zo, tw;
  HIP_TRY(dalloc(I, p.sz.fields64));
  HIP_TRY(dalloc(a1, p.sz.a1_64));
  HIP_TRY(dalloc(a2, p.sz.a2_64));
  HIP_TRY(dalloc(sums, (size_t)p.sz.n_tri * sizeof(double)));
  ShellPassPlan pp;
  plan_shell_passes(c.geo, g, true, pp);
  HIP_TRY(upload(shells, pp.shells, st));
  HIP_TRY(upload(xt, pp.x_tiles, st));
  HIP_TRY(upload(yo, pp.y_off, st));
  HIP_TRY(upload(zo, pp.z_off, st));
  HIP_TRY(upload(tw, twiddles64(g), st));
  ShellLaunch L = shell_launch(pp, shells, xt, yo, zo, c.geo.n_s, p.geo.n_g);
  HIP_TRY(launch_unit_shells(a1.as<double2>(), a2.as<double2>(), I.as<double>(), L, g, tw.as<double2>(), st));
  HIP_TRY(launch_contract4_f64(I.as<double>(), quad_args(p, p.partial_mfma.as<double>()), st));
  HIP_TRY(launch_reduce(p.partial_mfma.as<double>(), p.n_krange4, (long long)p.qt.n_wg * kTilesPerWg * kMTileElems,
                        p.sz.n_tri, p.q_slot.as<int32_t>(), nullptr, nullptr, sums.as<double>(), st));
  std::vector<double> h(p.sz.n_tri);
  HIP_TRY(hipMemcpyAsync(h.data(), sums.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  p.ntri.resize(p.sz.n_tri);
  double worst = 0.0;
  long long worst_t = -1;
  for (long long t = 0; t < p.sz.n_tri; ++t) {
    const double v = h[t] / (double)c.n_vox;
    const double r = std::nearbyint(v);
    if (std::fabs(v - r) > worst) {
      worst = std::fabs(v - r);
      worst_t = t;
    }
    p.ntri[t] = (int64_t)r;
  }
  if (worst > 1e-3) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "N_quad sum of bin %lld is %.6f from an integer", worst_t, worst);
    return set_err(BISPEC_EPREC, buf);
  }
  return BISPEC_OK;
}

// Device side of an order-4 plan.
int plan_build_quad(bispec_plan_s& p, hipStream_t s) {
#define PLAN_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return set_err(BISPEC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
  PLAN_HIP(hipGetDevice(&p.device));
  PLAN_HIP(upload(p.q_pairs, p.qt.pair_ij, s));
  PLAN_HIP(upload(p.q_rb, p.qt.rb_pairs, s));
  PLAN_HIP(upload(p.q_cb, p.qt.cb_pairs, s));
  PLAN_HIP(upload(p.q_tiles, p.qt.tiles, s));
  PLAN_HIP(upload(p.q_wave, p.qt.wave_t0, s));
  PLAN_HIP(upload(p.q_slot, p.qt.slot_of, s));
  PLAN_HIP(dalloc(p.partial_mfma, p.sz.partial_mfma));
  PLAN_HIP(prepare_contract4());
  int st = compute_nquad(p, s);
  if (st) return st;
  GridClass& c = p.cls[0];
  PLAN_HIP(upload(c.shells, c.pass32.shells, s));
  PLAN_HIP(upload(c.x_tiles, c.pass32.x_tiles, s));
  PLAN_HIP(upload(c.y_off, c.pass32.y_off, s));
  PLAN_HIP(upload(c.z_off, c.pass32.z_off, s));
  PLAN_HIP(upload(c.tw32, twiddles32(c.spec.g), s));
  const int n = p.geo.n_g;
  PLAN_HIP(upload(p.tw32, twiddles32(n), s));
  // T = (dV N^{3/2})^4 sum_y F_s F_s F_s F_s / (V N_quad G^3)
  const double V = p.geo.box_l * p.geo.box_l * p.geo.box_l;
  const double dV = V / ((double)n * n * n);
  const double cc = dV * dV * dV * dV * std::pow((double)n, 6.0) / (V * (double)c.n_vox);
  std::vector<double> norm(p.sz.n_tri);
  for (long long t = 0; t < p.sz.n_tri; ++t) norm[t] = p.ntri[t] > 0 ? cc / (double)p.ntri[t] : NAN;
  PLAN_HIP(upload(p.norm, norm, s));
  PLAN_HIP(dalloc(p.spec, p.sz.spec));
  PLAN_HIP(dalloc(p.a1, p.sz.a1_32));
  PLAN_HIP(dalloc(p.a2, p.sz.a2_32));
  PLAN_HIP(dalloc(p.F, p.sz.fields32));
  PLAN_HIP(dalloc(p.partial, 16));
  if (p.cfg.flags & BISPEC_FLAG_STAGE_TIMING)
    for (auto& e : p.ev) PLAN_HIP(hipEventCreate(&e));
  PLAN_HIP(prepare_forward());
  PLAN_HIP(hipStreamSynchronize(s));
#undef PLAN_HIP
  return BISPEC_OK;
}

int check_memory(size_t need) {
  size_t free_b = 0, total_b = 0;
  hipError_t e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return set_err(BISPEC_EHIP, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
  const size_t cap = max_bytes_env();
  if (need > free_b || (cap && need > cap)) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "plan needs %.3f GB of device memory; %.3f GB free%s", need / 1e9, free_b / 1e9,
                  cap ? " (or above BISPEC_MAX_BYTES)" : "");
    return set_err(BISPEC_ENOMEM, buf);
  }
  return BISPEC_OK;
}

// The run workspace of a plan: its own buffers, or views of a batch's shared ones.
struct Workspace {
  DevBuf spec, F, a1, a2, partial, partial_mfma;
};

// Byte offsets of one pass's buffers in the static scratch (256-byte aligned).
struct ScratchLayout {
  size_t spec, a1, a2, F, partial, partial_mfma, total;
};

ScratchLayout scratch_layout(const Sizes& z) {
  ScratchLayout l;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o += (bytes + 255) / 256 * 256;
    return at;
  };
  l.spec = take(z.spec);
  l.a1 = take(z.a1_32);
  l.a2 = take(z.a2_32);
  l.F = take(z.fields32);
  l.partial = take(z.partial_vec);
  l.partial_mfma = take(z.partial_mfma);
  l.total = o;
  return l;
}

// Device address of the static scratch on device dev (looked up once per
// device, with that device current).
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

int scratch_base(int dev, void** out) {
  if (dev < 0 || dev >= kMaxScratchDevices) return set_err(BISPEC_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_err(BISPEC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BISPEC_OK;
}

}  // namespace

struct ManyLane {
  Workspace ws;
  hipStream_t stream = nullptr;
  hipEvent_t ev_join = nullptr;
  ~ManyLane() {
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

constexpr int kMaxLanes = 4;

hipError_t take_workspace(bispec_plan_s& p, const Workspace* shared, bool fields) {
  if (shared) {
    // a batch member: lane buffers (spectrum, pass intermediates, vector
    // partials) shared; its fields and MFMA partials are its own pieces of the
    // batch's resident buffers (views set before plan_build)
    if (!fields) {
      p.partial.view(shared->partial);
    } else {
      p.spec.view(shared->spec);
      p.a1.view(shared->a1);
      p.a2.view(shared->a2);
    }
    return hipSuccess;
  }
  hipError_t e = hipSuccess;
  if (!fields) {
    e = dalloc(p.partial_mfma, p.sz.partial_mfma);
    if (e == hipSuccess) e = dalloc(p.partial, p.sz.partial_vec);
  } else {
    e = dalloc(p.spec, p.sz.spec);
    if (e == hipSuccess) e = dalloc(p.a1, p.sz.a1_32);
    if (e == hipSuccess) e = dalloc(p.a2, p.sz.a2_32);
    if (e == hipSuccess) e = dalloc(p.F, p.sz.fields32);
  }
  return e;
}

// Device buffers one pass writes: the plan's own workspace (or a batch lane's),
// or pieces of the static scratch array (bispec_run_noalloc).
struct RunBufs {
  float2 *spec = nullptr, *a1 = nullptr, *a2 = nullptr;
  float* F = nullptr;
  double *partial = nullptr, *partial_mfma = nullptr;
};

RunBufs own_bufs(bispec_plan_s& p) {
  RunBufs b;
  b.spec = p.spec.as<float2>();
  b.a1 = p.a1.as<float2>();
  b.a2 = p.a2.as<float2>();
  b.F = p.F.as<float>();
  b.partial = p.partial.as<double>();
  b.partial_mfma = p.partial_mfma.as<double>();
  return b;
}

// The forward transform and shell passes of one pass (batch lanes).
int run_fields(bispec_plan_s& p, const RunBufs& w, const float* delta, hipStream_t s) {
  HIP_TRY(launch_forward(delta, w.spec, p.geo.n_g, (float)p.geo.beta, p.tw32.as<float2>(), s));
  for (GridClass& c : p.cls)
    HIP_TRY(launch_data_shells(w.spec, w.a1, w.a2, w.F + c.f_off, class_launch(p, c), c.spec.g, c.tw32.as<float2>(),
                               s));
  return BISPEC_OK;
}

// The vector (fp32) contraction and its reductions.
int run_contract_fp32(bispec_plan_s& p, const RunBufs& w, double* B, hipStream_t s) {
  for (GridClass& c : p.cls) HIP_TRY(launch_contract_fp32(w.F + c.f_off, contract_args(c, w.partial), s));
  for (GridClass& c : p.cls)
    HIP_TRY(launch_reduce(w.partial + c.pv_off, c.n_krange_vec, c.n_tri, c.n_tri, nullptr, p.norm.as<double>(),
                          c.tri_out.as<int32_t>(), B, s));
  return BISPEC_OK;
}

// A streamed pass after the forward transform: per class the x pass once,
// then per x-slab the y and z passes into the one-slab field buffer, the
// slab's contraction (split-bf16: one group for a full and one for the last
// slab; fp32: the vector kernels on the slab's voxels) and its reduction
// added into B in slab order.
int run_streamed(bispec_plan_s& p, const RunBufs& w, double* B, hipStream_t s) {
  for (GridClass& c : p.cls) {
    const ShellLaunch L = class_launch(p, c);
    const int g = c.spec.g;
    HIP_TRY(launch_inv_x_f32(w.spec, w.a1, L, g, c.tw32.as<float2>(), s));
    for (int k = 0; k < c.n_slab; ++k) {
      const ShellLaunch Lk = slab_of(L, c, k);
      HIP_TRY(launch_inv_y_f32(w.a1, w.a2, Lk, g, c.tw32.as<float2>(), s));
      HIP_TRY(launch_c2r_f32(w.a2, w.F + c.f_off, Lk, g, c.tw32.as<float2>(), s));
      if (p.precision == BISPEC_PREC_FP32) {
        ContractArgs ca = contract_args(c, w.partial);
        ca.n_vox = c.slab_voxels(k);
        HIP_TRY(launch_contract_fp32(w.F + c.f_off, ca, s));
        HIP_TRY(launch_reduce(w.partial + c.pv_off, c.n_krange_vec, c.n_tri, c.n_tri, nullptr, p.norm.as<double>(),
                              c.tri_out.as<int32_t>(), B, s, k > 0));
      } else {
        const bool last = k + 1 == c.n_slab && c.slab_planes(k) != c.slab_x;
        const WsGroup& grp = c.ws_slab_host[last ? 1 : 0];
        HIP_TRY(launch_contract_bf16x3(w.F, w.partial_mfma, c.ws_slab.as<WsGroup>() + (last ? 1 : 0), 1,
                                       bf16x3_lds_bytes(grp.max_s, grp.rep), grp.n_wg * grp.n_krange, s));
        HIP_TRY(launch_reduce(w.partial_mfma + c.pm_off, mfma_ranges(c), (long long)c.tile_stride * kMTileElems,
                              c.n_tri, c.mfma_slot.as<int32_t>(), p.norm.as<double>(), c.tri_out.as<int32_t>(), B, s,
                              k > 0));
      }
    }
  }
  return BISPEC_OK;
}

// The four stages of one pass; events only when timing (never under capture).
// A streamed plan interleaves shell passes and contraction per slab: its
// shell stage then holds both and its contraction stage is empty.
int run_core(bispec_plan_s& p, const RunBufs& w, const float* delta, double* B, hipStream_t s, bool timing) {
  const int n = p.geo.n_g;
  if (timing) HIP_TRY(hipEventRecord(p.ev[0], s));
  HIP_TRY(launch_forward(delta, w.spec, n, (float)p.geo.beta, p.tw32.as<float2>(), s));
  if (timing) HIP_TRY(hipEventRecord(p.ev[1], s));
  if (p.slabs > 1) {
    const int st = run_streamed(p, w, B, s);
    if (st) return st;
    if (timing) {
      HIP_TRY(hipEventRecord(p.ev[2], s));
      HIP_TRY(hipEventRecord(p.ev[3], s));
      HIP_TRY(hipEventRecord(p.ev[4], s));
    }
    return BISPEC_OK;
  }
  for (GridClass& c : p.cls)
    HIP_TRY(launch_data_shells(w.spec, w.a1, w.a2, w.F + c.f_off, class_launch(p, c), c.spec.g, c.tw32.as<float2>(),
                               s));
  if (timing) HIP_TRY(hipEventRecord(p.ev[2], s));
  if (p.quad) {
    HIP_TRY(launch_contract4_bf16x3(w.F, quad_args(p, w.partial_mfma), s));
    if (timing) HIP_TRY(hipEventRecord(p.ev[3], s));
    HIP_TRY(launch_reduce(w.partial_mfma, p.n_krange4, (long long)p.qt.n_wg * kTilesPerWg * kMTileElems, p.sz.n_tri,
                          p.q_slot.as<int32_t>(), p.norm.as<double>(), nullptr, B, s));
  } else if (p.precision == BISPEC_PREC_FP32) {
    for (GridClass& c : p.cls) HIP_TRY(launch_contract_fp32(w.F + c.f_off, contract_args(c, w.partial), s));
    if (timing) HIP_TRY(hipEventRecord(p.ev[3], s));
    for (GridClass& c : p.cls)
      HIP_TRY(launch_reduce(w.partial + c.pv_off, c.n_krange_vec, c.n_tri, c.n_tri, nullptr, p.norm.as<double>(),
                            c.tri_out.as<int32_t>(), B, s));
  } else {
    HIP_TRY(launch_contract_bf16x3(w.F, w.partial_mfma, p.ws_groups.as<WsGroup>(), (int)p.ws_host.size(),
                                   p.ws_lds, p.ws_blocks, s));
    if (timing) HIP_TRY(hipEventRecord(p.ev[3], s));
    for (GridClass& c : p.cls)
      HIP_TRY(launch_reduce(w.partial_mfma + c.pm_off, mfma_ranges(c),
                            (long long)c.tile_stride * kMTileElems, c.n_tri, c.mfma_slot.as<int32_t>(),
                            p.norm.as<double>(), c.tri_out.as<int32_t>(), B, s));
  }
  if (timing) HIP_TRY(hipEventRecord(p.ev[4], s));
  return BISPEC_OK;
}

// A cohort's forward transforms and shell passes: one launch per pass for all
// its members (the tables of its first member serve all of them).
int run_fields_cohort(bispec_many_s& m, const bispec_many_s::Unit& u, const float* delta, hipStream_t s) {
  bispec_plan_s& p = *m.plans[u.i0];
  const long long n = p.geo.n_g;
  const long long spec_el = (long long)(u.spec_b / sizeof(float2));
  HIP_TRY(launch_forward(delta + m.d_off[u.i0], u.spec.as<float2>(), (int)n, (float)p.geo.beta, p.tw32.as<float2>(),
                         s, u.m, n * n * n, spec_el));
  for (GridClass& c : p.cls) {
    ShellLaunch L = class_launch(p, c);
    L.n_members = u.m;
    L.spec_stride = spec_el;
    L.a1_stride = (long long)(u.a1_b / sizeof(float2));
    L.a2_stride = (long long)(u.a2_b / sizeof(float2));
    L.f_stride = (long long)((m.f_at[u.i0 + 1] - m.f_at[u.i0]) / sizeof(float));
    HIP_TRY(launch_data_shells(u.spec.as<float2>(), u.a1.as<float2>(), u.a2.as<float2>(), p.F.as<float>() + c.f_off,
                               L, c.spec.g, c.tw32.as<float2>(), s));
  }
  return BISPEC_OK;
}

// Enqueue a batch pass, forked from and joined back into stream s (which may
// be capturing): each unit's forward transforms and shell passes (and, for
// fp32 members, their contraction and reductions) on its lane; then, on s,
// one grouped split-bf16 contraction of every split member's classes and one
// grouped reduction of them into B.
int many_enqueue(bispec_many_s& m, const float* delta, double* B, hipStream_t s) {
  HIP_TRY(hipEventRecord(m.ev_fork, s));
  for (ManyLane* l : m.lanes) HIP_TRY(hipStreamWaitEvent(l->stream, m.ev_fork, 0));
  for (size_t k = 0; k < m.units.size(); ++k) {
    const bispec_many_s::Unit& u = *m.units[k];
    const hipStream_t ls = m.lanes[m.unit_lane[k]]->stream;
    if (u.m > 1) {
      const int st = run_fields_cohort(m, u, delta, ls);
      if (st) return st;
    } else {
      bispec_plan_s& p = *m.plans[u.i0];
      int st = run_fields(p, own_bufs(p), delta + m.d_off[u.i0], ls);
      if (!st && p.precision == BISPEC_PREC_FP32) st = run_contract_fp32(p, own_bufs(p), B + m.b_off[u.i0], ls);
      if (st) return st;
    }
    for (int i = u.i0; i < u.i0 + u.m; ++i) m.plans[i]->ran = true;
  }
  for (ManyLane* l : m.lanes) {
    HIP_TRY(hipEventRecord(l->ev_join, l->stream));
    HIP_TRY(hipStreamWaitEvent(s, l->ev_join, 0));
  }
  if (m.ws_n > 0) {
    HIP_TRY(launch_contract_bf16x3(m.F_all.as<float>(), m.pm_all.as<double>(), m.ws_groups.as<WsGroup>(), m.ws_n,
                                   m.ws_lds, m.ws_blocks, s));
    HIP_TRY(launch_reduce_grouped(m.red_groups.as<RedGroup>(), m.red_n, m.red_blocks, B, s));
  }
  return BISPEC_OK;
}

// Upload the grouped-launch table of the classes' current range counts.
int upload_ws_groups(bispec_plan_s& p, hipStream_t s) {
  build_ws_groups(p);
  for (const WsGroup& g : p.ws_host)
    if (!ws_group_ok(g)) return set_err(BISPEC_EINVAL, "a grid class does not fit the split-bf16 kernel");
  HIP_TRY(upload(p.ws_groups, p.ws_host, s));
  if (p.slabs > 1)
    for (GridClass& c : p.cls) {
      // one-group tables of a full slab and of the (shorter) last slab
      for (int q = 0; q < 2; ++q) {
        WsGroup w = class_group(c, c.n_krange_mfma);
        w.n_vox = q == 0 ? c.slab_vox : c.slab_voxels(c.n_slab - 1);
        if (!ws_group_ok(w)) return set_err(BISPEC_EINVAL, "a slab does not fit the split-bf16 kernel");
        c.ws_slab_host[q] = w;
      }
      HIP_TRY(upload(c.ws_slab, std::vector<WsGroup>(c.ws_slab_host, c.ws_slab_host + 2), s));
    }
  return BISPEC_OK;
}

// Tuning cache: JSON lines {"key": "<hex>", "max_cols": c, "n_krange": k, "ms": t}
// in the file named by BISPEC_TUNE_CACHE (none: no cache).  The key hashes
// what the timing depends on: the class grid, its shells and triangles.
unsigned long long class_key(const GridClass& c) {
  unsigned long long h = 1469598103934665603ULL;  // FNV-1a, 64 bit
  auto mix = [&h](long long v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (unsigned long long)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ULL;
    }
  };
  mix(c.spec.g);
  mix(c.geo.n_s);
  mix((long long)c.sel.tri.size());
  for (const Tri& t : c.sel.tri) mix(((long long)t.a1 << 32) | ((long long)t.a2 << 16) | t.a3);
  return h;
}

std::mutex g_tune_mu;

bool tune_cache_get(unsigned long long key, int& max_cols, int& n_krange, float& ms) {
  const char* path = std::getenv("BISPEC_TUNE_CACHE");
  if (!path || !*path) return false;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char want[40], line[512];
  std::snprintf(want, sizeof want, "\"key\": \"%016llx\"", key);
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    if (!std::strstr(line, want)) continue;
    int mc = 0, kr = 0;
    float t = 0.f;
    const char* a = std::strstr(line, "\"max_cols\":");
    const char* b = std::strstr(line, "\"n_krange\":");
    const char* d = std::strstr(line, "\"ms\":");
    if (a && b && d && std::sscanf(a + 11, "%d", &mc) == 1 && std::sscanf(b + 11, "%d", &kr) == 1 &&
        std::sscanf(d + 5, "%f", &t) == 1) {
      max_cols = mc;
      n_krange = kr;
      ms = t;
      found = true;   // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_put(unsigned long long key, const GridClass& c) {
  const char* path = std::getenv("BISPEC_TUNE_CACHE");
  if (!path || !*path) return;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%016llx\", \"grid\": %d, \"n_shells\": %d, \"n_tri\": %lld, \"max_cols\": %d, "
               "\"n_krange\": %d, \"ms\": %.4f}\n", key, c.spec.g, c.geo.n_s, c.n_tri, c.max_cols, c.n_krange_mfma,
               c.tuned_ms);
  std::fclose(f);
}

// Rebuild a class's MFMA tiling for a column-tile window and upload its tables.
hipError_t retile_class(GridClass& c, int max_cols, hipStream_t s) {
  if (c.max_cols == max_cols) return hipSuccess;
  c.mfma = MfmaTiling();
  build_mfma_tiles(c.sel, c.geo.n_s, c.mfma, max_cols);
  c.max_cols = max_cols;
  c.rep = ws_max_rep(c.mfma);
  c.tile_stride = ws_tile_stride(c.mfma);
  hipError_t e = upload(c.mfma_rows, c.mfma.rows, s);
  if (e == hipSuccess) e = upload(c.mfma_cols, c.mfma.cols, s);
  if (e == hipSuccess) e = upload(c.mfma_wgrows, c.mfma.wg_rows, s);
  if (e == hipSuccess) e = upload(c.mfma_slot, c.mfma.slot_of, s);
  return e;
}

// Autotuner: per class, the column-tile window of its MFMA tiling and the
// voxel-range count of its contraction, each candidate timed alone on
// pseudo-random fields in the plan's own field buffer; choices are read from
// and written to the tuning cache.
int autotune_mfma(bispec_plan_s& p, hipStream_t s) {
  if (p.precision != BISPEC_PREC_SPLITBF16) return BISPEC_OK;
  HIP_TRY(launch_fill_random(p.F.as<float>(), (long long)(p.sz.fields32 / sizeof(float)), 0x5eedULL, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int st = BISPEC_OK;
  DevBuf one;
  for (GridClass& c : p.cls) {
    if (c.n_tri == 0) continue;
    const unsigned long long key = class_key(c);
    int mc_c = 0, kr_c = 0;
    float ms_c = 0.f;
    if (tune_cache_get(key, mc_c, kr_c, ms_c) && mc_c >= 1 && mc_c <= kMaxColTiles && kr_c >= 8 &&
        kr_c % 8 == 0 && kr_c <= c.n_krange_mfma_cap) {
      hipError_t e = retile_class(c, mc_c, s);
      if (e != hipSuccess) { st = set_err(BISPEC_EHIP, std::string("autotune: ") + hipGetErrorString(e)); break; }
      if (c.rep * c.tile_stride <= c.tiles_cap) {
        c.n_krange_mfma = kr_c;
        c.tuned_ms = ms_c;
        c.tune_source = 2;
        continue;
      }
    }
    float best = 1e30f;
    int best_k = c.n_krange_mfma, best_mc = c.max_cols;
    // range candidates: the tuner's sizes that fit the class's partials, and its default
    std::vector<int> ranges;
    for (int k : kTuneRanges)
      if (k <= c.n_krange_mfma_cap) ranges.push_back(k);
    if (std::find(ranges.begin(), ranges.end(), c.n_krange_mfma) == ranges.end()) ranges.push_back(c.n_krange_mfma);
    for (int mc : kTuneCols) {
      hipError_t e = retile_class(c, mc, s);
      if (e != hipSuccess) { st = set_err(BISPEC_EHIP, std::string("autotune: ") + hipGetErrorString(e)); break; }
      if (c.rep * c.tile_stride > c.tiles_cap) continue;
      for (int k : ranges) {
        const WsGroup w = class_group(c, k);
        if (!ws_group_ok(w)) continue;
        e = upload(one, std::vector<WsGroup>{w}, s);
        const int blocks = w.n_wg * k;
        const size_t lds = bf16x3_lds_bytes(w.max_s, w.rep);
        if (e == hipSuccess)
          e = launch_contract_bf16x3(p.F.as<float>(), p.partial_mfma.as<double>(), one.as<WsGroup>(), 1, lds, blocks,
                                     s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < 3 && e == hipSuccess; ++r)
          e = launch_contract_bf16x3(p.F.as<float>(), p.partial_mfma.as<double>(), one.as<WsGroup>(), 1, lds, blocks,
                                     s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          st = set_err(BISPEC_EHIP, std::string("autotune: ") + hipGetErrorString(e));
          break;
        }
        if (ms < best) {
          best = ms;
          best_k = k;
          best_mc = mc;
        }
      }
      if (st) break;
    }
    if (st) break;
    hipError_t e = retile_class(c, best_mc, s);
    if (e != hipSuccess) { st = set_err(BISPEC_EHIP, std::string("autotune: ") + hipGetErrorString(e)); break; }
    c.n_krange_mfma = best_k;
    c.tuned_ms = best / 3.f;
    c.tune_source = 1;
    tune_cache_put(key, c);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Device side of a plan: tables, N_tri (float64 unit shells), normalisation,
// run workspace (own or shared), gradient tables, events, autotuning.
int plan_build(bispec_plan_s& pr, hipStream_t s, const Workspace* shared) {
  bispec_plan_s* p = &pr;
  {
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) return set_err(BISPEC_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
#define PLAN_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return set_err(BISPEC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
  for (GridClass& c : p->cls) {
    const int ns = c.geo.n_s;
    // triangle index table (i-1, j-1, l-1) -> class triangle
    std::vector<int32_t> idx((size_t)ns * ns * ns, -1);
    for (size_t t = 0; t < c.sel.tri.size(); ++t) {
      const Tri& q = c.sel.tri[t];
      idx[((size_t)(q.a1 - 1) * ns + (q.a2 - 1)) * ns + (q.a3 - 1)] = (int32_t)t;
    }
    PLAN_HIP(upload(c.tri_index, idx, s));
    PLAN_HIP(upload(c.rows, c.tiles.rows, s));
    PLAN_HIP(upload(c.tile_list, c.tiles.tiles, s));
    PLAN_HIP(upload(c.task_off, c.tiles.task_off, s));
    PLAN_HIP(upload(c.mfma_rows, c.mfma.rows, s));
    PLAN_HIP(upload(c.mfma_cols, c.mfma.cols, s));
    PLAN_HIP(upload(c.mfma_wgrows, c.mfma.wg_rows, s));
    PLAN_HIP(upload(c.mfma_slot, c.mfma.slot_of, s));
    PLAN_HIP(upload(c.tri_out, c.spec.tri, s));
  }
  PLAN_HIP(take_workspace(*p, shared, false));
  PLAN_HIP(prepare_contract_vec());
  // N_tri first (largest memory phase), then the run workspace
  int st = compute_ntri(*p, s);
  if (st) return st;
  for (GridClass& c : p->cls) {
    PLAN_HIP(upload(c.shells, c.pass32.shells, s));
    PLAN_HIP(upload(c.x_tiles, c.pass32.x_tiles, s));
    PLAN_HIP(upload(c.y_off, c.pass32.y_off, s));
    PLAN_HIP(upload(c.z_off, c.pass32.z_off, s));
    PLAN_HIP(upload(c.tw32, twiddles32(c.spec.g), s));
  }
  {
    const int n = p->geo.n_g;
    PLAN_HIP(upload(p->tw32, twiddles32(n), s));
    // The fields are F_s = D / (dV N^{3/2}) on G_c^3 points (forward transform
    // scaled by N^{-3/2}); eq. bsfin with the sum over the class grid:
    //   B = (dV N^{3/2})^3 sum_y F_s F_s F_s / (V N_tri G_c^3),
    // times 2 ell + 1 for a multipole
    const double V = p->geo.box_l * p->geo.box_l * p->geo.box_l;
    const double dV = V / ((double)n * n * n);
    std::vector<double> norm(p->sz.n_tri);
    for (const GridClass& c : p->cls) {
      const double cc = (2.0 * p->cfg.ell + 1.0) * dV * dV * dV * std::pow((double)n, 4.5) / (V * (double)c.n_vox);
      for (int32_t t : c.spec.tri) norm[t] = p->ntri[t] > 0 ? cc / (double)p->ntri[t] : NAN;
    }
    PLAN_HIP(upload(p->norm, norm, s));
  }
  if (p->sz.own_workspace) {
    PLAN_HIP(take_workspace(*p, shared, true));
  } else {
    p->partial.release();
    p->partial_mfma.release();
    void* base = nullptr;
    st = scratch_base(p->device, &base);
    if (st) return st;
  }
  if (p->cfg.flags & BISPEC_FLAG_GRAD) {
    PLAN_HIP(dalloc(p->G, p->sz.fields32));
    for (GridClass& c : p->cls) {
      const int ns = c.geo.n_s;
      // terms (t, j, l) of every class shell n: d(F_a1 F_a2 F_a3)/dF_n, t the plan's triangle index
      std::vector<std::vector<int4>> per(ns);
      for (size_t k = 0; k < c.sel.tri.size(); ++k) {
        const Tri& q = c.sel.tri[k];
        const int t = c.spec.tri[k];
        per[q.a1 - 1].push_back(make_int4(t, q.a2 - 1, q.a3 - 1, 0));
        per[q.a2 - 1].push_back(make_int4(t, q.a1 - 1, q.a3 - 1, 0));
        per[q.a3 - 1].push_back(make_int4(t, q.a1 - 1, q.a2 - 1, 0));
      }
      std::vector<int4> terms;
      std::vector<int32_t> off(1, 0);
      for (int m = 0; m < ns; ++m) {
        terms.insert(terms.end(), per[m].begin(), per[m].end());
        off.push_back((int32_t)terms.size());
      }
      c.n_terms = (long long)terms.size();
      PLAN_HIP(upload(c.g_terms, terms, s));
      PLAN_HIP(upload(c.g_term_off, off, s));
      PLAN_HIP(dalloc(c.g_w, terms.size() * sizeof(double)));
    }
    // split-bf16 plans build the adjoint fields on the matrix cores
    p->adj_mfma = p->precision == BISPEC_PREC_SPLITBF16 && p->geo.n_s <= kMaxSplitShells;
    if (p->adj_mfma) {
      std::vector<AdjGroup> groups;
      int block = 0;
      p->adj_max_s = 0;
      for (GridClass& c : p->cls) {
        AdjTables at;
        build_adjoint_tables(c.sel, c.spec.tri, c.geo.n_s, at);
        c.adj_tiles = at.n_tiles;
        c.adj_wg = at.n_wg;
        const long long chunks = c.n_vox / kAdjVox;
        long long kr = ((2048 / c.adj_wg) + 7) / 8 * 8;
        kr = std::min(kr, std::max(8LL, (chunks / 2) / 8 * 8));
        c.adj_krange = (int)std::max(8LL, std::min(kr, 256LL));
        PLAN_HIP(upload(c.adj_rbs, at.rbs, s));
        PLAN_HIP(upload(c.adj_ns, at.ns, s));
        PLAN_HIP(upload(c.adj_waves, at.waves, s));
        PLAN_HIP(upload(c.adj_off, at.off, s));
        PLAN_HIP(upload(c.adj_tri, at.tri, s));
        PLAN_HIP(dalloc(c.adj_W, (size_t)std::max(1LL, at.n_tiles) * 1024 * sizeof(uint16_t)));
        AdjGroup g;
        g.f_off = c.f_off;
        g.rbs = c.adj_rbs.as<AdjRowBlock>();
        g.ns = c.adj_ns.as<AdjN>();
        g.waves = c.adj_waves.as<AdjWave>();
        g.W = c.adj_W.as<uint16_t>();
        g.n_vox = c.n_vox;
        g.n_s = c.geo.n_s;
        g.n_wg = c.adj_wg;
        g.n_krange = c.adj_krange;
        g.block0 = block;
        block += g.n_wg * g.n_krange;
        p->adj_max_s = std::max(p->adj_max_s, g.n_s);
        groups.push_back(g);
      }
      p->adj_groups_n = (int)groups.size();
      p->adj_blocks = block;
      PLAN_HIP(upload(p->adj_groups, groups, s));
      PLAN_HIP(prepare_adjoint_mfma());
    }
    PLAN_HIP(upload(p->ball_shells, p->pass_ball.shells, s));
    PLAN_HIP(upload(p->ball_x, p->pass_ball.x_tiles, s));
    PLAN_HIP(upload(p->ball_y, p->pass_ball.y_off, s));
    PLAN_HIP(upload(p->ball_z, p->pass_ball.z_off, s));
  }
  if (p->cfg.flags & BISPEC_FLAG_STAGE_TIMING)
    for (auto& e : p->ev) PLAN_HIP(hipEventCreate(&e));
  PLAN_HIP(prepare_contract_bf16x3());
  PLAN_HIP(prepare_forward());
  if (p->cfg.flags & BISPEC_FLAG_AUTOTUNE) {
    st = autotune_mfma(*p, s);
    if (st) return st;
  }
  st = upload_ws_groups(*p, s);
  if (st) return st;
  PLAN_HIP(hipStreamSynchronize(s));
#undef PLAN_HIP
  return BISPEC_OK;
}

// The class holding shell n (1-based) on the largest grid.
const GridClass* field_class(const bispec_plan_s& p, int shell) {
  const GridClass* best = nullptr;
  for (const GridClass& c : p.cls)
    if (shell - 1 >= c.spec.s_lo && shell - 1 < c.spec.s_lo + c.spec.n_s && (!best || c.spec.g > best->spec.g))
      best = &c;
  return best;
}

}  // namespace

extern "C" {

const char* bispec_last_error(void) { return g_err.c_str(); }

int bispec_query_triangles(const bispec_config* cfg, int64_t* n_tri, int32_t* abc, double* k1_mu_t,
                           int64_t capacity) {
  if (!cfg || !n_tri) return set_err(BISPEC_EINVAL, "null argument");
  if (cfg->order == 4) return set_err(BISPEC_EINVAL, "an order-4 configuration: use bispec_query_quads");
  std::string err;
  ShellGeometry g;
  int st = build_shells(*cfg, g, err);
  if (st) return set_err(st, err);
  Selection s;
  st = select_triangles(*cfg, g, s, err);
  if (st) return set_err(st, err);
  *n_tri = (int64_t)s.tri.size();
  const int64_t m = std::min<int64_t>(*n_tri, capacity);
  for (int64_t t = 0; t < m; ++t) {
    if (abc) {
      abc[3 * t] = s.tri[t].a1;
      abc[3 * t + 1] = s.tri[t].a2;
      abc[3 * t + 2] = s.tri[t].a3;
    }
    if (k1_mu_t)
      for (int q = 0; q < 3; ++q) k1_mu_t[3 * t + q] = s.k1_mu_t[3 * t + q];
  }
  return BISPEC_OK;
}

int bispec_shell_stats(const bispec_config* cfg, int64_t* counts, double* mean_k) {
  if (!cfg) return set_err(BISPEC_EINVAL, "null config");
  std::string err;
  ShellGeometry g;
  int st = build_shells(*cfg, g, err);
  if (st) return set_err(st, err);
  for (int n = 0; n < g.n_s; ++n) {
    if (counts) counts[n] = g.counts[n];
    if (mean_k) mean_k[n] = g.mean_k[n];
  }
  return BISPEC_OK;
}

int bispec_estimator_grid(const bispec_config* cfg, int32_t* n_est) {
  if (!cfg || !n_est) return set_err(BISPEC_EINVAL, "null argument");
  std::string err;
  ShellGeometry g;
  int st = build_shells(*cfg, g, err);
  if (st) return set_err(st, err);
  *n_est = g.n_est;
  return BISPEC_OK;
}

int bispec_grid_classes(const bispec_config* cfg, int32_t* n_classes, int32_t* grid, int32_t* shell_lo,
                        int32_t* shell_hi, int32_t capacity, int32_t* tri_class) {
  if (!cfg || !n_classes) return set_err(BISPEC_EINVAL, "null argument");
  std::string err;
  ShellGeometry g;
  int st = build_shells(*cfg, g, err);
  if (st) return set_err(st, err);
  if (cfg->order == 4) {  // one grid for every bin
    std::vector<Quad> q;
    st = select_quads(*cfg, g, q, err);
    if (st) return set_err(st, err);
    *n_classes = 1;
    if (capacity > 0) {
      if (grid) grid[0] = g.n_est;
      if (shell_lo) shell_lo[0] = 1;
      if (shell_hi) shell_hi[0] = g.n_s;
    }
    if (tri_class)
      for (size_t t = 0; t < q.size(); ++t) tri_class[t] = 0;
    return BISPEC_OK;
  }
  Selection s;
  st = select_triangles(*cfg, g, s, err);
  if (st) return set_err(st, err);
  std::vector<GridClassSpec> cl;
  choose_grid_classes(g, s, cfg->n_est != 0 || (cfg->flags & BISPEC_FLAG_ONE_GRID), cl);
  *n_classes = (int32_t)cl.size();
  for (int k = 0; k < (int)cl.size(); ++k) {
    if (k < capacity) {
      if (grid) grid[k] = cl[k].g;
      if (shell_lo) shell_lo[k] = cl[k].s_lo + 1;
      if (shell_hi) shell_hi[k] = cl[k].s_lo + cl[k].n_s;
    }
    if (tri_class)
      for (int32_t t : cl[k].tri) tri_class[t] = k;
  }
  return BISPEC_OK;
}

int bispec_contraction_tiles(const bispec_config* cfg, int64_t capacity, int32_t* tile, int32_t* shape) {
  if (cfg && cfg->order == 4) return set_err(BISPEC_EINVAL, "order-4 configurations use the pair tiling");
  bispec_plan_s p;
  int st = build_host(cfg, p);
  if (st) return st;
  int32_t base = 0;
  for (const GridClass& c : p.cls) {
    for (size_t k = 0; k < c.spec.tri.size(); ++k) {
      const int32_t t = c.spec.tri[k];
      if (t >= capacity) continue;
      const int32_t loc = c.mfma.slot_of[k] / kMTileElems;   // tile index within the class
      const SlotCols& sc = c.mfma.cols[loc / kSlotTiles];     // slot = work group * kSlotsPerWg + wave
      if (tile) tile[t] = base + loc;
      if (shape) shape[t] = sc.n * 16 + sc.n_rb;
    }
    base += c.mfma.n_wg * kTilesPerWg;
  }
  return BISPEC_OK;
}

int bispec_workspace_bytes(const bispec_config* cfg, int64_t* run_bytes, int64_t* plan_peak_bytes) {
  bispec_plan_s p;
  int st = build_host(cfg, p);
  if (st) return st;
  if (run_bytes) *run_bytes = (int64_t)p.sz.run_total();
  if (plan_peak_bytes) *plan_peak_bytes = (int64_t)p.sz.plan_peak();
  return BISPEC_OK;
}

constexpr int kMaxSlabs = 1024;   // at most one x-plane per slab of the largest grid

int bispec_plan(const bispec_config* cfg, void* hip_stream, bispec_plan_t* out) {
  if (!out) return set_err(BISPEC_EINVAL, "null output");
  *out = nullptr;
  // x-slabs per grid class: BISPEC_SLABS (at least), doubled while the plan
  // does not fit the device (whole fields first; streaming keeps one slab)
  int slabs = 1;
  if (const char* e = std::getenv("BISPEC_SLABS")) slabs = std::max(1, std::atoi(e));
  const bool streamable = cfg && cfg->order != 4 && !(cfg->flags & BISPEC_FLAG_GRAD);
  if (!streamable) slabs = 1;
  bispec_plan_s* p = nullptr;
  int st = BISPEC_OK;
  for (;;) {
    p = new (std::nothrow) bispec_plan_s();
    if (!p) return set_err(BISPEC_ENOMEM, "host allocation failed");
    st = build_host(cfg, *p, slabs);
    if (st == BISPEC_OK) st = check_memory(p->sz.plan_peak());
    if (st != BISPEC_ENOMEM || !streamable || slabs >= kMaxSlabs) break;
    delete p;
    slabs *= 2;
  }
  if (st == BISPEC_OK)
    st = p->quad ? plan_build_quad(*p, (hipStream_t)hip_stream) : plan_build(*p, (hipStream_t)hip_stream, nullptr);
  if (st != BISPEC_OK) {
    delete p;
    return st;
  }
  *out = p;
  return BISPEC_OK;
}

int bispec_plan_slabs(bispec_plan_t p, int32_t* slabs) {
  if (!p || !slabs) return set_err(BISPEC_EINVAL, "null argument");
  *slabs = p->slabs;
  return BISPEC_OK;
}

int bispec_query_quads(const bispec_config* cfg, int64_t* n_quad, int32_t* abcd, int64_t capacity) {
  if (!cfg || !n_quad) return set_err(BISPEC_EINVAL, "null argument");
  if (cfg->order != 4) return set_err(BISPEC_EINVAL, "not an order-4 configuration");
  std::string err;
  ShellGeometry g;
  int st = build_shells(*cfg, g, err);
  if (st) return set_err(st, err);
  std::vector<Quad> q;
  st = select_quads(*cfg, g, q, err);
  if (st) return set_err(st, err);
  *n_quad = (int64_t)q.size();
  for (int64_t t = 0; t < std::min<int64_t>(*n_quad, capacity); ++t)
    if (abcd) {
      abcd[4 * t] = q[t].a1;
      abcd[4 * t + 1] = q[t].a2;
      abcd[4 * t + 2] = q[t].a3;
      abcd[4 * t + 3] = q[t].a4;
    }
  return BISPEC_OK;
}

int bispec_quads(bispec_plan_t p, int32_t* abcd, int64_t* nquad) {
  if (!p) return set_err(BISPEC_EINVAL, "null plan");
  if (!p->quad) return set_err(BISPEC_EINVAL, "not an order-4 plan");
  for (long long t = 0; t < p->sz.n_tri; ++t) {
    if (abcd) {
      abcd[4 * t] = p->quads[t].a1;
      abcd[4 * t + 1] = p->quads[t].a2;
      abcd[4 * t + 2] = p->quads[t].a3;
      abcd[4 * t + 3] = p->quads[t].a4;
    }
    if (nquad) nquad[t] = p->ntri[t];
  }
  return BISPEC_OK;
}

int bispec_num_triangles(bispec_plan_t p, int64_t* n_tri) {
  if (!p || !n_tri) return set_err(BISPEC_EINVAL, "null argument");
  *n_tri = p->sz.n_tri;
  return BISPEC_OK;
}

int bispec_triangles(bispec_plan_t p, int32_t* abc, double* k1_mu_t, int64_t* ntri) {
  if (!p) return set_err(BISPEC_EINVAL, "null plan");
  if (p->quad) return set_err(BISPEC_EINVAL, "an order-4 plan: use bispec_quads");
  for (long long t = 0; t < p->sz.n_tri; ++t) {
    if (abc) {
      abc[3 * t] = p->sel.tri[t].a1;
      abc[3 * t + 1] = p->sel.tri[t].a2;
      abc[3 * t + 2] = p->sel.tri[t].a3;
    }
    if (k1_mu_t)
      for (int q = 0; q < 3; ++q) k1_mu_t[3 * t + q] = p->sel.k1_mu_t[3 * t + q];
    if (ntri) ntri[t] = p->ntri[t];
  }
  return BISPEC_OK;
}

int bispec_set_precision(bispec_plan_t p, int32_t precision) {
  if (!p) return set_err(BISPEC_EINVAL, "null plan");
  if (precision != BISPEC_PREC_SPLITBF16 && precision != BISPEC_PREC_FP32)
    return set_err(BISPEC_EINVAL, "unknown precision");
  if (precision == BISPEC_PREC_SPLITBF16 && p->geo.n_s > kMaxSplitShells)
    return set_err(BISPEC_EINVAL, "split-bf16 contraction supports n_shells <= 128");
  if (p->quad && precision != BISPEC_PREC_SPLITBF16)
    return set_err(BISPEC_EINVAL, "order-4 plans contract in split-bf16 only");
  p->precision = precision;
  return BISPEC_OK;
}

int bispec_run(bispec_plan_t p, const float* delta, double* B, void* hip_stream) {
  if (!p || !delta || !B) return set_err(BISPEC_EINVAL, "null argument");
  if (p->cfg.flags & BISPEC_FLAG_NO_WORKSPACE)
    return set_err(BISPEC_ESTATE, "plan was made with BISPEC_FLAG_NO_WORKSPACE: run it with bispec_run_noalloc");
  const int st = run_core(*p, own_bufs(*p), delta, B, (hipStream_t)hip_stream,
                          (p->cfg.flags & BISPEC_FLAG_STAGE_TIMING) != 0);
  if (st == BISPEC_OK) p->ran = true;
  return st;
}

int bispec_run_noalloc(bispec_plan_t p, const float* delta, double* B, void* hip_stream) {
  if (!p || !delta || !B) return set_err(BISPEC_EINVAL, "null argument");
  if (p->quad) return set_err(BISPEC_EINVAL, "order-4 plans run with bispec_run");
  const ScratchLayout l = scratch_layout(p->sz);
  if (l.total > kScratchBytes) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "plan needs %.1f MiB of run scratch; the static scratch holds %.0f MiB",
                  l.total / 1048576.0, kScratchBytes / 1048576.0);
    return set_err(BISPEC_EINVAL, buf);
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return set_err(BISPEC_EINVAL, "the plan belongs to another device than the current one");
  void* base = nullptr;
  int st = scratch_base(dev, &base);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  unsigned char* b = static_cast<unsigned char*>(base);
  // the scratch keeps the previous call's contents (of any plan): start from
  // zero, with a fill kernel (no memset node if the caller is capturing)
  HIP_TRY(launch_zero(b, l.total, s));
  RunBufs w;
  w.spec = reinterpret_cast<float2*>(b + l.spec);
  w.a1 = reinterpret_cast<float2*>(b + l.a1);
  w.a2 = reinterpret_cast<float2*>(b + l.a2);
  w.F = reinterpret_cast<float*>(b + l.F);
  w.partial = reinterpret_cast<double*>(b + l.partial);
  w.partial_mfma = reinterpret_cast<double*>(b + l.partial_mfma);
  return run_core(*p, w, delta, B, s, (p->cfg.flags & BISPEC_FLAG_STAGE_TIMING) != 0);
}

int bispec_grad(bispec_plan_t p, const double* gB, float* gdelta, void* hip_stream) {
  if (!p || !gB || !gdelta) return set_err(BISPEC_EINVAL, "null argument");
  if (!(p->cfg.flags & BISPEC_FLAG_GRAD)) return set_err(BISPEC_ESTATE, "plan was made without BISPEC_FLAG_GRAD");
  if (!p->ran) return set_err(BISPEC_ESTATE, "bispec_grad needs a preceding bispec_run");
  hipStream_t s = (hipStream_t)hip_stream;
  const int n = p->geo.n_g;
  // G_n = sum_t gB_t norm_t d(F_a1 F_a2 F_a3)/dF_n on each class's (scaled) fields of the last run:
  // on the matrix cores (split-bf16 plans) or with float64 vector sums (fp32 plans)
  if (p->adj_mfma) {
    for (GridClass& c : p->cls)
      HIP_TRY(launch_adj_weights(gB, p->norm.as<double>(), c.adj_off.as<int32_t>(), c.adj_tri.as<int32_t>(),
                                 c.adj_tiles, c.adj_W.as<uint16_t>(), s));
    HIP_TRY(launch_adjoint_mfma(p->F.as<float>(), p->G.as<float>(), p->adj_groups.as<AdjGroup>(), p->adj_groups_n,
                                p->adj_max_s, p->adj_blocks, s));
  } else {
    for (GridClass& c : p->cls)
      HIP_TRY(launch_gbuild(p->F.as<float>() + c.f_off, gB, p->norm.as<double>(), c.g_terms.as<int4>(), c.n_terms,
                            c.g_term_off.as<int32_t>(), c.geo.n_s, c.n_vox, c.g_w.as<double>(),
                            p->G.as<float>() + c.f_off, s));
  }
  // S = sum_c sum_n mask_n Z DFT_{G_c}(G_n) * N^{-3/2}, gathered into the n_g spectrum buffer
  const float scale = (float)std::pow((double)n, -1.5);
  for (size_t k = 0; k < p->cls.size(); ++k) {
    GridClass& c = p->cls[k];
    HIP_TRY(launch_adjoint_shells(p->G.as<float>() + c.f_off, p->a1.as<float2>(), p->a2.as<float2>(),
                                  p->spec.as<float2>(), class_launch(*p, c), c.spec.g, c.tw32.as<float2>(), scale,
                                  (float)p->geo.beta, k == 0, s));
  }
  // gdelta = unnormalised inverse transform of S on the n_g grid (one pseudo-shell: natural layout)
  ShellLaunch B = shell_launch(p->pass_ball, p->ball_shells, p->ball_x, p->ball_y, p->ball_z, 1, n);
  HIP_TRY(launch_data_shells(p->spec.as<float2>(), p->a1.as<float2>(), p->a2.as<float2>(), gdelta, B, n,
                             p->tw32.as<float2>(), s));
  return BISPEC_OK;
}

int bispec_stage_times(bispec_plan_t p, float* ms, int32_t n) {
  if (!p || !ms || n < 0 || n > 4) return set_err(BISPEC_EINVAL, "bad argument");
  if (!(p->cfg.flags & BISPEC_FLAG_STAGE_TIMING)) return set_err(BISPEC_ESTATE, "plan was made without stage timing");
  if (!p->ran) return set_err(BISPEC_ESTATE, "no run recorded");
  for (int q = 0; q < n; ++q) HIP_TRY(hipEventElapsedTime(&ms[q], p->ev[q], p->ev[q + 1]));
  return BISPEC_OK;
}

int bispec_plan_classes(bispec_plan_t p, int32_t capacity, int32_t* n_classes, int32_t* grid, int32_t* n_krange,
                        int32_t* max_cols, int32_t* n_wg, int32_t* rep, float* tuned_ms, int32_t* tune_source) {
  if (!p || !n_classes) return set_err(BISPEC_EINVAL, "null argument");
  *n_classes = (int32_t)p->cls.size();
  for (int k = 0; k < (int)p->cls.size() && k < capacity; ++k) {
    const GridClass& c = p->cls[k];
    if (grid) grid[k] = c.spec.g;
    if (n_krange) n_krange[k] = p->quad ? p->n_krange4 : c.n_krange_mfma;
    if (max_cols) max_cols[k] = c.max_cols;
    if (n_wg) n_wg[k] = p->quad ? p->qt.n_wg : c.mfma.n_wg;
    if (rep) rep[k] = p->quad ? 1 : c.rep;
    if (tuned_ms) tuned_ms[k] = c.tuned_ms;
    if (tune_source) tune_source[k] = c.tune_source;
  }
  return BISPEC_OK;
}

int bispec_field_grid(bispec_plan_t p, int32_t shell, int32_t* grid) {
  if (!p || !grid) return set_err(BISPEC_EINVAL, "null argument");
  const GridClass* c = (shell >= 1 && shell <= p->geo.n_s) ? field_class(*p, shell) : nullptr;
  if (!c) return set_err(BISPEC_EINVAL, "shell out of range or used by no selected triangle");
  *grid = c->spec.g;
  return BISPEC_OK;
}

int bispec_copy_field(bispec_plan_t p, int32_t shell, float* dst, void* hip_stream) {
  if (!p || !dst) return set_err(BISPEC_EINVAL, "null argument");
  const GridClass* c = (shell >= 1 && shell <= p->geo.n_s) ? field_class(*p, shell) : nullptr;
  if (!c) return set_err(BISPEC_EINVAL, "shell out of range or used by no selected triangle");
  if (!p->ran) return set_err(BISPEC_ESTATE, "no run recorded");
  if (p->slabs > 1) return set_err(BISPEC_ESTATE, "a streamed plan keeps one x-slab of its fields");
  HIP_TRY(launch_unblock(p->F.as<float>() + c->f_off, shell - 1 - c->spec.s_lo, c->geo.n_s, c->n_vox, dst,
                         (hipStream_t)hip_stream));
  return BISPEC_OK;
}

int bispec_copy_class_field(bispec_plan_t p, int32_t cls, int32_t shell, float* dst, void* hip_stream) {
  if (!p || !dst) return set_err(BISPEC_EINVAL, "null argument");
  if (cls < 0 || cls >= (int32_t)p->cls.size()) return set_err(BISPEC_EINVAL, "grid class out of range");
  const GridClass& c = p->cls[cls];
  if (shell - 1 < c.spec.s_lo || shell - 1 >= c.spec.s_lo + c.spec.n_s)
    return set_err(BISPEC_EINVAL, "the class's fields do not cover this shell");
  if (!p->ran) return set_err(BISPEC_ESTATE, "no run recorded");
  if (p->slabs > 1) return set_err(BISPEC_ESTATE, "a streamed plan keeps one x-slab of its fields");
  HIP_TRY(launch_unblock(p->F.as<float>() + c.f_off, shell - 1 - c.spec.s_lo, c.geo.n_s, c.n_vox, dst,
                         (hipStream_t)hip_stream));
  return BISPEC_OK;
}

int bispec_destroy(bispec_plan_t p) {
  if (p && p->in_batch) return set_err(BISPEC_EINVAL, "this plan belongs to a batch (bispec_destroy_many)");
  delete p;
  return BISPEC_OK;
}

int bispec_plan_many(const bispec_config* cfgs, int32_t n, void* hip_stream, bispec_many_t* out) {
  if (!out || !cfgs || n < 1) return set_err(BISPEC_EINVAL, "bad argument");
  *out = nullptr;
  bispec_many_s* m = new (std::nothrow) bispec_many_s();
  if (!m) return set_err(BISPEC_ENOMEM, "host allocation failed");
  auto fail = [&](int code) {
    delete m;
    return code;
  };
  hipStream_t s = (hipStream_t)hip_stream;
  m->d_off.assign(1, 0);
  m->b_off.assign(1, 0);
  size_t ws_spec = 0, ws_a1 = 0, ws_a2 = 0, ws_pv = 0, tables = 0, temp = 0;
  std::vector<double> cost(n);
  long long n_classes = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (cfgs[i].flags & (BISPEC_FLAG_GRAD | BISPEC_FLAG_NO_WORKSPACE))
      return fail(set_err(BISPEC_EINVAL, "batched plans do not take BISPEC_FLAG_GRAD or BISPEC_FLAG_NO_WORKSPACE"));
    if (cfgs[i].order == 4) return fail(set_err(BISPEC_EINVAL, "batched plans are bispectrum plans"));
    bispec_plan_s* p = new (std::nothrow) bispec_plan_s();
    if (!p) return fail(set_err(BISPEC_ENOMEM, "host allocation failed"));
    p->in_batch = true;
    m->plans.push_back(p);
    int st = build_host(&cfgs[i], *p);
    if (st) return fail(st);
    n_classes += (long long)p->cls.size();
  }
  // voxel ranges per class for a few thousand work groups in the grouped launch
  const int range_cap = (int)std::max(8LL, std::min(256LL, (4096 / std::max(1LL, n_classes)) / 8 * 8));
  size_t f_total = 0, pm_total = 0;
  m->f_at.resize(n);
  m->pm_at.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    bispec_plan_s* p = m->plans[i];
    cap_mfma_ranges(*p, range_cap);
    const Sizes& z = p->sz;
    ws_spec = std::max(ws_spec, z.spec);
    ws_a1 = std::max(ws_a1, z.a1_32);
    ws_a2 = std::max(ws_a2, z.a2_32);
    ws_pv = std::max(ws_pv, z.partial_vec);
    m->f_at[i] = f_total;
    f_total += (z.fields32 + 255) / 256 * 256;
    m->pm_at[i] = pm_total;
    pm_total += (z.partial_mfma + 255) / 256 * 256;
    tables += z.tables;
    temp = std::max(temp, z.plan_temp());
    m->d_off.push_back(m->d_off.back() + (int64_t)p->geo.n_g * p->geo.n_g * p->geo.n_g);
    m->b_off.push_back(m->b_off.back() + (int64_t)z.n_tri);
    // run-time estimate of a member's lane work: shell fields written
    double c = 0.0;
    for (const GridClass& k : p->cls) c += (double)k.n_vox * k.geo.n_s;
    cost[i] = c;
  }
  // units: cohorts of identical consecutive members (split-bf16, no autotuning:
  // their tables are then equal) in chunks within kCohortBytes of per-member
  // spectra and pass intermediates, and the other members one by one
  auto r256 = [](size_t v) { return (v + 255) / 256 * 256; };
  auto same = [&](int a, int b) {
    const bispec_config &x = cfgs[a], &y = cfgs[b];
    const bispec_plan_s &pa = *m->plans[a], &pb = *m->plans[b];
    if (pa.precision != BISPEC_PREC_SPLITBF16 || pb.precision != BISPEC_PREC_SPLITBF16) return false;
    if (((x.flags | y.flags) & BISPEC_FLAG_AUTOTUNE) || x.flags != y.flags || pa.slabs != 1 || pb.slabs != 1)
      return false;
    if (x.n_g != y.n_g || x.n_shells != y.n_shells || x.box_l != y.box_l || x.dk != y.dk ||
        x.rsd_beta != y.rsd_beta || x.n_est != y.n_est || x.ell != y.ell)
      return false;
    if (pa.sel.tri.size() != pb.sel.tri.size() || pa.cls.size() != pb.cls.size()) return false;
    for (size_t k = 0; k < pa.sel.tri.size(); ++k) {
      const Tri &u = pa.sel.tri[k], &v = pb.sel.tri[k];
      if (u.a1 != v.a1 || u.a2 != v.a2 || u.a3 != v.a3) return false;
    }
    for (size_t k = 0; k < pa.cls.size(); ++k)
      if (pa.cls[k].spec.g != pb.cls[k].spec.g || pa.cls[k].spec.s_lo != pb.cls[k].spec.s_lo ||
          pa.cls[k].spec.n_s != pb.cls[k].spec.n_s || pa.cls[k].spec.tri != pb.cls[k].spec.tri)
        return false;
    return pa.sz.spec == pb.sz.spec && pa.sz.a1_32 == pb.sz.a1_32 && pa.sz.a2_32 == pb.sz.a2_32 &&
           pa.sz.fields32 == pb.sz.fields32 && pa.sz.partial_mfma == pb.sz.partial_mfma;
  };
  constexpr size_t kCohortBytes = 8ULL << 30;
  constexpr int kCohortMax = 1024;
  auto make_units = [&](bool cohorts) {
    m->units.clear();
    size_t bytes = 0;
    for (int i = 0; i < n;) {
      int j = i + 1;
      if (cohorts)
        while (j < n && same(i, j)) ++j;
      const Sizes& z = m->plans[i]->sz;
      const size_t per = r256(z.spec) + r256(z.a1_32) + r256(z.a2_32);
      const int chunk = (int)std::max<size_t>(1, std::min<size_t>(kCohortMax, kCohortBytes / std::max<size_t>(1, per)));
      for (int k = i; k < j; k += chunk) {
        std::unique_ptr<bispec_many_s::Unit> u(new (std::nothrow) bispec_many_s::Unit());
        if (!u) return (size_t)-1;
        u->i0 = k;
        u->m = std::min(chunk, j - k);
        if (u->m > 1) {
          u->spec_b = r256(z.spec);
          u->a1_b = r256(z.a1_32);
          u->a2_b = r256(z.a2_32);
          bytes += (size_t)u->m * per;
        }
        m->units.push_back(std::move(u));
      }
      i = j;
    }
    return bytes;
  };
  size_t cohort_bytes = make_units(true);
  if (cohort_bytes == (size_t)-1) return fail(set_err(BISPEC_ENOMEM, "host allocation failed"));
  // lanes: as many concurrent workspaces as units, kMaxLanes and memory allow
  const size_t lane_bytes = ws_spec + ws_a1 + ws_a2 + ws_pv;
  size_t free_b = 0, total_b = 0;
  {
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return fail(set_err(BISPEC_EHIP, std::string("hipMemGetInfo: ") + hipGetErrorString(e)));
  }
  const size_t cap = max_bytes_env();
  const size_t avail = cap ? std::min(free_b, cap) : free_b;
  const size_t fixed = f_total + pm_total + tables + temp;
  int n_lanes = std::min<int>(kMaxLanes, (int)m->units.size());
  while (n_lanes > 1 && (size_t)n_lanes * lane_bytes + cohort_bytes + fixed > avail) --n_lanes;
  if (cohort_bytes > 0 && lane_bytes + cohort_bytes + fixed > avail) {
    cohort_bytes = make_units(false);   // no room for per-member workspaces: members one by one
    if (cohort_bytes == (size_t)-1) return fail(set_err(BISPEC_ENOMEM, "host allocation failed"));
    n_lanes = std::min<int>(kMaxLanes, (int)m->units.size());
    while (n_lanes > 1 && (size_t)n_lanes * lane_bytes + fixed > avail) --n_lanes;
  }
  int st = check_memory((size_t)n_lanes * lane_bytes + cohort_bytes + fixed);
  if (st) return fail(st);
  // units to lanes: costliest first onto the least-loaded lane
  {
    const int n_units = (int)m->units.size();
    std::vector<double> ucost(n_units, 0.0);
    for (int k = 0; k < n_units; ++k)
      for (int i = m->units[k]->i0; i < m->units[k]->i0 + m->units[k]->m; ++i) ucost[k] += cost[i];
    std::vector<int> order(n_units);
    for (int k = 0; k < n_units; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ucost[x] > ucost[y]; });
    std::vector<double> load(n_lanes, 0.0);
    m->unit_lane.assign(n_units, 0);
    m->lane_of.assign(n, 0);
    for (int k : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      m->unit_lane[k] = l;
      load[l] += ucost[k];
      for (int i = m->units[k]->i0; i < m->units[k]->i0 + m->units[k]->m; ++i) m->lane_of[i] = l;
    }
  }
  for (auto& u : m->units) {
    if (u->m < 2) continue;
    hipError_t e = dalloc(u->spec, (size_t)u->m * u->spec_b);
    if (e == hipSuccess) e = dalloc(u->a1, (size_t)u->m * u->a1_b);
    if (e == hipSuccess) e = dalloc(u->a2, (size_t)u->m * u->a2_b);
    if (e != hipSuccess) return fail(set_err(BISPEC_EHIP, std::string("batch cohort: ") + hipGetErrorString(e)));
  }
  for (int k = 0; k < n_lanes; ++k) {
    ManyLane* l = new (std::nothrow) ManyLane();
    if (!l) return fail(set_err(BISPEC_ENOMEM, "host allocation failed"));
    m->lanes.push_back(l);
    hipError_t e = dalloc(l->ws.spec, ws_spec);
    if (e == hipSuccess) e = dalloc(l->ws.a1, ws_a1);
    if (e == hipSuccess) e = dalloc(l->ws.a2, ws_a2);
    if (e == hipSuccess) e = dalloc(l->ws.partial, ws_pv);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&l->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&l->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return fail(set_err(BISPEC_EHIP, std::string("batch lane: ") + hipGetErrorString(e)));
  }
  {
    hipError_t e = dalloc(m->F_all, f_total);
    if (e == hipSuccess) e = dalloc(m->pm_all, pm_total);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming);
    if (e != hipSuccess) return fail(set_err(BISPEC_EHIP, std::string("batch buffers: ") + hipGetErrorString(e)));
  }
  // the plans take views of their lane's workspace and of their pieces of the
  // resident field and partial buffers
  std::vector<WsGroup> groups;
  for (int32_t i = 0; i < n; ++i) {
    bispec_plan_s* p = m->plans[i];
    p->F.view(m->F_all, m->f_at[i], p->sz.fields32);
    p->partial_mfma.view(m->pm_all, m->pm_at[i], p->sz.partial_mfma);
    st = plan_build(*p, s, &m->lanes[m->lane_of[i]]->ws);
    if (st) return fail(st);
    if (p->precision != BISPEC_PREC_FP32)
      append_ws_groups(*p, (long long)(m->f_at[i] / sizeof(float)), (long long)(m->pm_at[i] / sizeof(double)), groups);
  }
  // one grouped launch over every split member's classes: costliest first
  std::stable_sort(groups.begin(), groups.end(), [](const WsGroup& a, const WsGroup& b) {
    return (double)a.n_vox / a.n_krange * a.n_wg > (double)b.n_vox / b.n_krange * b.n_wg;
  });
  int block = 0;
  for (WsGroup& g : groups) {
    g.block0 = block;
    block += g.n_wg * g.n_krange;
    m->ws_lds = std::max(m->ws_lds, bf16x3_lds_bytes(g.max_s, g.rep));
    if (!ws_group_ok(g)) return fail(set_err(BISPEC_EINVAL, "a grid class does not fit the split-bf16 kernel"));
  }
  m->ws_n = (int)groups.size();
  m->ws_blocks = block;
  // the reductions of every split member's classes, in member and class order
  std::vector<RedGroup> red;
  long long red_blocks = 0;
  for (int32_t i = 0; i < n; ++i) {
    bispec_plan_s* p = m->plans[i];
    if (p->precision == BISPEC_PREC_FP32) continue;
    for (GridClass& c : p->cls) {
      if (c.n_tri <= 0) continue;
      RedGroup g;
      g.partial = p->partial_mfma.as<double>() + c.pm_off;
      g.slot = c.mfma_slot.as<int32_t>();
      g.norm = p->norm.as<double>();
      g.out_idx = c.tri_out.as<int32_t>();
      g.stride = (long long)c.tile_stride * kMTileElems;
      g.n_tri = c.n_tri;
      g.b_off = m->b_off[i];
      g.n_krange = mfma_ranges(c);
      g.block0 = (int)red_blocks;
      red_blocks += reduce_blocks(c.n_tri);
      red.push_back(g);
    }
  }
  if (red_blocks > (1LL << 30)) return fail(set_err(BISPEC_EINVAL, "batch has too many triangles for one reduction launch"));
  m->red_n = (int)red.size();
  m->red_blocks = (int)red_blocks;
  if (m->ws_n > 0) {
    hipError_t e = upload(m->ws_groups, groups, s);
    if (e == hipSuccess && m->red_n > 0) e = upload(m->red_groups, red, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(set_err(BISPEC_EHIP, std::string("batch table: ") + hipGetErrorString(e)));
  }
  if ((m->ws_n > 0) != (m->red_n > 0)) return fail(set_err(BISPEC_EINVAL, "batch tables disagree"));
  *out = m;
  return BISPEC_OK;
}

int bispec_many_layout(bispec_many_t m, int32_t* n, int64_t* delta_off, int64_t* b_off) {
  if (!m) return set_err(BISPEC_EINVAL, "null batch");
  if (n) *n = (int32_t)m->plans.size();
  for (size_t i = 0; i < m->d_off.size(); ++i) {
    if (delta_off) delta_off[i] = m->d_off[i];
    if (b_off) b_off[i] = m->b_off[i];
  }
  return BISPEC_OK;
}

int bispec_many_units(bispec_many_t m, int32_t* n_units, int32_t* n_cohort_members) {
  if (!m || !n_units) return set_err(BISPEC_EINVAL, "bad argument");
  *n_units = (int32_t)m->units.size();
  if (n_cohort_members) {
    int32_t c = 0;
    for (const auto& u : m->units)
      if (u->m > 1) c += u->m;
    *n_cohort_members = c;
  }
  return BISPEC_OK;
}

int bispec_many_plan(bispec_many_t m, int32_t i, bispec_plan_t* plan) {
  if (!m || !plan || i < 0 || i >= (int32_t)m->plans.size()) return set_err(BISPEC_EINVAL, "bad argument");
  *plan = m->plans[i];
  return BISPEC_OK;
}

int bispec_run_many(bispec_many_t m, const float* delta, double* B, int32_t use_graph, void* hip_stream) {
  if (!m || !delta || !B) return set_err(BISPEC_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)hip_stream;
  if (!use_graph) return many_enqueue(*m, delta, B, s);
  if (!m->exec || m->g_delta != delta || m->g_B != B) {
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    m->exec = nullptr;
    m->graph = nullptr;
    if (!m->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
    const int st = many_enqueue(*m, delta, B, m->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(m->cap_stream, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return set_err(BISPEC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    m->graph = g;
    HIP_TRY(hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0));
    m->g_delta = delta;
    m->g_B = B;
  }
  HIP_TRY(hipGraphLaunch(m->exec, s));
  return BISPEC_OK;
}

int bispec_destroy_many(bispec_many_t m) {
  delete m;
  return BISPEC_OK;
}

}  // extern "C"

bispec_many_s::~bispec_many_s() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  for (bispec_plan_s* p : plans) delete p;  // views of the lanes' workspaces
  for (ManyLane* l : lanes) delete l;
}
