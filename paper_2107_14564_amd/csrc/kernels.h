// Launch interface between the plan runtime (api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "geometry.h"

namespace bispec {

// Tile shapes of the FFT passes (shared by kernels and host planning).
// Strided passes: TW columns x N rows per block plus the N-entry twiddle table
// (<= 64 KB of LDS together).
__host__ __device__ constexpr int fft_tile_cols_max(int n, bool f64) {
  return (((f64 ? 4096 : 8192) - n) / n) < 64 ? (((f64 ? 4096 : 8192) - n) / n) : 64;
}
// ... rounded down to whole 128-byte row pieces (16 float2, 8 double2) where at
// least one piece fits, so tiles start on cache-line boundaries of padded rows
__host__ __device__ constexpr int fft_tile_cols(int n, bool f64) {
  return fft_tile_cols_max(n, f64) >= (f64 ? 8 : 16) ? fft_tile_cols_max(n, f64) / (f64 ? 8 : 16) * (f64 ? 8 : 16)
                                                     : fft_tile_cols_max(n, f64);
}
// Row length (complex entries) of the per-shell intermediates A1_n, A2_n: the
// R + 1 used kz columns rounded up to 128 bytes, so rows start on cache lines.
__host__ __device__ constexpr int shell_row(int r, bool f64) {
  return f64 ? (r + 1 + 7) / 8 * 8 : (r + 1 + 15) / 16 * 16;
}
// Row length (complex entries) of the half spectrum [N][N][.]: N/2 + 1 rounded
// up to 16 (128 bytes), so rows start on cache-line boundaries and the strided
// forward passes' 16-column tiles read and write whole lines.  The entries past
// N/2 are never read.
__host__ __device__ constexpr long long spec_row(int n) { return ((long long)(n / 2 + 1) + 15) / 16 * 16; }
// Contiguous passes over lines of length len (LDS stride len + 1): lines per block.
__host__ __device__ constexpr int fft_z_lines(int len, bool f64) { return (f64 ? 2048 : 2048) / (len + 1); }

// Supported grid sizes: N = 2^a * {1, 3, 5}, 8 <= N <= 1024.
inline bool fft_size_supported(int n) {
  if (n < 8 || n > 1024) return false;
  int m = n;
  while (m % 2 == 0) m /= 2;
  return (m == 1 || m == 3 || m == 5) && (n / m) >= 8;
}

// Shell fields (F, its bf16 planes, the float64 unit shells) are stored
// voxel-blocked: value of shell n at voxel v sits at
//   (v / kVoxBlock) * n_s * kVoxBlock + n * kVoxBlock + v % kVoxBlock,
// so one block of kVoxBlock voxels of every shell is contiguous (the unit the
// contraction streams), and a chunk touches one memory page instead of n_s.
constexpr int kVoxBlock = 32;
__host__ __device__ inline long long vox_index(long long v, int n, int n_s) {
  return (v / kVoxBlock) * (long long)n_s * kVoxBlock + (long long)n * kVoxBlock + (v % kVoxBlock);
}
__host__ inline long long blocked_elems(long long n_vox, int n_s) {
  return (n_vox + kVoxBlock - 1) / kVoxBlock * (long long)n_s * kVoxBlock;
}

struct ShellDev {
  long long lo2, hi2;   // shell holds lo2 <= |m|^2 < hi2
  long long a1_off;     // element offset of A1_n
  long long a2_off;     // element offset of A2_n
  int rad;              // R = floor(sqrt(hi2 - 1))
  int wrow;             // row length of A1_n and A2_n: shell_row(R) >= R + 1
  int ell;              // data fields: weight L_ell(m_z/|m|) on every mode (0: none)
  int pad_;
};

struct ShellLaunch {
  int n_shells = 0;
  int spec_n = 0;                     // grid of the half spectrum read (x pass) or written (adjoint)
  const ShellDev* shells = nullptr;   // device [n_shells]
  const int4* x_tiles = nullptr;      // device (shell, ky, kz0, 0)
  long long n_x_tiles = 0;
  const long long* y_off = nullptr;   // device prefix sums [n_shells + 1]
  long long n_y_blocks = 0;
  const long long* z_off = nullptr;   // device prefix sums [n_shells + 1]
  long long n_z_blocks = 0;
  // an x-slab of the grid (0: the whole grid): the y pass takes planes
  // x0 .. x_end - 1 (A2 and the fields hold only those), the z pass n_lines
  // lines (the slab's planes times n)
  int x0 = 0, x_end = 0;
  long long n_lines = 0;
  // a cohort of identical problems in one launch (grid y = member): member m's
  // spectrum, A1, A2 and fields at m times these element strides
  int n_members = 1;
  long long spec_stride = 0, a1_stride = 0, a2_stride = 0, f_stride = 0;
};

// host-side description of the shell passes; device arrays are uploaded by the caller
struct ShellPassPlan {
  std::vector<ShellDev> shells;
  std::vector<int4> x_tiles;
  std::vector<long long> y_off, z_off;
  long long a1_elems = 0, a2_elems = 0;
};
// passes of every shell of g on a grid of n points per side
// nx: x-planes per slab (A2 and the y and z blocks cover nx planes; 0 = n)
void plan_shell_passes(const ShellGeometry& g, int n, bool f64, ShellPassPlan& p, int nx = 0);

hipError_t prepare_forward();   // once per plan, before any launch (and before graph capture)
// members > 1: a cohort of identical problems, member m at delta + m delta_stride
// and spec + m spec_stride (elements)
hipError_t launch_forward(const float* delta, float2* spec, int n, float beta, const float2* tw, hipStream_t st,
                          int members = 1, long long delta_stride = 0, long long spec_stride = 0);
// the three inverse passes of every shell (fft_inv_x.hip, fft_inv_y.hip, fft_c2r.hip)
hipError_t launch_inv_x_f32(const float2* spec, float2* a1, const ShellLaunch& L, int n, const float2* tw,
                            hipStream_t st);
hipError_t launch_inv_x_unit_f64(double2* a1, const ShellLaunch& L, int n, const double2* tw, hipStream_t st);
hipError_t launch_inv_y_f32(const float2* a1, float2* a2, const ShellLaunch& L, int n, const float2* tw,
                            hipStream_t st);
hipError_t launch_inv_y_f64(const double2* a1, double2* a2, const ShellLaunch& L, int n, const double2* tw,
                            hipStream_t st);
hipError_t launch_c2r_f32(const float2* a2, float* F, const ShellLaunch& L, int n, const float2* tw,
                          hipStream_t st);
hipError_t launch_c2r_f64(const double2* a2, double* I, const ShellLaunch& L, int n, const double2* tw,
                          hipStream_t st);
// n: the grid of the passes (the estimator grid); the spectrum grid is L.spec_n.
// Fields are written voxel-blocked (vox_index).
hipError_t launch_data_shells(const float2* spec, float2* a1, float2* a2, float* F, const ShellLaunch& L, int n,
                              const float2* tw, hipStream_t st);
hipError_t launch_unit_shells(double2* a1, double2* a2, double* I, const ShellLaunch& L, int n, const double2* tw,
                              hipStream_t st);
// dst[v] = F[vox_index(v, shell, n_s)] for v < n_vox (float32)
hipError_t launch_unblock(const float* F, int shell, int n_s, long long n_vox, float* dst, hipStream_t st);

// ---- contraction ---------------------------------------------------------------
struct ContractArgs {
  const RowBlock* rows = nullptr;   // device
  const Tile* tiles = nullptr;      // device, task-major
  const int32_t* task_off = nullptr;  // device [n_tasks + 1] (task grouping of the kernel launched)
  int n_tasks = 0;
  const int32_t* tri_index = nullptr; // device [n_s^3]: (i-1, j-1, l-1) -> triangle or -1
  int n_s = 0;
  long long n_vox = 0;               // voxels per field
  int n_krange = 0;                  // voxel ranges (multiple of 8)
  double* partial = nullptr;         // device [n_krange][n_tri]
  long long n_tri = 0;
};

hipError_t prepare_contract_vec();   // once per plan, before the first vector-kernel launch
hipError_t launch_contract_fp32(const float* F, const ContractArgs& a, hipStream_t st);
hipError_t launch_contract_fp64(const double* F, const ContractArgs& a, hipStream_t st);

struct WsArgs {
  const MRowBlock* rows = nullptr;    // device [n_wg * kRbPerWg]
  const SlotCols* cols = nullptr;     // device [n_wg * kSlotsPerWg]
  const WgRows* wg_rows = nullptr;    // device [n_wg]
  int n_wg = 0;                       // work groups per voxel range
  int n_s = 0;
  int max_s = 0;                      // most shells staged by one work group (LDS sizing)
  long long n_vox = 0;
  int n_krange = 0;                   // multiple of 8
  int rep = 1;                        // replicas of the slot set (voxel ranges per work group)
  int tile_stride = 0;                // tiles per voxel range in the partials
  double* partial = nullptr;          // device [rep * n_krange][tile_stride][kMTileElems]
};
// One group of the grouped split-bf16 launch (a grid class of a plan): its
// fields and partials as element offsets from the launch's F and partial
// pointers, so one table serves any placement of those buffers.
struct WsGroup {
  long long f_off = 0;                // fields: F + f_off, voxel-blocked over n_s shells
  long long p_off = 0;                // partials: partial + p_off, [rep * n_krange][tile_stride][kMTileElems]
  const MRowBlock* rows = nullptr;    // device [n_wg * kRbPerWg]
  const SlotCols* cols = nullptr;     // device [n_wg * kSlotsPerWg]
  const WgRows* wg_rows = nullptr;    // device [n_wg]
  long long n_vox = 0;
  int n_wg = 0, n_s = 0, max_s = 0;
  int n_krange = 0;                   // multiple of 8
  int block0 = 0;                     // first block of the group (multiple of 8); groups ascending
  // replicas (1, 2, 3, 4 or 6; n_wg = 1 when above 1): the work group's waves run rep
  // copies of slots 0 .. kSlotsPerWg / rep - 1, copy r on voxel range
  // rep * kr + r of rep * n_krange ranges
  int rep = 1;
  // tiles per voxel range in the partials: n_wg * kTilesPerWg, or for one work
  // group only its busy slots' (slots 0 .. top), (top + 1) * kSlotTiles
  int tile_stride = 0;
  int pad_ = 0;
};
constexpr int kMaxSplitShells = 128;   // most shells of a split-bf16 plan
constexpr size_t kWsLdsMax = 160 * 1024;   // LDS of one work group on gfx950
size_t bf16x3_lds_bytes(int max_s, int rep = 1);
// the largest replica count a one-work-group tiling allows (slots used, rows
// staged, LDS): 1 when n_wg > 1
int ws_max_rep(const MfmaTiling& mt);
// tiles per voxel range of a tiling's partials (the tile_stride of its group)
int ws_tile_stride(const MfmaTiling& mt);
bool ws_group_ok(const WsGroup& g);
hipError_t prepare_contract_bf16x3();   // once per plan, before any launch (and before graph capture)
// groups_dev: device [n_groups]; lds_bytes: the largest bf16x3_lds_bytes(max_s,
// rep) of the groups; n_blocks: sum of n_wg * n_krange
hipError_t launch_contract_bf16x3(const float* F, double* partial, const WsGroup* groups_dev, int n_groups,
                                  size_t lds_bytes, int n_blocks, hipStream_t st);
// Gradient: w_k = gB[t_k] norm[t_k]; G_n = sum_{terms (t, j, l) of n} w F_j F_l
// (terms: int4 (t, j, l, 0) with 0-based shells, grouped by n via term_off[n_s + 1])
hipError_t launch_gbuild(const float* F, const double* gB, const double* norm, const int4* terms, long long n_terms,
                        const int32_t* term_off, int n_s, long long n_vox, double* w, float* G, hipStream_t st);
// ---- adjoint field build on the matrix cores (row blocks: geometry.h) --------
constexpr int kAdjVox = 64;         // voxels per staged chunk (two voxel blocks; two work groups fit a CU)
struct AdjGroup {
  long long f_off = 0;            // fields and adjoint fields: F + f_off, G + f_off (voxel-blocked, n_s shells)
  const AdjRowBlock* rbs = nullptr;
  const AdjN* ns = nullptr;
  const AdjWave* waves = nullptr; // [n_wg * kAdjWaves]
  const uint16_t* W = nullptr;    // [tiles][2 (hi, lo)][64 lanes][8] bf16 bits
  long long n_vox = 0;
  int n_s = 0, n_wg = 0, n_krange = 0, block0 = 0;
};
size_t adj_lds_bytes(int max_s);
hipError_t prepare_adjoint_mfma();   // once per plan (LDS limit)
// W of one class: tile-lane slot q = (tile * 64 + lane) * 8 + i takes
// sum_{k in [off[q], off[q+1])} gB[tri[k]] norm[tri[k]], split into hi and lo bf16
hipError_t launch_adj_weights(const double* gB, const double* norm, const int32_t* off, const int32_t* tri,
                              long long n_tiles, uint16_t* W, hipStream_t st);
hipError_t launch_adjoint_mfma(const float* F, float* G, const AdjGroup* groups_dev, int n_groups, int max_s,
                               int n_blocks, hipStream_t st);

// pruned forward transforms of every G_n, added (times scale * Z) into the half
// spectrum S; zero_first clears S before
hipError_t launch_adjoint_shells(const float* G, float2* a1, float2* a2, float2* S, const ShellLaunch& L, int n,
                                 const float2* tw, float scale, float beta, bool zero_first, hipStream_t st);

// ---- order-4 contraction (QuadTiling, geometry.h) --------------------------
struct Quad4Args {
  const int32_t* pair_ij = nullptr;   // device [n_pairs + 1]
  const int32_t* rb_pairs = nullptr;  // device [n_rb * 16]
  const int32_t* cb_pairs = nullptr;  // device [n_cb * 16]
  const int4* tiles = nullptr;        // device [n_tiles]: slot, row block, column block
  const int32_t* wave_t0 = nullptr;   // device [n_wg * kSlotsPerWg + 1]
  int n_pairs = 0, n_s = 0, n_wg = 0, n_krange = 0;
  long long n_vox = 0;
  double* partial = nullptr;          // device [n_krange][n_wg * kTilesPerWg][kMTileElems]
};
size_t quad4_lds_bytes(int n_pairs, int n_s, bool f64);
constexpr int kMaxQuadPairs = 496;    // pair products staged per chunk
hipError_t prepare_contract4();
// sum_x P_(i,j) P_(k,l): float32 fields on split-bf16 MFMAs, or float64 fields
// (the unit shells, for N_quad) on float64 MFMAs
hipError_t launch_contract4_bf16x3(const float* F, const Quad4Args& a, hipStream_t st);
hipError_t launch_contract4_f64(const double* F, const Quad4Args& a, hipStream_t st);

// dst[0 .. n) = pseudo-random values in [-1, 1) (autotuner timing fields)
hipError_t launch_fill_random(float* dst, long long n, unsigned long long seed, hipStream_t st);
// dst[0 .. bytes) = 0 with a fill kernel (capture-safe; bytes and dst 16-byte aligned)
hipError_t launch_zero(void* dst, size_t bytes, hipStream_t st);
// The reductions of many grid classes (of the members of a batch) in one
// launch: group g turns its class's partials into results B[b_off + o] as
// launch_reduce does with norm, slot and out_idx (same order of additions).
struct RedGroup {
  const double* partial = nullptr;    // the class's partials, n_krange ranges at stride
  const int32_t* slot = nullptr;      // triangle -> element of a range
  const double* norm = nullptr;       // indexed by result
  const int32_t* out_idx = nullptr;   // triangle -> result of the member
  long long stride = 0, n_tri = 0;
  long long b_off = 0;                // the member's results at B + b_off
  int n_krange = 0;
  int block0 = 0;                     // first block of the group (reduce_blocks(n_tri) blocks each)
};
long long reduce_blocks(long long n_tri);
hipError_t launch_reduce_grouped(const RedGroup* groups_dev, int n_groups, int n_blocks, double* B, hipStream_t st);

// out[o] = norm[o] * sum_k partial[k * stride + (slot ? slot[t] : t)] with o = out_idx ? out_idx[t] : t,
// for t < n_tri (fixed order, float64; norm may be null); accumulate: out[o] += that
hipError_t launch_reduce(const double* partial, int n_krange, long long stride, long long n_tri, const int32_t* slot,
                         const double* norm, const int32_t* out_idx, double* out, hipStream_t st,
                         bool accumulate = false);

}  // namespace bispec
