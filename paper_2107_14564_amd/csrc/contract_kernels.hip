// Triple contraction (step c, and c2 for the unit shells):
//   T(i, j, l) = sum_x F_i(x) F_j(x) F_l(x)      for the selected triangles,
// the numerator of eq. bsfin (data shells) and of eq. Ntri2 (unit shells).
//
// Work decomposition (geometry.h): rows are shell pairs (i, j), columns single
// shells l, a tile is 32 pairs x 32 consecutive shells, a task <= 8 tiles.
// Every kernel walks a voxel range [k_lo, k_hi) in chunks staged in LDS (all
// shells of the chunk, so one HBM read serves every tile of the work group),
// keeps its tiles' sums in registers over the whole range and writes one
// float64 partial per (voxel range, triangle).  A fixed-order float64
// reduction over the ranges then gives T, so results are deterministic.
//
// Work groups that share a voxel range are placed on the same XCD (blocks are
// dealt round-robin to the 8 XCDs), so their repeated reads of a chunk hit
// that XCD's L2.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace bispec {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void xcd_map(int n_groups, int& group, int& krange) {
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int q = b >> 3;
  group = q % n_groups;
  krange = xcd + 8 * (q / n_groups);
}

// voxel ranges start on multiples of 64 voxels (aligned vector loads)
__device__ __forceinline__ long long range_lo(long long n_vox, int n_krange, int kr) {
  return kr >= n_krange ? n_vox : ((n_vox * kr) / n_krange) & ~63LL;
}

// ============================================================================
// Vector form: T = float (step c', plain fp32 FMAs) or double (step c2).
// One work group = one task (<= 8 tiles).  Thread t: tile t/32; within the
// tile, rows 4*((t%32)/4) .. +3 and columns 8*(t%4) .. +7 (32 sums per thread).
// LDS chunk: [Kc][n_s + 1] (shell-contiguous per voxel, one zero shell last).
// Sums run in T over one chunk (<= 256 voxels) and are then added into float64
// totals: a long float32 chain would carry rounding error proportional to its
// running partial sum, which for shells of box-scale wavelength is far larger
// than the final (cancelling) total.
// ============================================================================
template <typename T>
__global__ void __launch_bounds__(kThreads) k_contract_vec(const T* __restrict__ F, ContractArgs a, int kc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* chunk = reinterpret_cast<T*>(smem_raw);
  int task, kr;
  xcd_map(a.n_tasks, task, kr);
  const int ns = a.n_s;
  const int ls = ns + 1;  // row stride; entry ns is the zero shell
  const int t0 = a.task_off[task], t1 = a.task_off[task + 1];
  const int tl = threadIdx.x >> 5;            // tile slot
  const int q = threadIdx.x & 31;
  const int rq = q >> 2, cq = q & 3;
  const bool active = t0 + tl < t1;
  Tile tile{0, 1};
  if (active) tile = a.tiles[t0 + tl];
  int ri[4], rj[4], cl[8];
  const RowBlock* rb = a.rows + tile.rb;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = 4 * rq + u;
    const int i = active ? rb->i[r] : 0, j = active ? rb->j[r] : 0;
    ri[u] = (j > 0) ? i - 1 : ns;
    rj[u] = (j > 0) ? j - 1 : ns;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int l = tile.col0 + 8 * cq + c;
    cl[c] = (l >= 1 && l <= ns) ? l - 1 : ns;
  }
  // float32: per-chunk sums in acc, flushed into tot; float64: tot directly
  constexpr bool kF32 = sizeof(T) == 4;
  T acc[4][8];
  double tot[4][8];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int c = 0; c < 8; ++c) tot[u][c] = 0.0;

  const long long k_lo = range_lo(a.n_vox, a.n_krange, kr), k_hi = range_lo(a.n_vox, a.n_krange, kr + 1);
  // zero shell column
  for (int x = threadIdx.x; x < kc; x += kThreads) chunk[x * ls + ns] = (T)0;
  for (long long x0 = k_lo; x0 < k_hi; x0 += kc) {
    const int len = (int)min((long long)kc, k_hi - x0);
    __syncthreads();
    for (int e = threadIdx.x; e < ns * kc; e += kThreads) {
      const int s = e / kc, x = e % kc;
      chunk[x * ls + s] = x < len ? F[(long long)s * a.n_vox + x0 + x] : (T)0;
    }
    __syncthreads();
    if (!active) continue;
    if constexpr (kF32) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[u][c] = (T)0;
    }
    for (int x = 0; x < len; ++x) {
      const T* row = chunk + x * ls;
      T p[4], f[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) p[u] = row[ri[u]] * row[rj[u]];
#pragma unroll
      for (int c = 0; c < 8; ++c) f[c] = row[cl[c]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if constexpr (kF32)
            acc[u][c] = fma(p[u], f[c], acc[u][c]);
          else
            tot[u][c] = fma((double)p[u], (double)f[c], tot[u][c]);
        }
    }
    if constexpr (kF32) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c) tot[u][c] += (double)acc[u][c];
    }
  }
  if (!active) return;
  double* out = a.partial + (long long)kr * a.n_tri;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = 4 * rq + u;
    const int i = rb->i[r], j = rb->j[r];
    if (j <= 0) continue;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int l = tile.col0 + 8 * cq + c;
      if (l < 1 || l > j) continue;
      const int t = a.tri_index[((long long)(i - 1) * ns + (j - 1)) * ns + (l - 1)];
      if (t >= 0) out[t] = tot[u][c];
    }
  }
}

// ============================================================================
// Split-BF16 MFMA form (step c).  Each fp32 operand v is written as
// v = hi + lo with hi = bf16(v), lo = bf16(v - hi); the product of two
// operands is accumulated as hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-16
// relative, is dropped) by three v_mfma_f32_32x32x16_bf16 per 16 voxels.
// Row operand: the pair product F_i F_j formed in fp32 then split; column
// operand: F_l split once per chunk into LDS.
//
// One work group = 4 wavefronts = up to 4 tasks; wavefront w runs task 4g + w.
// LDS chunk (Kc = 64 voxels): Ff [n_s + 1][Kc + 4] fp32, Bh/Bl [n_s + 1][Kc + 8]
// bf16 (row n_s is the zero shell; the pads stagger rows across banks).
// ============================================================================
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kKc = 64;
constexpr int kFfStride = kKc + 4;   // floats
constexpr int kBStride = kKc + 8;    // bf16
constexpr int kFlush = 16;           // chunks (1024 voxels) per float32 accumulation chain
constexpr int kMT = kMaxTilesPerTaskMfma;

// Output element v (0..15) of lane `lane` of a 32x32 MFMA accumulator sits
// at row mfma_row(v, lane), column lane % 32.
__device__ __forceinline__ int mfma_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

__device__ __forceinline__ void split8(const float* p, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)p[e];
    hi[e] = h;
    lo[e] = (__bf16)(p[e] - (float)h);
  }
}

__global__ void __launch_bounds__(kThreads) k_contract_bf16x3(const float* __restrict__ F, ContractArgs a,
                                                              int n_groups) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ns = a.n_s;
  float* Ff = reinterpret_cast<float*>(smem_raw);
  __bf16* Bh = reinterpret_cast<__bf16*>(Ff + (ns + 1) * kFfStride);
  __bf16* Bl = Bh + (ns + 1) * kBStride;
  int g, kr;
  xcd_map(n_groups, g, kr);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int task = 4 * g + wave;
  const bool active = task < a.n_tasks;
  const int t0 = active ? a.task_off[task] : 0;
  const int t1 = active ? a.task_off[task + 1] : 0;
  const int nt = t1 - t0;  // <= kMT

  // per tile: this lane's row (pair) and column indices into the chunk
  int rowi[kMT], rowj[kMT], col[kMT], rbk[kMT];
  const int r = lane & 31, kg = lane >> 5;
#pragma unroll
  for (int k = 0; k < kMT; ++k) {
    rowi[k] = ns;
    rowj[k] = ns;
    col[k] = ns;
    rbk[k] = -1;
    if (k < nt) {
      const Tile tl = a.tiles[t0 + k];
      rbk[k] = tl.rb;
      const int i = a.rows[tl.rb].i[r], j = a.rows[tl.rb].j[r];
      if (j > 0) { rowi[k] = i - 1; rowj[k] = j - 1; }
      const int l = tl.col0 + r;
      if (l >= 1 && l <= ns) col[k] = l - 1;
    }
  }
  f32x16 acc[kMT];
  double tot[kMT][16];
#pragma unroll
  for (int k = 0; k < kMT; ++k)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      acc[k][v] = 0.f;
      tot[k][v] = 0.0;
    }
  int chain = 0;

  // zero shell rows
  for (int e = threadIdx.x; e < kFfStride; e += kThreads) Ff[ns * kFfStride + e] = 0.f;
  for (int e = threadIdx.x; e < kBStride; e += kThreads) {
    Bh[ns * kBStride + e] = (__bf16)0.f;
    Bl[ns * kBStride + e] = (__bf16)0.f;
  }
  const long long k_lo = range_lo(a.n_vox, a.n_krange, kr), k_hi = range_lo(a.n_vox, a.n_krange, kr + 1);
  for (long long x0 = k_lo; x0 < k_hi; x0 += kKc) {
    const int len = (int)min((long long)kKc, k_hi - x0);
    __syncthreads();
    // stage the chunk: 4 voxels per thread step
    for (int e = threadIdx.x; e < ns * (kKc / 4); e += kThreads) {
      const int s = e / (kKc / 4), x4 = (e % (kKc / 4)) * 4;
      float v[4];
      const float* src = F + (long long)s * a.n_vox + x0 + x4;
      if (x4 + 4 <= len && ((((uintptr_t)src) & 15) == 0)) {
        const float4 q = *reinterpret_cast<const float4*>(src);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (x4 + u < len) ? src[u] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        Ff[s * kFfStride + x4 + u] = v[u];
        const __bf16 h = (__bf16)v[u];
        Bh[s * kBStride + x4 + u] = h;
        Bl[s * kBStride + x4 + u] = (__bf16)(v[u] - (float)h);
      }
    }
    __syncthreads();
    if (!active) continue;
#pragma unroll
    for (int ks = 0; ks < kKc / 16; ++ks) {
      const int off = ks * 16 + kg * 8;
      int prev_rb = -1;  // wave-uniform: tiles of one row block share the row operand
      bf16x8 ahi, alo;
#pragma unroll
      for (int k = 0; k < kMT; ++k) {
        if (k >= nt) break;
        if (rbk[k] != prev_rb) {
          const float* fi = Ff + rowi[k] * kFfStride + off;
          const float* fj = Ff + rowj[k] * kFfStride + off;
          const float4 i0 = *reinterpret_cast<const float4*>(fi), i1 = *reinterpret_cast<const float4*>(fi + 4);
          const float4 j0 = *reinterpret_cast<const float4*>(fj), j1 = *reinterpret_cast<const float4*>(fj + 4);
          float p[8] = {i0.x * j0.x, i0.y * j0.y, i0.z * j0.z, i0.w * j0.w,
                        i1.x * j1.x, i1.y * j1.y, i1.z * j1.z, i1.w * j1.w};
          split8(p, ahi, alo);
          prev_rb = rbk[k];
        }
        const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(Bh + col[k] * kBStride + off);
        const bf16x8 blo = *reinterpret_cast<const bf16x8*>(Bl + col[k] * kBStride + off);
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi, acc[k], 0, 0, 0);
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo, acc[k], 0, 0, 0);
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, acc[k], 0, 0, 0);
      }
    }
    if (++chain == kFlush || x0 + kKc >= k_hi) {
      chain = 0;
#pragma unroll
      for (int k = 0; k < kMT; ++k)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          tot[k][v] += (double)acc[k][v];
          acc[k][v] = 0.f;
        }
    }
  }
  if (!active) return;
  double* out = a.partial + (long long)kr * a.n_tri;
#pragma unroll
  for (int k = 0; k < kMT; ++k) {
    if (k >= nt) break;
    const Tile tl = a.tiles[t0 + k];
    const int l = tl.col0 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = mfma_row(v, lane);
      const int i = a.rows[tl.rb].i[row], j = a.rows[tl.rb].j[row];
      if (j <= 0 || l < 1 || l > j) continue;
      const int t = a.tri_index[((long long)(i - 1) * ns + (j - 1)) * ns + (l - 1)];
      if (t >= 0) out[t] = tot[k][v];
    }
  }
}

__global__ void k_reduce(const double* __restrict__ partial, int n_krange, long long n_tri,
                         const double* __restrict__ norm, double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  double s = 0.0;
  for (int k = 0; k < n_krange; ++k) s += partial[(long long)k * n_tri + t];
  out[t] = norm ? s * norm[t] : s;
}

template <typename T>
hipError_t launch_vec(const T* F, const ContractArgs& a, hipStream_t st) {
  const int ls = a.n_s + 1;
  int kc = (int)((40 * 1024) / ((size_t)ls * sizeof(T)));
  kc = kc >= 256 ? 256 : (kc / 16) * 16;
  if (kc < 16) return hipErrorInvalidValue;
  const size_t lds = (size_t)kc * ls * sizeof(T);
  const unsigned blocks = (unsigned)a.n_tasks * (unsigned)a.n_krange;
  hipLaunchKernelGGL(k_contract_vec<T>, dim3(blocks), dim3(kThreads), lds, st, F, a, kc);
  return hipGetLastError();
}

}  // namespace

size_t bf16x3_lds_bytes(int n_s) {
  return (size_t)(n_s + 1) * kFfStride * sizeof(float) + 2 * (size_t)(n_s + 1) * kBStride * sizeof(__bf16);
}

hipError_t launch_contract_fp32(const float* F, const ContractArgs& a, hipStream_t st) { return launch_vec<float>(F, a, st); }
hipError_t launch_contract_fp64(const double* F, const ContractArgs& a, hipStream_t st) { return launch_vec<double>(F, a, st); }

hipError_t launch_contract_bf16x3(const float* F, const ContractArgs& a, hipStream_t st) {
  const int n_groups = (a.n_tasks + 3) / 4;
  const size_t lds = bf16x3_lds_bytes(a.n_s);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)n_groups * (unsigned)a.n_krange;
  hipLaunchKernelGGL(k_contract_bf16x3, dim3(blocks), dim3(kThreads), lds, st, F, a, n_groups);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int n_krange, long long n_tri, const double* norm, double* out,
                         hipStream_t st) {
  const unsigned blocks = (unsigned)((n_tri + 255) / 256);
  hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(256), 0, st, partial, n_krange, n_tri, norm, out);
  return hipGetLastError();
}

}  // namespace bispec
