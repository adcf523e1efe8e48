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
      chunk[x * ls + s] = x < len ? F[vox_index(x0 + x, s, ns)] : (T)0;
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
// v = hi + lo with hi = bf16(v), lo = bf16(v - hi); a product of two operands
// is accumulated as hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-16 relative, is
// dropped) by three v_mfma_f32_32x32x16_bf16 per 16 voxels.  The row operand
// is the pair product F_i F_j formed in fp32 and then split; the column
// operand comes pre-split as bf16 planes written by the C2R pass.
//
// Work group = 8 wavefronts (512 threads), two per SIMD:
//   consumers (waves 0-3): slot w = kRbPerSlot row blocks of one span and
//     their <= kMaxColTiles column tiles; per 16 voxels it reads the row fragments of its
//     row blocks and each column fragment once (shared by both row blocks) and
//     issues 3 MFMAs per (row block, tile);
//   producers (waves 4-7): copy the work group's F rows (chunk c+2) and column
//     plane rows (chunk c+1) from registers loaded two chunks earlier, and
//     form + split the pair products of chunk c+1 for all kRbPerWg row blocks.
// Only the shell rows the work group needs are staged (WgRows).  LDS holds two
// buffers of everything (one barrier per chunk of kC2 = 32 voxels):
//   F32 [2][max_f + 1][kC2 + 4] fp32, Bh/Bl [2][max_b + 1][kC2 + 8] bf16,
//   Ah/Al [2][kRbPerWg][32][kC2 + 8] bf16      (the extra row is all zero).
// Accumulation: fp32 MFMA chains of kFlushChunks chunks, added in float64 into
// partial[range][tile][element] (tile-major, coalesced); the reduction maps
// elements to triangles.
// ============================================================================
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kC2 = 32;              // voxels per chunk (= one voxel block)
constexpr int kF32S = kC2 + 4;       // fp32 row stride (floats)
constexpr int kBS = kC2 + 8;         // bf16 row stride (elements)
constexpr int kFlushChunks = 256;    // 8192 voxels per float32 accumulation chain
constexpr int kWsThreads = 512;
constexpr int kProd = 256;           // producer threads
constexpr int kNV = 4;               // float4 / uint4 staging slots per producer thread
static_assert(kC2 == kVoxBlock, "chunks are voxel blocks");

struct WsLds {
  float* f32;      // [2][nf1][kF32S]
  __bf16* bh;      // [2][nb1][kBS]
  __bf16* bl;
  __bf16* ah;      // [2][kRbPerWg][32][kBS]
  __bf16* al;
  int nf1, nb1;    // rows per buffer including the zero row
  __device__ float* F(int buf, int r) const { return f32 + (buf * nf1 + r) * kF32S; }
  __device__ __bf16* Bh(int buf, int r) const { return bh + (buf * nb1 + r) * kBS; }
  __device__ __bf16* Bl(int buf, int r) const { return bl + (buf * nb1 + r) * kBS; }
  __device__ __bf16* Ah(int buf, int rb, int r) const { return ah + ((buf * kRbPerWg + rb) * 32 + r) * kBS; }
  __device__ __bf16* Al(int buf, int rb, int r) const { return al + ((buf * kRbPerWg + rb) * 32 + r) * kBS; }
};

__device__ __forceinline__ void split8(const float* p, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)p[e];
    hi[e] = h;
    lo[e] = (__bf16)(p[e] - (float)h);
  }
}

struct WsRange {
  long long k_lo, k_hi;
  int n_chunks;
};

// ---- producers ---------------------------------------------------------------
struct WsPf {
  float4 f[kNV];
  uint4 b[kNV];    // slots [0, 4 b_n) hi plane rows, [4 b_n, 8 b_n) lo plane rows
};

__device__ __forceinline__ void ws_load_f(const float* __restrict__ F, const WsArgs& a, const WgRows& wr,
                                          const WsRange& R, int c, WsPf& pf, int tid) {
  if (c >= R.n_chunks) return;
  const float4* base = reinterpret_cast<const float4*>(F + ((R.k_lo / kC2) + c) * (long long)a.n_s * kC2 +
                                                       (long long)wr.f_lo * kC2);
  const int n4 = wr.f_n * (kC2 / 4);
#pragma unroll
  for (int u = 0; u < kNV; ++u) {
    const int idx = tid + u * kProd;
    if (idx < n4) pf.f[u] = base[idx];
  }
}

__device__ __forceinline__ void ws_load_b(const __bf16* __restrict__ fh, const __bf16* __restrict__ fl,
                                          const WsArgs& a, const WgRows& wr, const WsRange& R, int c, WsPf& pf,
                                          int tid) {
  if (c >= R.n_chunks) return;
  const long long off = ((R.k_lo / kC2) + c) * (long long)a.n_s * kC2 + (long long)wr.b_lo * kC2;
  const uint4* bh = reinterpret_cast<const uint4*>(fh + off);
  const uint4* bl = reinterpret_cast<const uint4*>(fl + off);
  const int per_plane = wr.b_n * (kC2 / 8);
#pragma unroll
  for (int u = 0; u < kNV; ++u) {
    const int idx = tid + u * kProd;
    if (idx < per_plane)
      pf.b[u] = bh[idx];
    else if (idx < 2 * per_plane)
      pf.b[u] = bl[idx - per_plane];
  }
}

__device__ __forceinline__ void ws_store_f(const WsLds& L, const WgRows& wr, int buf, const WsPf& pf, int tid) {
#pragma unroll
  for (int u = 0; u < kNV; ++u) {
    const int idx = tid + u * kProd;
    if (idx < wr.f_n * (kC2 / 4)) *reinterpret_cast<float4*>(L.F(buf, idx >> 3) + 4 * (idx & 7)) = pf.f[u];
  }
}

__device__ __forceinline__ void ws_store_b(const WsLds& L, const WgRows& wr, int buf, const WsPf& pf, int tid) {
  const int per_plane = wr.b_n * (kC2 / 8);
#pragma unroll
  for (int u = 0; u < kNV; ++u) {
    const int idx = tid + u * kProd;
    if (idx < 2 * per_plane) {
      const int plane = idx >= per_plane;
      const int k = idx - plane * per_plane;
      __bf16* dst = (plane ? L.Bl(buf, k >> 2) : L.Bh(buf, k >> 2)) + 8 * (k & 3);
      *reinterpret_cast<uint4*>(dst) = pf.b[u];
    }
  }
}

// pair products of the chunk in F32 buffer buf, split into A[buf]:
// kRbPerWg * 32 pairs x 4 groups of 8 voxels, 4 groups per thread
__device__ __forceinline__ void ws_products(const WsLds& L, int buf, const int (&pi)[4], const int (&pj)[4],
                                            int tid) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    // two groups in flight at a time (bounds the producer's register use)
    if (u == 2) asm volatile("" ::: "memory");
    const int g = tid + u * kProd;
    const int rbr = g >> 2, xg = (g & 3) * 8;  // rbr = rb * 32 + row
    const float* fi = L.F(buf, pi[u]) + xg;
    const float* fj = L.F(buf, pj[u]) + xg;
    const float4 i0 = *reinterpret_cast<const float4*>(fi), i1 = *reinterpret_cast<const float4*>(fi + 4);
    const float4 j0 = *reinterpret_cast<const float4*>(fj), j1 = *reinterpret_cast<const float4*>(fj + 4);
    const float p[8] = {i0.x * j0.x, i0.y * j0.y, i0.z * j0.z, i0.w * j0.w,
                        i1.x * j1.x, i1.y * j1.y, i1.z * j1.z, i1.w * j1.w};
    bf16x8 hi, lo;
    split8(p, hi, lo);
    *reinterpret_cast<bf16x8*>(L.Ah(buf, rbr >> 5, rbr & 31) + xg) = hi;
    *reinterpret_cast<bf16x8*>(L.Al(buf, rbr >> 5, rbr & 31) + xg) = lo;
  }
}

// Iteration c: products of chunk c+1 (F32[(c+1)%2] -> A[(c+1)%2]); F32[c%2] <- F rows
// of chunk c+2 and B[(c+1)%2] <- plane rows of chunk c+1 from registers loaded two
// iterations earlier; then the loads of chunks c+4 (F) and c+3 (planes) are issued.
__device__ __forceinline__ void ws_producer(const float* __restrict__ F, const __bf16* __restrict__ fh,
                                            const __bf16* __restrict__ fl, const WsArgs& a, const WsLds& L,
                                            const WsRange& R, int wg, int tid) {
  const WgRows wr = a.wg_rows[wg];
  int pi[4], pj[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int g = tid + u * kProd;
    const int rb = wg * kRbPerWg + ((g >> 2) >> 5), r = (g >> 2) & 31;
    const int i = a.rows[rb].i[r], j = a.rows[rb].j[r];
    pi[u] = j > 0 ? i - 1 - wr.f_lo : wr.f_n;  // row f_n of the buffer is zero
    pj[u] = j > 0 ? j - 1 - wr.f_lo : wr.f_n;
  }
  WsPf p0, p1;
  ws_load_f(F, a, wr, R, 0, p0, tid);
  ws_load_f(F, a, wr, R, 1, p1, tid);
  ws_load_b(fh, fl, a, wr, R, 0, p0, tid);
  ws_store_f(L, wr, 0, p0, tid);
  ws_store_f(L, wr, 1, p1, tid);
  ws_store_b(L, wr, 0, p0, tid);
  ws_load_f(F, a, wr, R, 2, p0, tid);
  ws_load_f(F, a, wr, R, 3, p1, tid);
  ws_load_b(fh, fl, a, wr, R, 1, p0, tid);
  ws_load_b(fh, fl, a, wr, R, 2, p1, tid);
  __syncthreads();                 // barrier P1
  ws_products(L, 0, pi, pj, tid);  // chunk 0 -> A[0]
  __syncthreads();                 // barrier P2
  for (int c = 0; c < R.n_chunks; c += 2) {
    if (c + 1 < R.n_chunks) ws_products(L, 1, pi, pj, tid);
    ws_store_f(L, wr, 0, p0, tid);   // F of chunk c+2
    ws_store_b(L, wr, 1, p0, tid);   // planes of chunk c+1
    ws_load_f(F, a, wr, R, c + 4, p0, tid);
    ws_load_b(fh, fl, a, wr, R, c + 3, p0, tid);
    __syncthreads();
    if (c + 1 >= R.n_chunks) break;
    if (c + 2 < R.n_chunks) ws_products(L, 0, pi, pj, tid);
    ws_store_f(L, wr, 1, p1, tid);   // F of chunk c+3
    ws_store_b(L, wr, 0, p1, tid);   // planes of chunk c+2
    ws_load_f(F, a, wr, R, c + 5, p1, tid);
    ws_load_b(fh, fl, a, wr, R, c + 4, p1, tid);
    __syncthreads();
  }
}

// ---- consumers ---------------------------------------------------------------
// NT = column tiles of this slot (constant over the run).
template <int NT>
__device__ __forceinline__ void ws_consumer_nt(const WsArgs& a, const WsLds& L, const WsRange& R, int wg, int w,
                                               const SlotCols& sc, const WgRows& wr, int lane, int kr) {
  const int kg = lane >> 5;
  int cs[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int l = sc.col0[t] + (lane & 31);  // 1-based column shell
    cs[t] = (l <= a.n_s) ? l - 1 - wr.b_lo : wr.b_n;  // row b_n of the buffer is zero
  }
  f32x16 acc[kRbPerSlot][NT];
#pragma unroll
  for (int q = 0; q < kRbPerSlot; ++q)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[q][t][v] = 0.f;
  // partial[kr][tile][element] with tile = wg*kTilesPerWg + (slot rows)*kMaxColTiles + t
  double* out = a.partial + ((long long)kr * a.n_wg * kTilesPerWg + (long long)wg * kTilesPerWg) * 1024 + lane;
  bool first = true;
  __syncthreads();  // matches producer barrier P1
  __syncthreads();  // matches producer barrier P2
  int chain = 0;
  for (int c = 0; c < R.n_chunks; ++c) {
    const int buf = c & 1;
#pragma unroll
    for (int ks = 0; ks < kC2 / 16; ++ks) {
      const int off = ks * 16 + kg * 8;
      bf16x8 ahi[kRbPerSlot], alo[kRbPerSlot];
#pragma unroll
      for (int q = 0; q < kRbPerSlot; ++q) {
        ahi[q] = *reinterpret_cast<const bf16x8*>(L.Ah(buf, w * kRbPerSlot + q, lane & 31) + off);
        alo[q] = *reinterpret_cast<const bf16x8*>(L.Al(buf, w * kRbPerSlot + q, lane & 31) + off);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(L.Bh(buf, cs[t]) + off);
        const bf16x8 blo = *reinterpret_cast<const bf16x8*>(L.Bl(buf, cs[t]) + off);
#pragma unroll
        for (int q = 0; q < kRbPerSlot; ++q) {
          acc[q][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[q], bhi, acc[q][t], 0, 0, 0);
          acc[q][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[q], blo, acc[q][t], 0, 0, 0);
          acc[q][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[q], bhi, acc[q][t], 0, 0, 0);
        }
      }
    }
    if (++chain == kFlushChunks || c + 1 == R.n_chunks) {
      chain = 0;
#pragma unroll
      for (int q = 0; q < kRbPerSlot; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          double* o = out + (long long)((w * kRbPerSlot + q) * kMaxColTiles + t) * 1024;
          // one tile at a time: keeps the float64 read-modify-write of the
          // partials from being hoisted across tiles (register pressure)
          asm volatile("" ::: "memory");
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            o[v * 64] = first ? (double)acc[q][t][v] : o[v * 64] + (double)acc[q][t][v];
            acc[q][t][v] = 0.f;
          }
        }
      first = false;
    }
    __syncthreads();  // matches the producer's per-chunk barrier
  }
  if (R.n_chunks == 0) {  // empty range: its partials are zero
#pragma unroll
    for (int q = 0; q < kRbPerSlot; ++q)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) out[(long long)((w * kRbPerSlot + q) * kMaxColTiles + t) * 1024 + v * 64] = 0.0;
  }
}

__device__ __forceinline__ void ws_consumer(const WsArgs& a, const WsLds& L, const WsRange& R, int wg, int w,
                                            int lane, int kr) {
  const SlotCols sc = a.cols[wg * kSlotsPerWg + w];
  const WgRows wr = a.wg_rows[wg];
  switch (sc.n) {
    case 1: ws_consumer_nt<1>(a, L, R, wg, w, sc, wr, lane, kr); break;
    case 2: ws_consumer_nt<2>(a, L, R, wg, w, sc, wr, lane, kr); break;
    default:  // idle slot: keep the barrier count of the work group
      for (int c = 0; c < R.n_chunks + 2; ++c) __syncthreads();
      break;
  }
}

__global__ void __launch_bounds__(kWsThreads) k_contract_bf16x3(const float* __restrict__ F,
                                                                const __bf16* __restrict__ fh,
                                                                const __bf16* __restrict__ fl, WsArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  WsLds L;
  L.nf1 = a.max_f + 1;
  L.nb1 = a.max_b + 1;
  L.f32 = reinterpret_cast<float*>(smem_raw);
  L.bh = reinterpret_cast<__bf16*>(L.f32 + 2 * L.nf1 * kF32S);
  L.bl = L.bh + 2 * L.nb1 * kBS;
  L.ah = L.bl + 2 * L.nb1 * kBS;
  L.al = L.ah + 2 * kRbPerWg * 32 * kBS;
  int wg, kr;
  xcd_map(a.n_wg, wg, kr);
  const WgRows wr = a.wg_rows[wg];
  // zero rows (index f_n / b_n of each buffer), never overwritten afterwards
  for (int e = threadIdx.x; e < 2 * kF32S; e += kWsThreads) L.F(e / kF32S, wr.f_n)[e % kF32S] = 0.f;
  for (int e = threadIdx.x; e < 2 * kBS; e += kWsThreads) {
    L.Bh(e / kBS, wr.b_n)[e % kBS] = (__bf16)0.f;
    L.Bl(e / kBS, wr.b_n)[e % kBS] = (__bf16)0.f;
  }
  __syncthreads();
  WsRange R;
  R.k_lo = range_lo(a.n_vox, a.n_krange, kr);
  R.k_hi = range_lo(a.n_vox, a.n_krange, kr + 1);
  R.n_chunks = (int)((R.k_hi - R.k_lo + kC2 - 1) / kC2);
  const int wave = threadIdx.x >> 6;
  if (wave < kSlotsPerWg)
    ws_consumer(a, L, R, wg, wave, threadIdx.x & 63, kr);
  else
    ws_producer(F, fh, fl, a, L, R, wg, threadIdx.x - 256);
}

// ============================================================================
// Adjoint field build (gradient of L = sum_t gB_t B_t with respect to the
// scaled shell fields): for every shell n and voxel x
//   G_n(x) = sum over the terms (t, j, l) of n of w_t F_j(x) F_l(x),
// where each selected triangle (a1, a2, a3) contributes the terms (t, a2, a3)
// to G_a1, (t, a1, a3) to G_a2 and (t, a1, a2) to G_a3 (the three factors of
// d(F_a1 F_a2 F_a3)), and w_t = gB_t * norm_t.  Thread = voxel; the F block
// of kGbVox voxels x n_s shells is staged in LDS; G is written voxel-blocked.
// ============================================================================
constexpr int kGbVox = 128;

__global__ void k_gweights(const double* __restrict__ gB, const double* __restrict__ norm,
                           const int4* __restrict__ terms, long long n_terms, float* __restrict__ w) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_terms) w[k] = (float)(gB[terms[k].x] * norm[terms[k].x]);
}

__global__ void __launch_bounds__(kGbVox) k_gbuild(const float* __restrict__ F, const int4* __restrict__ terms,
                                                   const float* __restrict__ w,
                                                   const int32_t* __restrict__ term_off, int n_s,
                                                   float* __restrict__ G) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* f = reinterpret_cast<float*>(smem_raw);  // [n_s][kGbVox]
  const long long blk0 = (long long)blockIdx.x * (kGbVox / kVoxBlock);
  // stage: kGbVox/32 voxel blocks, each n_s x 32 contiguous
  for (int e = threadIdx.x; e < n_s * kGbVox; e += kGbVox) {
    const int b = e / (n_s * kVoxBlock), r = e % (n_s * kVoxBlock);
    const int sh = r / kVoxBlock, v = r % kVoxBlock;
    f[sh * kGbVox + b * kVoxBlock + v] = F[(blk0 + b) * (long long)n_s * kVoxBlock + r];
  }
  __syncthreads();
  const int v = threadIdx.x;
  float* g = G + (blk0 + v / kVoxBlock) * (long long)n_s * kVoxBlock + (v % kVoxBlock);
  for (int n = 0; n < n_s; ++n) {
    float acc = 0.f;
    const int k1 = term_off[n + 1];
    for (int k = term_off[n]; k < k1; ++k) {
      const int4 tm = terms[k];
      acc = fmaf(w[k] * f[tm.y * kGbVox + v], f[tm.z * kGbVox + v], acc);
    }
    g[n * kVoxBlock] = acc;
  }
}

__global__ void k_reduce(const double* __restrict__ partial, int n_krange, long long stride, long long n_tri,
                         const int32_t* __restrict__ slot, const double* __restrict__ norm,
                         double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  const long long at = slot ? slot[t] : t;
  double s = 0.0;
  for (int k = 0; k < n_krange; ++k) s += partial[(long long)k * stride + at];
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

size_t bf16x3_lds_bytes(int max_f, int max_b) {
  return 2 * (size_t)(max_f + 1) * kF32S * sizeof(float) + 4 * (size_t)(max_b + 1) * kBS * sizeof(__bf16) +
         4 * (size_t)kRbPerWg * 32 * kBS * sizeof(__bf16);
}

hipError_t launch_contract_fp32(const float* F, const ContractArgs& a, hipStream_t st) { return launch_vec<float>(F, a, st); }
hipError_t launch_contract_fp64(const double* F, const ContractArgs& a, hipStream_t st) { return launch_vec<double>(F, a, st); }

hipError_t launch_contract_bf16x3(const float* F, const __bf16* f_hi, const __bf16* f_lo, const WsArgs& a,
                                  hipStream_t st) {
  if (a.max_f * (kC2 / 4) > kProd * kNV || 2 * a.max_b * (kC2 / 8) > kProd * kNV) return hipErrorInvalidValue;
  const size_t lds = bf16x3_lds_bytes(a.max_f, a.max_b);
  hipError_t e = hipFuncSetAttribute((const void*)k_contract_bf16x3, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)a.n_wg * (unsigned)a.n_krange;
  hipLaunchKernelGGL(k_contract_bf16x3, dim3(blocks), dim3(kWsThreads), lds, st, F, f_hi, f_lo, a);
  return hipGetLastError();
}

hipError_t launch_gbuild(const float* F, const double* gB, const double* norm, const int4* terms, long long n_terms,
                        const int32_t* term_off, int n_s, long long n_vox, float* w, float* G, hipStream_t st) {
  if (n_vox % kGbVox) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gweights, dim3((unsigned)((n_terms + 255) / 256)), dim3(256), 0, st, gB, norm, terms, n_terms,
                     w);
  const size_t lds = (size_t)n_s * kGbVox * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)k_gbuild, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gbuild, dim3((unsigned)(n_vox / kGbVox)), dim3(kGbVox), lds, st, F, terms, w, term_off, n_s,
                     G);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int n_krange, long long stride, long long n_tri, const int32_t* slot,
                         const double* norm, double* out, hipStream_t st) {
  const unsigned blocks = (unsigned)((n_tri + 255) / 256);
  hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(256), 0, st, partial, n_krange, stride, n_tri, slot, norm, out);
  return hipGetLastError();
}

}  // namespace bispec
