// Triple contraction (step c, and c2 for the unit shells):
//   T(i, j, l) = sum_x F_i(x) F_j(x) F_l(x)      for the selected triangles,
// the numerator of eq. bsfin (data shells) and of eq. Ntri2 (unit shells).
//
// Work decomposition (geometry.h): rows are shell pairs (i, j), columns single
// shells l; a tile is 32 pairs x 32 consecutive shells in the vector kernels
// (a task <= 8 tiles), 16 x 16 in the split-bf16 MFMA kernel.
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

#include <type_traits>

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
// LDS chunk: [n_s + 1][ps] (voxel-contiguous per shell, row n_s all zero), so
// a thread reads kVec consecutive voxels of a shell with one 16-byte load;
// ps = kc + kVec puts consecutive shells an odd number of 16-byte bank groups
// apart (kc a multiple of 8 kVec).  Sums run in T over one chunk (<= 256
// voxels) and are then added into float64 totals: a long float32 chain would
// carry rounding error proportional to its running partial sum, which for
// shells of box-scale wavelength is far larger than the final (cancelling)
// total.
// ============================================================================
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float2 type;
  static constexpr int n = 2;
};
template <>
struct Vec16<double> {
  typedef double2 type;
  static constexpr int n = 2;
};
template <typename T>
__device__ __forceinline__ T vget(const typename Vec16<T>::type& v, int k);
template <>
__device__ __forceinline__ float vget<float>(const float2& v, int k) {
  return k == 0 ? v.x : v.y;
}
template <>
__device__ __forceinline__ double vget<double>(const double2& v, int k) {
  return k == 0 ? v.x : v.y;
}

template <typename T>
__global__ void __launch_bounds__(kThreads, 3) k_contract_vec(const T* __restrict__ F, ContractArgs a, int kc) {
  typedef typename Vec16<T>::type VT;
  constexpr int kVec = Vec16<T>::n;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* chunk = reinterpret_cast<T*>(smem_raw);
  int task, kr;
  xcd_map(a.n_tasks, task, kr);
  const int ns = a.n_s;
  const int ps = kc + kVec;  // row pitch (elements); row ns is the zero shell
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
    ri[u] = ((j > 0) ? i - 1 : ns) * ps;
    rj[u] = ((j > 0) ? j - 1 : ns) * ps;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int l = tile.col0 + 8 * cq + c;
    cl[c] = ((l >= 1 && l <= ns) ? l - 1 : ns) * ps;
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
  // zero shell row
  for (int x = threadIdx.x; x < kc; x += kThreads) chunk[ns * ps + x] = (T)0;
  for (long long x0 = k_lo; x0 < k_hi; x0 += kc) {
    const int len = (int)min((long long)kc, k_hi - x0);
    __syncthreads();
    // voxels x0 .. x0 + kc - 1 (zero past the range; x0 and kc are whole
    // 32-voxel blocks, whose 32 voxels of a shell are contiguous in F): lane
    // = voxel of the block, the 8 lane groups take shells g, g + 8, ...; eight
    // loads per thread are in flight before they are stored
    {
      const int lane = threadIdx.x & 31, g = threadIdx.x >> 5;
      for (int b = 0; b < kc / 32; ++b) {
        const int x = 32 * b + lane;
        const T* fb = F + ((x0 >> 5) + b) * (long long)ns * 32 + lane;
        for (int s0 = g; s0 < ns; s0 += 64) {
          T v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int sh = s0 + 8 * k;
            v[k] = (sh < ns && x < len) ? fb[sh * 32] : (T)0;
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int sh = s0 + 8 * k;
            if (sh < ns) chunk[sh * ps + x] = v[k];
          }
        }
      }
    }
    __syncthreads();
    if (!active) continue;
    if constexpr (kF32) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[u][c] = (T)0;
    }
    for (int x = 0; x < len; x += kVec) {
      VT vi[4], vj[4], vf[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        vi[u] = *reinterpret_cast<const VT*>(chunk + ri[u] + x);
        vj[u] = *reinterpret_cast<const VT*>(chunk + rj[u] + x);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) vf[c] = *reinterpret_cast<const VT*>(chunk + cl[c] + x);
#pragma unroll
      for (int k = 0; k < kVec; ++k) {
        T p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] = vget<T>(vi[u], k) * vget<T>(vj[u], k);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            if constexpr (kF32)
              acc[u][c] = fma(p[u], vget<T>(vf[c], k), acc[u][c]);
            else
              tot[u][c] = fma(p[u], vget<T>(vf[c], k), tot[u][c]);
          }
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
// dropped) by three v_mfma_f32_16x16x32_bf16 per 32 voxels.
//
// GEMM view per voxel range: C[(i,j), l] = sum_x A[(i,j), x] B[x, l] with the
// row operand A = F_i F_j (a pair product) and the column operand B = F_l.
// Tiles are 16 pairs x 16 shells: finer than 32 x 32 tiles, they waste less
// of the triangle wedge l <= j, j + l >= i (68 % of the tile entries are
// triangles at 100 shells, against 54 % for 32 x 32).
// Work group = kSlotsPerWg = 12 wavefronts (three per SIMD); wave w owns slot
// w: NT <= kMaxColTiles column tiles and n_rb <= slot_row_blocks(NT) row
// blocks that meet them (at most kSlotTiles = 16 accumulator tiles of 4 fp32
// per lane; NT is uniform over the wave, so the code path is too).  The
// matrix unit and the vector ALU of a SIMD overlap only in part on this chip
// (the VALU co-executes on about a third of the MFMA busy cycles), so the slot
// placement balances MFMA plus VALU cycles per SIMD.
//
// Voxel range kr is the set of voxel blocks kr + m n_krange (interleaved over
// the box).  Per chunk of 32 voxels (one block) each thread loads one 8-voxel
// segment (2 float4) of the work group's shell rows s_lo .. s_lo + s_n - 1
// (contiguous in the voxel-blocked layout) one chunk ahead, and stores it into
// the other LDS buffer as fp32 (row operands) and as bf16 hi/lo (column
// operands, split once per value) with four 16-byte stores.  Per chunk a lane
// (row or column lane % 16, voxel octet lane / 16) then
//   - reads its column fragments (hi, lo: 8 voxels of shell l each),
//   - for each row block reads 8 voxels of F_i and F_j, forms the 8 pair
//     products in registers, splits them (the MFMA row-operand layout), and
//     issues 3 MFMAs per column tile.
// There is no LDS round trip for the products and one barrier per chunk.
//
// LDS (two buffers): F32 [2][4][s + 1][8] fp32 (one plane per voxel octet),
// Bh/Bl [2][s + 1][48] bf16, with s = the largest s_n and the extra row all
// zero (padding rows and columns point there).  LDS has 128 banks of 4 bytes
// and serves a 16-byte read for lanes 0-31, then 32-63, i.e. 16 rows at two
// voxel octets: the bf16 row stride of 24 dwords puts 16 consecutive column
// shells at both octets on distinct banks, and the octet planes (16 bytes
// longer than their rows, an odd number of bank groups) put distinct pair
// shells of a block on distinct banks unless they differ by a multiple of 16.
// LDS addresses are 32-bit byte offsets from the shared array.
// Accumulation: fp32 MFMA chains of kFlushChunks chunks, added in float64 into
// partial[range][tile][element] (tile-major, coalesced); the reduction maps
// elements to triangles.  Output element (v, lane) of a tile is row
// 4 (lane / 16) + v, column lane % 16.
// ============================================================================
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC2 = 32;              // voxels per chunk (= one voxel block)
constexpr int kOct = kC2 / 8;        // voxel octets per chunk (one per 16 lanes of a wave)
constexpr int kBS = kC2 + 16;        // bf16 row stride (elements): 24 dwords
constexpr int kFlushChunks = 256;    // 8192 voxels per float32 accumulation chain
constexpr int kWsThreads = kSlotsPerWg * 64;
static_assert(kC2 == kVoxBlock, "chunks are voxel blocks");

// LDS byte layout for ns1 rows per buffer (row ns1 - 1 is all zero) and nsub
// = 2 rep buffers (double buffering of one voxel block per replica; buffer
// b rep + r holds replica r's block of chunk parity b):
//   F32 [nsub][kOct][ns1 * 8 + 4] fp32 | Bh [nsub][ns1][kBS] bf16 | Bl [nsub][ns1][kBS] bf16
// The fp32 rows are split by voxel octet: plane k holds octet k of every row
// (32 bytes per row) and the planes are 16 bytes longer than their rows, an
// odd number of 16-byte bank groups.
struct WsLayout {
  unsigned f_plane, f_buf; // bytes per fp32 octet plane and per fp32 buffer
  unsigned b_buf;          // bytes per buffer of one bf16 plane
  unsigned bh0, bl0;       // byte offsets of the Bh and Bl regions
};

__host__ __device__ __forceinline__ WsLayout ws_layout(int ns1, int nsub) {
  WsLayout y;
  y.f_plane = (unsigned)ns1 * 32 + 16;
  y.f_buf = kOct * y.f_plane;
  y.b_buf = (unsigned)ns1 * kBS * 2;
  y.bh0 = nsub * y.f_buf;
  y.bl0 = y.bh0 + nsub * y.b_buf;
  return y;
}

// hi = bf16(v) (round to nearest even) for two values, and the exact fp32 of each hi
__device__ __forceinline__ unsigned bf16_pair(float v0, float v1, float& h0, float& h1) {
  bf16x2 h;
  h[0] = (__bf16)v0;
  h[1] = (__bf16)v1;
  const unsigned u = __builtin_bit_cast(unsigned, h);
  h0 = __builtin_bit_cast(float, u << 16);
  h1 = __builtin_bit_cast(float, u & 0xffff0000u);
  return u;
}

__device__ __forceinline__ unsigned bf16_pack(float v0, float v1) {
  bf16x2 h;
  h[0] = (__bf16)v0;
  h[1] = (__bf16)v1;
  return __builtin_bit_cast(unsigned, h);
}

// Staging of one voxel block per replica and chunk: rows s_lo .. s_lo + s_n - 1,
// each 4 octets of 8 voxels (two float4, contiguous in global memory).  Thread
// tid serves replica rs = tid / (64 g16), g16 = ceil(s_n / 16), and within it
// staging index idx = tid % (64 g16): row 16 (idx / 64) + idx % 16, octet
// (idx / 16) % 4.  Lanes 0-31 of a wave, which LDS serves together, store 16
// rows at two octets, on distinct banks in both layouts; a wave still covers
// 16 whole rows (2 KiB contiguous) of global memory.
struct Seg {
  float4 a, b;
};

struct WsStage {
  int rs, row, oct;
  bool on;   // the thread stages a row
};

__device__ __forceinline__ WsStage ws_stage_of(int tid, int s_n, int rep) {
  const int per = 64 * ((s_n + 15) >> 4);
  WsStage q;
  q.rs = tid / per;
  const int idx = tid - q.rs * per;
  q.row = 16 * (idx >> 6) + (idx & 15);
  q.oct = (idx >> 4) & 3;
  q.on = q.rs < rep && q.row < s_n;
  return q;
}

// this thread's segment of replica rs's block blk0 + rs (if it exists)
__device__ __forceinline__ bool ws_load(const float* __restrict__ F, int n_s, long long blk0, long long n_blocks,
                                        const WgRows& wr, const WsStage& q, Seg& pf) {
  const long long blk = blk0 + q.rs;
  if (!q.on || blk >= n_blocks) return false;
  const float4* base = reinterpret_cast<const float4*>(F + blk * (long long)n_s * kC2 + (long long)wr.s_lo * kC2);
  const int o = 2 * (kOct * q.row + q.oct);
  pf.a = base[o];
  pf.b = base[o + 1];
  return true;
}

// fp32 row segment, and the bf16 split hi = bf16(v), lo = bf16(v - hi) of
// every value, into buffer sub: four 16-byte stores
__device__ __forceinline__ void ws_store(unsigned char* lds, const WsLayout& y, int sub, const WsStage& q,
                                         const Seg& pf) {
  const unsigned r = q.row, k = q.oct, x = 8 * k;
  unsigned char* f = lds + sub * y.f_buf + k * y.f_plane + r * 32;
  *reinterpret_cast<float4*>(f) = pf.a;
  *reinterpret_cast<float4*>(f + 16) = pf.b;
  const float v[8] = {pf.a.x, pf.a.y, pf.a.z, pf.a.w, pf.b.x, pf.b.y, pf.b.z, pf.b.w};
  u32x4 hi, lo;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float h0, h1;
    hi[e] = bf16_pair(v[2 * e], v[2 * e + 1], h0, h1);
    lo[e] = bf16_pack(v[2 * e] - h0, v[2 * e + 1] - h1);
  }
  const unsigned o = sub * y.b_buf + (r * kBS + x) * 2;
  *reinterpret_cast<u32x4*>(lds + y.bh0 + o) = hi;
  *reinterpret_cast<u32x4*>(lds + y.bl0 + o) = lo;
}

// Row operand of one row block for 8 voxels: F_i and F_j (8 floats each) are
// read into registers first (ws_row_read), and the products p = F_i F_j are
// split later (ws_row_split) into hi = bf16(p) and lo = bf16(F_i F_j - hi)
// (the fma keeps lo exact), so the reads of one block can be issued before
// the previous block's products and MFMAs.
struct RowIn {
  float4 i0, i1, j0, j1;
};

__device__ __forceinline__ RowIn ws_row_read(const unsigned char* lds, unsigned oi, unsigned oj) {
  RowIn r;
  r.i0 = *reinterpret_cast<const float4*>(lds + oi);
  r.i1 = *reinterpret_cast<const float4*>(lds + oi + 16);
  r.j0 = *reinterpret_cast<const float4*>(lds + oj);
  r.j1 = *reinterpret_cast<const float4*>(lds + oj + 16);
  return r;
}

__device__ __forceinline__ void ws_row_split(const RowIn& r, bf16x8& ahi, bf16x8& alo) {
  const float a[8] = {r.i0.x, r.i0.y, r.i0.z, r.i0.w, r.i1.x, r.i1.y, r.i1.z, r.i1.w};
  const float b[8] = {r.j0.x, r.j0.y, r.j0.z, r.j0.w, r.j1.x, r.j1.y, r.j1.z, r.j1.w};
  u32x4 h, l;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float h0, h1;
    h[e] = bf16_pair(a[2 * e] * b[2 * e], a[2 * e + 1] * b[2 * e + 1], h0, h1);
    l[e] = bf16_pack(__builtin_fmaf(a[2 * e], b[2 * e], -h0), __builtin_fmaf(a[2 * e + 1], b[2 * e + 1], -h1));
  }
  ahi = __builtin_bit_cast(bf16x8, h);
  alo = __builtin_bit_cast(bf16x8, l);
}

// 3 MFMAs per tile: hi*hi + hi*lo + lo*hi (16 x 16 output, K = 32 voxels)
__device__ __forceinline__ void ws_mfma3(const bf16x8& ahi, const bf16x8& alo, const bf16x8& bhi, const bf16x8& blo,
                                         f32x4& c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, c, 0, 0, 0);
}

// One chunk (32 voxels of buffer buf) for a slot with NT column tiles and
// NRB row blocks (accumulator tile q * NT + t); both are template parameters,
// so every slot shape runs straight-line code with constant indices (the
// accumulators stay in registers).  fo[q], go[q]: byte offsets of this lane's
// F_i and F_j rows (+ its voxel octet) in buffer 0; co[t]: of its column row
// in plane Bh, buffer 0.
// NT <= 4 ("tall"): the column fragments of all tiles stay in registers and
// the row blocks stream through, one block ahead: block q + 1 is split while
// block q's MFMAs run, and block q + 2's rows are read.  NT >= 5 ("wide",
// NRB <= 3): the row operands of all blocks stay in registers and the column
// fragments stream through.
template <int NT, int NRB>
__device__ __forceinline__ void ws_compute(const unsigned char* lds, const WsLayout& y, int buf,
                                           const unsigned* fo, const unsigned* go, const unsigned* co, f32x4* acc) {
  const unsigned fb = buf * y.f_buf, bb = y.bh0 + buf * y.b_buf, lb = y.bl0 + buf * y.b_buf;
  if constexpr (NT <= 4) {
    bf16x8 bhi[NT], blo[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bhi[t] = *reinterpret_cast<const bf16x8*>(lds + bb + co[t]);
      blo[t] = *reinterpret_cast<const bf16x8*>(lds + lb + co[t]);
    }
    // two register sets for the row operand, used alternately: block q's
    // MFMAs read set q & 1 while block q + 1 is split into the other set (so
    // the split never overwrites an operand an MFMA in flight still reads)
    // and block q + 2's rows are read from LDS
    bf16x8 ahi[2], alo[2];
    RowIn r = ws_row_read(lds, fb + fo[0], fb + go[0]);
    ws_row_split(r, ahi[0], alo[0]);
    if (NRB > 1) r = ws_row_read(lds, fb + fo[1 % NRB], fb + go[1 % NRB]);
#pragma unroll
    for (int q = 0; q < NRB; ++q) {
      if (q + 1 < NRB) ws_row_split(r, ahi[(q + 1) & 1], alo[(q + 1) & 1]);
      if (q + 2 < NRB) r = ws_row_read(lds, fb + fo[(q + 2) % NRB], fb + go[(q + 2) % NRB]);
#pragma unroll
      for (int t = 0; t < NT; ++t) ws_mfma3(ahi[q & 1], alo[q & 1], bhi[t], blo[t], acc[q * NT + t]);
    }
  } else {
    bf16x8 ahi[NRB], alo[NRB];
#pragma unroll
    for (int q = 0; q < NRB; ++q) ws_row_split(ws_row_read(lds, fb + fo[q], fb + go[q]), ahi[q], alo[q]);
    bf16x8 bhi = *reinterpret_cast<const bf16x8*>(lds + bb + co[0]);
    bf16x8 blo = *reinterpret_cast<const bf16x8*>(lds + lb + co[0]);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x8 nhi = bhi, nlo = blo;
      if (t + 1 < NT) {
        nhi = *reinterpret_cast<const bf16x8*>(lds + bb + co[t + 1]);
        nlo = *reinterpret_cast<const bf16x8*>(lds + lb + co[t + 1]);
      }
#pragma unroll
      for (int q = 0; q < NRB; ++q) ws_mfma3(ahi[q], alo[q], bhi, blo, acc[q * NT + t]);
      bhi = nhi;
      blo = nlo;
    }
  }
}

// float64 flush of the slot's accumulators (first: write, else add), then reset.
// The base pointer passes through an empty asm so the element addresses are
// formed here, not hoisted out of the main loop into live registers.
template <int NT, int NRB>
__device__ __forceinline__ void ws_flush(double* out, bool first, f32x4* acc) {
  asm volatile("" : "+v"(out));
#pragma unroll
  for (int k = 0; k < NRB * NT; ++k) {
    double* o = out + (long long)k * kMTileElems;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      o[v * 64] = first ? (double)acc[k][v] : o[v * 64] + (double)acc[k][v];
      acc[k][v] = 0.f;
    }
  }
}

// Chunk c of a work group stages, for each replica r, voxel block
// rep kr + r + c rep n_krange (when it exists) into buffer (c & 1) rep + r.
// Replica r's voxel range rep kr + r thus takes the blocks rep kr + r,
// + rep n_krange, + 2 rep n_krange, ...: every float32 chain samples the whole
// box, so its partial sums cancel like the total instead of growing with a
// slab's coherent sum.  n_chunks: chunks of the work group (those of replica
// 0, the longest); n_mine: those of this wave's replica.
struct WsChunks {
  long long blk0, step, n_blocks;   // replica 0's first block, blocks per chunk step, blocks of the box
  int n_chunks, n_mine, rep, sub;   // sub: this wave's replica (its buffer within a parity)
};

template <int NT, int NRB>
__device__ __forceinline__ void ws_run(const float* __restrict__ F, const WsArgs& a, unsigned char* lds,
                                       const WsLayout& y, const WgRows& wr, const WsChunks& ch, const WsStage& q,
                                       int tid, const SlotCols& sc, const MRowBlock* rows, double* out) {
  const int lane = tid & 63, kg = lane >> 4, zr = wr.s_n;
  // this lane's rows (pair shells) and columns as byte offsets in buffer 0
  unsigned fo[NRB], go[NRB], co[NT];
#pragma unroll
  for (int q = 0; q < NRB; ++q) {
    const MRowBlock& rb = rows[q];
    const int i = rb.i[lane & 15], j = rb.j[lane & 15];
    const int ri = j > 0 ? i - 1 - wr.s_lo : zr, rj = j > 0 ? j - 1 - wr.s_lo : zr;
    fo[q] = kg * y.f_plane + ri * 32;
    go[q] = kg * y.f_plane + rj * 32;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int l = sc.col0[t] + (lane & 15);  // 1-based column shell
    const int rc = (l >= 1 && l <= a.n_s) ? l - 1 - wr.s_lo : zr;
    co[t] = (unsigned)(rc * kBS + kg * 8) * 2;
  }
  f32x4 acc[NRB * NT];
#pragma unroll
  for (int k = 0; k < NRB * NT; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[k][v] = 0.f;
  Seg pf;
  if (ch.n_chunks > 0 && ws_load(F, a.n_s, ch.blk0, ch.n_blocks, wr, q, pf)) ws_store(lds, y, q.rs, q, pf);
  __syncthreads();
  bool first = true;
  int chain = 0;
  for (int c = 0; c < ch.n_chunks; ++c) {
    const bool more = c + 1 < ch.n_chunks;
    const bool got = more && ws_load(F, a.n_s, ch.blk0 + (c + 1) * ch.step, ch.n_blocks, wr, q, pf);
    if (c < ch.n_mine) {
      ws_compute<NT, NRB>(lds, y, (c & 1) * ch.rep + ch.sub, fo, go, co, acc);
      if (++chain == kFlushChunks || c + 1 == ch.n_mine) {
        ws_flush<NT, NRB>(out, first, acc);
        chain = 0;
        first = false;
      }
    }
    if (got) ws_store(lds, y, ((c + 1) & 1) * ch.rep + q.rs, q, pf);
    __syncthreads();
  }
}

// A wave without a slot only stages its share of every chunk.
__device__ __forceinline__ void ws_idle(const float* __restrict__ F, const WsArgs& a, unsigned char* lds,
                                        const WsLayout& y, const WgRows& wr, const WsChunks& ch, const WsStage& q) {
  Seg pf;
  if (ch.n_chunks > 0 && ws_load(F, a.n_s, ch.blk0, ch.n_blocks, wr, q, pf)) ws_store(lds, y, q.rs, q, pf);
  __syncthreads();
  for (int c = 0; c < ch.n_chunks; ++c) {
    // buffers of parity (c + 1) & 1 were last read in chunk c - 1, before the previous barrier
    if (c + 1 < ch.n_chunks && ws_load(F, a.n_s, ch.blk0 + (c + 1) * ch.step, ch.n_blocks, wr, q, pf))
      ws_store(lds, y, ((c + 1) & 1) * ch.rep + q.rs, q, pf);
    __syncthreads();
  }
}

// One launch over several groups (the estimator-grid classes of a plan, or of
// every member of a batch): group q owns blocks [block0, block0 + n_wg n_krange)
// (block0 a multiple of 8, so the local block index keeps the XCD of the
// global one), reads its fields at F + f_off and writes its partials at
// partial + p_off.
__device__ __forceinline__ int ws_group_of(const WsGroup* __restrict__ groups, int n_groups, int b) {
  int lo = 0, hi = n_groups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(kWsThreads) k_contract_bf16x3(const float* __restrict__ F_all,
                                                                double* __restrict__ partial_all,
                                                                const WsGroup* __restrict__ groups, int n_groups) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const WsGroup& grp = groups[ws_group_of(groups, n_groups, (int)blockIdx.x)];
  WsArgs a;
  a.rows = grp.rows;
  a.cols = grp.cols;
  a.wg_rows = grp.wg_rows;
  a.n_wg = grp.n_wg;
  a.n_s = grp.n_s;
  a.max_s = grp.max_s;
  a.n_vox = grp.n_vox;
  a.n_krange = grp.n_krange;
  a.rep = grp.rep;
  a.tile_stride = grp.tile_stride;
  a.partial = partial_all + grp.p_off;
  const float* __restrict__ F = F_all + grp.f_off;
  const int ns1 = a.max_s + 1, rep = a.rep;
  const WsLayout y = ws_layout(ns1, 2 * rep);
  int wg, kr;
  {
    const int b = (int)blockIdx.x - grp.block0;
    const int xcd = b & 7, qq = b >> 3;
    wg = qq % a.n_wg;
    kr = xcd + 8 * (qq / a.n_wg);
  }
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const WgRows wr = a.wg_rows[wg];
  const int zr = wr.s_n;  // the zero row
  // zero row of each buffer, never overwritten afterwards
  for (int e = tid; e < 2 * rep * kOct * 8; e += kWsThreads)
    *reinterpret_cast<float*>(smem_raw + (e / 8) * y.f_plane + zr * 32 + (e % 8) * 4) = 0.f;
  for (int e = tid; e < 2 * rep * kBS; e += kWsThreads) {
    const unsigned o = (e / kBS) * y.b_buf + (zr * kBS + e % kBS) * 2;
    *reinterpret_cast<__bf16*>(smem_raw + y.bh0 + o) = (__bf16)0.f;
    *reinterpret_cast<__bf16*>(smem_raw + y.bl0 + o) = (__bf16)0.f;
  }
  // wave w runs slot w % wpr of replica w / wpr
  const int wpr = kSlotsPerWg / rep, r = w / wpr, ws = w - r * wpr;
  const SlotCols sc = a.cols[wg * kSlotsPerWg + ws];
  const MRowBlock* rows = a.rows + wg * kRbPerWg + ws * kMaxRbPerSlot;
  // this replica's voxel range kr rep + r of rep n_krange; partial[range][tile][element]
  // with tile = wg*kTilesPerWg + ws*kSlotTiles + (q*NT + t) < tile_stride for busy slots
  const long long kre = (long long)kr * rep + r, n_kre = (long long)a.n_krange * rep;
  double* out = a.partial +
                (kre * a.tile_stride + (long long)wg * kTilesPerWg + (long long)ws * kSlotTiles) * kMTileElems + lane;
  WsChunks ch;
  ch.n_blocks = a.n_vox / kC2;
  ch.blk0 = (long long)kr * rep;
  ch.step = n_kre;
  ch.rep = rep;
  ch.sub = r;
  ch.n_chunks = ch.blk0 < ch.n_blocks ? (int)((ch.n_blocks - ch.blk0 + n_kre - 1) / n_kre) : 0;
  ch.n_mine = kre < ch.n_blocks ? (int)((ch.n_blocks - kre + n_kre - 1) / n_kre) : 0;
  if (ch.n_mine == 0 && sc.n > 0)  // empty range: a busy slot's partials are zero
    for (int e = 0; e < kSlotTiles * 4; ++e) out[(long long)(e >> 2) * kMTileElems + (e & 3) * 64] = 0.0;
  const WsStage q = ws_stage_of(tid, wr.s_n, rep);
  // every wave passes the same barriers whatever its variant (uniform per wave)
  switch (sc.n * 16 + sc.n_rb) {
#define WS_CASE(N, R) \
  case N * 16 + R: ws_run<N, R>(F, a, smem_raw, y, wr, ch, q, tid, sc, rows, out); break;
    WS_CASE(1, 1) WS_CASE(1, 2) WS_CASE(1, 3) WS_CASE(1, 4) WS_CASE(1, 5) WS_CASE(1, 6) WS_CASE(1, 7) WS_CASE(1, 8)
    WS_CASE(2, 1) WS_CASE(2, 2) WS_CASE(2, 3) WS_CASE(2, 4) WS_CASE(2, 5) WS_CASE(2, 6) WS_CASE(2, 7) WS_CASE(2, 8)
    WS_CASE(3, 1) WS_CASE(3, 2) WS_CASE(3, 3) WS_CASE(3, 4) WS_CASE(3, 5)
    WS_CASE(4, 1) WS_CASE(4, 2) WS_CASE(4, 3) WS_CASE(4, 4)
    WS_CASE(5, 1) WS_CASE(5, 2) WS_CASE(5, 3)
    WS_CASE(6, 1) WS_CASE(6, 2) WS_CASE(7, 1) WS_CASE(7, 2) WS_CASE(8, 1) WS_CASE(8, 2)
#undef WS_CASE
    default: ws_idle(F, a, smem_raw, y, wr, ch, q); break;
  }
}

// ============================================================================
// Adjoint field build (gradient of L = sum_t gB_t B_t with respect to the
// scaled shell fields): for every shell n and voxel x
//   G_n(x) = sum over the terms (t, j, l) of n of w_t F_j(x) F_l(x),
// where each selected triangle (a1, a2, a3) contributes the terms (t, a2, a3)
// to G_a1, (t, a1, a3) to G_a2 and (t, a1, a2) to G_a3 (the three factors of
// d(F_a1 F_a2 F_a3)), and w_t = gB_t * norm_t.  Thread = voxel; the F block
// of kGbVox voxels x n_s shells is staged in LDS; G is written voxel-blocked.
// The weights and each voxel's sum over its terms are float64 (the weights of
// one shell span many orders of magnitude and a shell collects thousands of
// terms); G itself is rounded to float32 for the adjoint transforms.
// ============================================================================
constexpr int kGbVox = 128;

__global__ void k_gweights(const double* __restrict__ gB, const double* __restrict__ norm,
                           const int4* __restrict__ terms, long long n_terms, double* __restrict__ w) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_terms) w[k] = gB[terms[k].x] * norm[terms[k].x];
}

__global__ void __launch_bounds__(kGbVox) k_gbuild(const float* __restrict__ F, const int4* __restrict__ terms,
                                                   const double* __restrict__ w,
                                                   const int32_t* __restrict__ term_off, int n_s,
                                                   float* __restrict__ G) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* f = reinterpret_cast<float*>(smem_raw);  // [n_s][kGbVox]
  const long long blk0 = (long long)blockIdx.x * (kGbVox / kVoxBlock);
  // stage: kGbVox/32 consecutive voxel blocks, each n_s x 32 contiguous, so
  // element e of the group's piece of F is at src[e]; eight loads per thread
  // are in flight before they are stored
  const float* src = F + blk0 * (long long)n_s * kVoxBlock;
  const int total = n_s * kGbVox;
  for (int e0 = threadIdx.x; e0 < total; e0 += 8 * kGbVox) {
    float val[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = e0 + k * kGbVox;
      val[k] = e < total ? src[e] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = e0 + k * kGbVox;
      if (e >= total) continue;
      const int b = e / (n_s * kVoxBlock), r = e % (n_s * kVoxBlock);
      f[(r / kVoxBlock) * kGbVox + b * kVoxBlock + r % kVoxBlock] = val[k];
    }
  }
  __syncthreads();
  const int v = threadIdx.x;
  float* g = G + (blk0 + v / kVoxBlock) * (long long)n_s * kVoxBlock + (v % kVoxBlock);
  for (int n = 0; n < n_s; ++n) {
    double acc = 0.0;
    const int k1 = term_off[n + 1];
    for (int k = term_off[n]; k < k1; ++k) {
      const int4 tm = terms[k];
      acc = fma(w[k] * (double)f[tm.y * kGbVox + v], (double)f[tm.z * kGbVox + v], acc);
    }
    g[n * kVoxBlock] = (float)acc;
  }
}

// Fixed-order float64 reduction over the voxel ranges: T_t = sum_k
// partial[k][slot_t], times norm_t (eq. FBE normalisation) when given.  A block
// takes kRedTri triangles, lane (tl, p): triangle tl, ranges k = p, p + kRedPart,
// ...; the kRedPart partial sums are then added in the order p = 0, 1, ...
// (deterministic).  Lanes run over the triangles, whose slots are mostly
// neighbouring tile elements, so the loads of one range coalesce.
constexpr int kRedTri = 16, kRedPart = 16;
__global__ void __launch_bounds__(kRedTri * kRedPart) k_reduce(const double* __restrict__ partial, int n_krange,
                                                              long long stride, long long n_tri,
                                                              const int32_t* __restrict__ slot,
                                                              const double* __restrict__ norm,
                                                              const int32_t* __restrict__ out_idx,
                                                              double* __restrict__ out, int accumulate) {
  __shared__ double part[kRedPart][kRedTri];
  const int tl = threadIdx.x % kRedTri, p = threadIdx.x / kRedTri;
  const long long t = (long long)blockIdx.x * kRedTri + tl;
  double s = 0.0;
  if (t < n_tri) {
    const long long at = slot ? slot[t] : t;
    for (int k = p; k < n_krange; k += kRedPart) s += partial[(long long)k * stride + at];
  }
  part[p][tl] = s;
  __syncthreads();
  if (p == 0 && t < n_tri) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < kRedPart; ++q) r += part[q][tl];
    const long long o = out_idx ? out_idx[t] : t;
    const double v = norm ? r * norm[o] : r;
    out[o] = accumulate ? out[o] + v : v;   // accumulate: the slabs of a streamed grid, in order
  }
}

__global__ void __launch_bounds__(kRedTri * kRedPart) k_reduce_grouped(const RedGroup* __restrict__ groups,
                                                                      int n_groups, double* __restrict__ B) {
  int lo = 0, hi = n_groups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].block0 <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const RedGroup& g = groups[lo];
  __shared__ double part[kRedPart][kRedTri];
  const int tl = threadIdx.x % kRedTri, p = threadIdx.x / kRedTri;
  const long long t = (long long)((int)blockIdx.x - g.block0) * kRedTri + tl;
  double s = 0.0;
  if (t < g.n_tri) {
    const long long at = g.slot[t];
    for (int k = p; k < g.n_krange; k += kRedPart) s += g.partial[(long long)k * g.stride + at];
  }
  part[p][tl] = s;
  __syncthreads();
  if (p == 0 && t < g.n_tri) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < kRedPart; ++q) r += part[q][tl];
    const long long o = g.out_idx[t];
    B[g.b_off + o] = r * g.norm[o];
  }
}

// chunk voxels kc of the vector kernels: whole 32-voxel blocks (a multiple of
// 8 x the voxels per load), <= 256, LDS <= 40 KB where one block fits; plans
// with more shells (>= 150 in float64) stage one block per chunk in up to
// kVecLdsMax bytes (the limit is raised at plan time)
constexpr size_t kVecLdsMax = 80 * 1024;
template <typename T>
int vec_chunk(int n_s) {
  constexpr int kVec = Vec16<T>::n;
  const int ls = n_s + 1;
  int kc = (int)((40 * 1024) / ((size_t)ls * sizeof(T))) - kVec;
  kc = kc >= 256 ? 256 : (kc / 32) * 32;
  if (kc < 32 && (size_t)(32 + kVec) * ls * sizeof(T) <= kVecLdsMax) kc = 32;
  return kc;
}

template <typename T>
hipError_t launch_vec(const T* F, const ContractArgs& a, hipStream_t st) {
  constexpr int kVec = Vec16<T>::n;
  static_assert(32 % (8 * kVec) == 0, "a voxel block holds whole load groups");
  const int ls = a.n_s + 1;
  const int kc = vec_chunk<T>(a.n_s);
  if (kc < 32 || a.n_vox % 32 != 0) return hipErrorInvalidValue;
  const size_t lds = (size_t)(kc + kVec) * ls * sizeof(T);
  const unsigned blocks = (unsigned)a.n_tasks * (unsigned)a.n_krange;
  hipLaunchKernelGGL(k_contract_vec<T>, dim3(blocks), dim3(kThreads), lds, st, F, a, kc);
  return hipGetLastError();
}

// ============================================================================
// Adjoint field build on the matrix cores (kernels.h): for every grid class,
// work group (wg, kr) holds the output shells n of its wavefronts and walks
// the voxel chunks kr, kr + n_krange, ... of kAdjVox = 64 voxels (two voxel
// blocks; 128-voxel chunks, one work group per CU, ran 21 % slower, 32-voxel
// ones 14 %).  Per chunk the group stages every shell of the class into LDS as
//   Bh, Bl [64][S_row] bf16 hi and lo (shell-contiguous per voxel; the shells
//   past n_s stay zero, up to the end of any K tile, which reaches at most 31
//   shells past the last), S_row = 128 + 31 rounded up to 32, plus 8, for
//   every class (a compile-time stride folds the LDS offsets into the reads),
//   and Ff [n_s + 1][64] float32 (row n_s all zero: padding rows of a block),
// then each wavefront, for each of its shells n and each row block of n:
//   acc[vt] (16 rows x 16 voxels of voxel tile vt) = sum over its K tiles of
//   W_hi F_hi + W_hi F_lo + W_lo F_hi (v_mfma_f32_16x16x32_bf16; W from the
//   weight buffer, one 16-byte load of hi and of lo per lane per K tile, used
//   for all four voxel tiles),
// and adds acc's rows times F_j (each lane's four rows summed in float32, then
// added in float64) into the shell's sums; the sum over the four row groups of
// a lane column ends the shell, and lanes 0-15 write
// G_n of the chunk.  Every shell n of the class belongs to exactly one
// wavefront (shells without rows write zeros), so G is written once.
// ============================================================================
__host__ __device__ constexpr int adj_spad(int n_s) { return (n_s + 31 + kAdjK - 1) / kAdjK * kAdjK; }
__host__ __device__ constexpr int adj_srow(int n_s) { return adj_spad(n_s) + 8; }
constexpr int kAdjSrow = adj_srow(kMaxSplitShells);   // one row stride for every class: LDS offsets fold into immediates

__device__ __forceinline__ int adj_group_of(const AdjGroup* __restrict__ groups, int n_groups, int b) {
  int lo = 0, hi = n_groups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_adj_weights(const double* __restrict__ gB, const double* __restrict__ norm,
                              const int32_t* __restrict__ off, const int32_t* __restrict__ tri, long long n_tiles,
                              uint16_t* __restrict__ W) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // tile * 64 + lane
  if (q >= n_tiles * 64) return;
  const long long tile = q >> 6;
  const int lane = (int)(q & 63);
  u32x4 hi, lo;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float h[2], l[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long long slot = q * 8 + 2 * e + u;
      double w = 0.0;
      for (int k = off[slot]; k < off[slot + 1]; ++k) w += gB[tri[k]] * norm[tri[k]];
      h[u] = (float)w;
      l[u] = (float)(w - (double)(float)(__bf16)h[u]);
    }
    float h0, h1;
    hi[e] = bf16_pair(h[0], h[1], h0, h1);
    lo[e] = bf16_pack(l[0], l[1]);
  }
  *reinterpret_cast<u32x4*>(W + tile * 1024 + lane * 8) = hi;
  *reinterpret_cast<u32x4*>(W + tile * 1024 + 512 + lane * 8) = lo;
}

__global__ void __launch_bounds__(kAdjWaves * 64) k_adjoint_mfma(const float* __restrict__ F_all,
                                                                 float* __restrict__ G_all,
                                                                 const AdjGroup* __restrict__ groups, int n_groups) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const AdjGroup& grp = groups[adj_group_of(groups, n_groups, (int)blockIdx.x)];
  const int b = (int)blockIdx.x - grp.block0;
  const int xcd = b & 7, qb = b >> 3;
  const int wg = qb % grp.n_wg, kr = xcd + 8 * (qb / grp.n_wg);
  const int ns = grp.n_s;
  constexpr int srow = kAdjSrow;
  constexpr int kThr = kAdjWaves * 64;
  __bf16* Bh = reinterpret_cast<__bf16*>(smem_raw);
  __bf16* Bl = Bh + kAdjVox * srow;
  float* Ff = reinterpret_cast<float*>(smem_raw + 2 * (size_t)kAdjVox * srow * 2);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int e = tid; e < kAdjVox; e += kThr) Ff[ns * kAdjVox + e] = 0.f;
  for (int e = tid; e < kAdjVox * (srow - ns); e += kThr) {
    const int v = e / (srow - ns), c = ns + e % (srow - ns);
    Bh[v * srow + c] = (__bf16)0.f;
    Bl[v * srow + c] = (__bf16)0.f;
  }
  const float* __restrict__ F = F_all + grp.f_off;
  float* __restrict__ G = G_all + grp.f_off;
  const long long n_chunks = grp.n_vox / kAdjVox;
  const AdjWave wv = grp.waves[wg * kAdjWaves + w];
  constexpr int kVt = kAdjVox / 16, kBlk = kAdjVox / 32;   // voxel tiles and voxel blocks of a chunk
  const int total = kBlk * ns * 32;
  for (long long c = kr; c < n_chunks; c += grp.n_krange) {
    __syncthreads();  // the previous chunk's reads (and the zeroing) are done
    // stage: the chunk's voxel blocks are contiguous in F (element e:
    // block e / (32 n_s), shell (e / 32) % n_s, voxel e % 32); eight loads in flight
    const float* src = F + c * (long long)total;
    for (int e0 = tid; e0 < total; e0 += 8 * kThr) {
      float val[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThr;
        val[u] = e < total ? src[e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThr;
        if (e >= total) continue;
        const int blk = e / (ns * 32), r = e - blk * ns * 32, sh = r >> 5, vox = blk * 32 + (r & 31);
        Ff[sh * kAdjVox + vox] = val[u];
        const __bf16 h = (__bf16)val[u];
        Bh[vox * srow + sh] = h;
        Bl[vox * srow + sh] = (__bf16)(val[u] - (float)h);
      }
    }
    __syncthreads();
    for (int e = wv.e0; e < wv.e1; ++e) {
      const AdjN nn = grp.ns[e];
      double sacc[kVt];
#pragma unroll
      for (int vt = 0; vt < kVt; ++vt) sacc[vt] = 0.0;
      for (int r = nn.rb0; r < nn.rb1; ++r) {
        const AdjRowBlock& rb = grp.rbs[r];
        const int l8 = rb.l8, nkt = rb.nkt;
        const uint16_t* wt = grp.W + (long long)rb.w_tile * 1024 + lane * 8;
        int jrow[4];   // this lane's rows, read before the K loop so the loads overlap it
#pragma unroll
        for (int v = 0; v < 4; ++v) jrow[v] = rb.j[4 * (lane >> 4) + v];
        f32x4 acc[kVt];
#pragma unroll
        for (int vt = 0; vt < kVt; ++vt)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[vt][v] = 0.f;
        for (int kt = 0; kt < nkt; ++kt) {
          const bf16x8 ahi = *reinterpret_cast<const bf16x8*>(wt + kt * 1024);
          const bf16x8 alo = *reinterpret_cast<const bf16x8*>(wt + kt * 1024 + 512);
          const int l0 = 8 * l8 + kt * kAdjK + 8 * (lane >> 4);
#pragma unroll
          for (int vt = 0; vt < kVt; ++vt) {
            const int vox = vt * 16 + (lane & 15);
            const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(Bh + vox * srow + l0);
            const bf16x8 blo = *reinterpret_cast<const bf16x8*>(Bl + vox * srow + l0);
            ws_mfma3(ahi, alo, bhi, blo, acc[vt]);
          }
        }
        // row 4 (lane / 16) + v of the block, voxel lane % 16 of each voxel tile:
        // the lane's four rows times F_j, summed in float32, then added in float64
        const float* fj[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = jrow[v];
          fj[v] = Ff + (j > 0 ? j - 1 : ns) * kAdjVox + (lane & 15);
        }
#pragma unroll
        for (int vt = 0; vt < kVt; ++vt) {
          float s = acc[vt][0] * fj[0][vt * 16];
#pragma unroll
          for (int v = 1; v < 4; ++v) s = __builtin_fmaf(acc[vt][v], fj[v][vt * 16], s);
          sacc[vt] += (double)s;
        }
      }
#pragma unroll
      for (int vt = 0; vt < kVt; ++vt) {
        double t = sacc[vt];
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        sacc[vt] = t;
      }
      if (lane < 16) {
#pragma unroll
        for (int vt = 0; vt < kVt; ++vt) {
          const int vox = vt * 16 + lane;
          G[(c * kBlk + (vox >> 5)) * (long long)ns * 32 + (long long)(nn.n - 1) * 32 + (vox & 31)] = (float)sacc[vt];
        }
      }
    }
  }
}

// ============================================================================
// Order-4 contraction (Section 4's polyspectrum with p = 4):
//   T(a1, a2, a3, a4) = sum_x P_(a1,a2)(x) P_(a3,a4)(x),  P_(i,j) = F_i F_j,
// a GEMM of row pairs against column pairs over the voxels.  Work group
// (wg, kr) walks the voxel blocks kr, kr + n_krange, ... (32 voxels each): it
// stages the block's fields (float32 or float64) in LDS, forms every pair
// product of the plan once per block into LDS (split into bf16 hi and lo, or
// kept in float64), and each wavefront adds its tiles' 16 x 16 products:
//   split-bf16: 3 v_mfma_f32_16x16x32_bf16 per tile (hi hi + hi lo + lo hi),
//     float32 chains of kFlushChunks blocks flushed into float64 partials;
//   float64: 8 v_mfma_f64_16x16x4_f64 per tile (K = 4 voxels each), float64
//     throughout (the exact N_quad of the unit shells).
// Row block rb's lane r (0..15) holds pair rb_pairs[16 rb + r] (the zero pair
// for padding), likewise for columns.  The split-bf16 accumulator's element
// (v, lane) is row 4 (lane / 16) + v, column lane % 16, as in the triple
// contraction; the float64 MFMA's is row 4 v + lane / 16, column lane % 16,
// and is stored at the position the first layout gives that (row, column), so
// one slot table serves both.
// ============================================================================
constexpr int kQStride = kC2 + 8;   // bf16 elements per pair row (80 bytes: bank spread)

template <bool F64>
__global__ void __launch_bounds__(kWsThreads) k_contract4(const void* __restrict__ Fv, Quad4Args a) {
  typedef typename std::conditional<F64, double, float>::type T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const T* __restrict__ F = reinterpret_cast<const T*>(Fv);
  int wg, kr;
  xcd_map(a.n_wg, wg, kr);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int ns = a.n_s, np = a.n_pairs;
  // LDS: fields [ns + 1][32] (row ns zero), then the pair products
  T* ff = reinterpret_cast<T*>(smem_raw);
  unsigned char* pbase = smem_raw + (size_t)(ns + 1) * kC2 * sizeof(T);
  for (int e = tid; e < kC2; e += kWsThreads) ff[ns * kC2 + e] = (T)0;
  // the zero pair row
  if constexpr (F64) {
    double* pp = reinterpret_cast<double*>(pbase);
    for (int e = tid; e < kC2; e += kWsThreads) pp[np * kC2 + e] = 0.0;
  } else {
    __bf16* ph = reinterpret_cast<__bf16*>(pbase);
    __bf16* pl = ph + (size_t)(np + 1) * kQStride;
    for (int e = tid; e < kQStride; e += kWsThreads) {
      ph[np * kQStride + e] = (__bf16)0.f;
      pl[np * kQStride + e] = (__bf16)0.f;
    }
  }
  // this wavefront's tiles (<= kSlotTiles) and its lane's row and column pairs
  const int wid = wg * kSlotsPerWg + w;
  const int t0 = a.wave_t0[wid], nt = a.wave_t0[wid + 1] - t0;
  int prow[kSlotTiles], pcol[kSlotTiles];
#pragma unroll
  for (int k = 0; k < kSlotTiles; ++k) {
    if (k < nt) {
      const int4 td = a.tiles[t0 + k];
      prow[k] = a.rb_pairs[td.y * 16 + (lane & 15)];
      pcol[k] = a.cb_pairs[td.z * 16 + (lane & 15)];
    } else {
      prow[k] = pcol[k] = np;
    }
  }
  typedef typename std::conditional<F64, double, float>::type A;
  typedef A acc4 __attribute__((ext_vector_type(4)));
  acc4 acc[kSlotTiles];
#pragma unroll
  for (int k = 0; k < kSlotTiles; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[k][v] = (A)0;
  double* out = a.partial + (long long)kr * a.n_wg * kTilesPerWg * kMTileElems;
  const long long n_blocks = a.n_vox / kC2;
  bool first = true;
  int chain = 0;
  for (long long blk = kr; blk < n_blocks; blk += a.n_krange) {
    __syncthreads();   // the previous block's reads are done
    const T* src = F + blk * (long long)ns * kC2;
    for (int e = tid; e < ns * kC2; e += kWsThreads) ff[e] = src[e];
    __syncthreads();
    for (int e = tid; e < np * kC2; e += kWsThreads) {
      const int p = e / kC2, v = e % kC2;
      const int ij = a.pair_ij[p];
      const T prod = ff[(ij & 0xffff) * kC2 + v] * ff[(ij >> 16) * kC2 + v];
      if constexpr (F64) {
        reinterpret_cast<double*>(pbase)[p * kC2 + v] = prod;
      } else {
        __bf16* ph = reinterpret_cast<__bf16*>(pbase);
        __bf16* pl = ph + (size_t)(np + 1) * kQStride;
        const __bf16 h = (__bf16)prod;
        ph[p * kQStride + v] = h;
        pl[p * kQStride + v] = (__bf16)(prod - (float)h);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSlotTiles; ++k) {
      if (k >= nt) continue;
      if constexpr (F64) {
        const double* pp = reinterpret_cast<const double*>(pbase);
#pragma unroll
        for (int q = 0; q < kC2 / 4; ++q) {
          const int v = 4 * q + (lane >> 4);
          acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(pp[prow[k] * kC2 + v], pp[pcol[k] * kC2 + v], acc[k], 0, 0,
                                                        0);
        }
      } else {
        const __bf16* ph = reinterpret_cast<const __bf16*>(pbase);
        const __bf16* pl = ph + (size_t)(np + 1) * kQStride;
        const int o = 8 * (lane >> 4);
        const bf16x8 ahi = *reinterpret_cast<const bf16x8*>(ph + prow[k] * kQStride + o);
        const bf16x8 alo = *reinterpret_cast<const bf16x8*>(pl + prow[k] * kQStride + o);
        const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(ph + pcol[k] * kQStride + o);
        const bf16x8 blo = *reinterpret_cast<const bf16x8*>(pl + pcol[k] * kQStride + o);
        ws_mfma3(ahi, alo, bhi, blo, acc[k]);
      }
    }
    if (!F64 && ++chain == kFlushChunks) {
      // float32 chains into the float64 partials
#pragma unroll
      for (int k = 0; k < kSlotTiles; ++k) {
        if (k >= nt) continue;
        double* o = out + ((long long)wg * kTilesPerWg + w * kSlotTiles + k) * kMTileElems + lane;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          o[v * 64] = first ? (double)acc[k][v] : o[v * 64] + (double)acc[k][v];
          acc[k][v] = (A)0;
        }
      }
      chain = 0;
      first = false;
    }
  }
#pragma unroll
  for (int k = 0; k < kSlotTiles; ++k) {
    if (k >= nt) continue;
    double* o = out + ((long long)wg * kTilesPerWg + w * kSlotTiles + k) * kMTileElems;
    if constexpr (F64) {
      // (v, lane) is (row 4 v + lane / 16, column lane % 16): position
      // (lane / 16) * 64 + 16 v + lane % 16 in the split layout
#pragma unroll
      for (int v = 0; v < 4; ++v) o[(lane >> 4) * 64 + 16 * v + (lane & 15)] = (double)acc[k][v];
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        o[v * 64 + lane] = first ? (double)acc[k][v] : o[v * 64 + lane] + (double)acc[k][v];
    }
  }
}

// dst[i] = uniform in [-1, 1) from a 64-bit hash of (seed, i) (splitmix64 finaliser)
__global__ void k_fill_random(float* __restrict__ dst, long long n, unsigned long long seed) {
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ULL * (unsigned long long)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    dst[i] = (float)((double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0);
  }
}

// dst[0 .. n16) = 0 in 16-byte stores (grid-stride)
__global__ void k_zero16(uint4* __restrict__ dst, long long n16) {
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += step)
    dst[k] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

size_t adj_lds_bytes(int max_s) {
  return (size_t)(max_s + 1) * kAdjVox * sizeof(float) + 2 * (size_t)kAdjVox * kAdjSrow * sizeof(__bf16);
}

hipError_t prepare_adjoint_mfma() {
  return hipFuncSetAttribute((const void*)k_adjoint_mfma, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)adj_lds_bytes(kMaxSplitShells));
}

hipError_t launch_adj_weights(const double* gB, const double* norm, const int32_t* off, const int32_t* tri,
                              long long n_tiles, uint16_t* W, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  const long long n = n_tiles * 64;
  hipLaunchKernelGGL(k_adj_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gB, norm, off, tri, n_tiles,
                     W);
  return hipGetLastError();
}

hipError_t launch_adjoint_mfma(const float* F, float* G, const AdjGroup* groups_dev, int n_groups, int max_s,
                               int n_blocks, hipStream_t st) {
  if (n_groups < 1 || n_blocks < 1 || max_s > kMaxSplitShells) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adjoint_mfma, dim3((unsigned)n_blocks), dim3(kAdjWaves * 64), adj_lds_bytes(max_s), st, F, G,
                     groups_dev, n_groups);
  return hipGetLastError();
}

size_t quad4_lds_bytes(int n_pairs, int n_s, bool f64) {
  return f64 ? (size_t)(n_s + 1) * kC2 * 8 + (size_t)(n_pairs + 1) * kC2 * 8
             : (size_t)(n_s + 1) * kC2 * 4 + 2 * (size_t)(n_pairs + 1) * kQStride * 2;
}

hipError_t prepare_contract4() {
  hipError_t e = hipFuncSetAttribute((const void*)k_contract4<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)quad4_lds_bytes(kMaxQuadPairs, 128, false));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_contract4<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)quad4_lds_bytes(kMaxQuadPairs, 128, true));
}

hipError_t launch_contract4_bf16x3(const float* F, const Quad4Args& a, hipStream_t st) {
  if (a.n_pairs < 1 || a.n_pairs > kMaxQuadPairs || a.n_s > 128 || a.n_vox % kC2 || a.n_krange % 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_contract4<false>, dim3((unsigned)(a.n_wg * a.n_krange)), dim3(kWsThreads),
                     quad4_lds_bytes(a.n_pairs, a.n_s, false), st, (const void*)F, a);
  return hipGetLastError();
}

hipError_t launch_contract4_f64(const double* F, const Quad4Args& a, hipStream_t st) {
  if (a.n_pairs < 1 || a.n_pairs > kMaxQuadPairs || a.n_s > 128 || a.n_vox % kC2 || a.n_krange % 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_contract4<true>, dim3((unsigned)(a.n_wg * a.n_krange)), dim3(kWsThreads),
                     quad4_lds_bytes(a.n_pairs, a.n_s, true), st, (const void*)F, a);
  return hipGetLastError();
}

hipError_t launch_fill_random(float* dst, long long n, unsigned long long seed, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long want = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_random, dim3((unsigned)(want < 8192 ? want : 8192)), dim3(256), 0, st, dst, n, seed);
  return hipGetLastError();
}

hipError_t launch_zero(void* dst, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (bytes % 16 != 0 || ((uintptr_t)dst & 15) != 0) return hipErrorInvalidValue;
  const long long n16 = (long long)(bytes / 16);
  const long long want = (n16 + 255) / 256;
  const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(k_zero16, dim3(blocks), dim3(256), 0, st, reinterpret_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

size_t bf16x3_lds_bytes(int max_s, int rep) {
  const WsLayout y = ws_layout(max_s + 1, 2 * rep);
  return (size_t)y.bl0 + 2 * (size_t)rep * y.b_buf;
}

// Tiles per voxel range in the partials: every work group's kTilesPerWg, or for
// one work group the tiles of slots 0 .. top (its highest busy slot).
int ws_tile_stride(const MfmaTiling& mt) {
  if (mt.n_wg != 1) return mt.n_wg * kTilesPerWg;
  int top = 0;
  for (int k = 0; k < kSlotsPerWg && k < (int)mt.cols.size(); ++k)
    if (mt.cols[k].n > 0 && mt.cols[k].n_rb > 0) top = k;
  return (top + 1) * kSlotTiles;
}

// Replicas need one work group whose used slots all sit below 12 / rep (the
// slot placement fills SIMD 0..3 first, so few slots take the low positions),
// rep g16 staging waves' worth of rows (g16 = ceil(s_n / 16), one 8-voxel
// segment per thread) and their LDS; rep divides the 12 wavefronts.
int ws_max_rep(const MfmaTiling& mt) {
  if (mt.n_wg != 1 || mt.wg_rows.empty()) return 1;
  int top = -1;
  for (int k = 0; k < kSlotsPerWg && k < (int)mt.cols.size(); ++k)
    if (mt.cols[k].n > 0 && mt.cols[k].n_rb > 0) top = k;
  const int g16 = (mt.wg_rows[0].s_n + 15) / 16;
  for (int rep : {6, 4, 3, 2})
    if (top < kSlotsPerWg / rep && rep * g16 * 64 <= kWsThreads && bf16x3_lds_bytes(mt.max_s, rep) <= kWsLdsMax)
      return rep;
  return 1;
}

hipError_t launch_contract_fp32(const float* F, const ContractArgs& a, hipStream_t st) { return launch_vec<float>(F, a, st); }
hipError_t launch_contract_fp64(const double* F, const ContractArgs& a, hipStream_t st) { return launch_vec<double>(F, a, st); }

// Raises the vector kernels' dynamic LDS limit to what 256 shells need; done
// at plan time, before the first launch.
hipError_t prepare_contract_vec() {
  hipError_t e = hipFuncSetAttribute((const void*)k_contract_vec<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kVecLdsMax);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_contract_vec<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kVecLdsMax);
}

// Raises the kernel's dynamic LDS limit to what 128 staged shells need (the
// split-bf16 maximum); done at plan time so launches stay capture-safe.
hipError_t prepare_contract_bf16x3() {
  return hipFuncSetAttribute((const void*)k_contract_bf16x3, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kWsLdsMax);
}

bool ws_group_ok(const WsGroup& g) {
  // every staged row of every replica fits the per-thread loads (rows of a work
  // group <= max_s); ranges are whole voxel blocks; replicas need one work group
  return g.rep >= 1 && g.rep <= 6 && kSlotsPerWg % g.rep == 0 && (g.rep == 1 || g.n_wg == 1) &&
         (g.n_wg == 1 ? g.tile_stride >= kSlotTiles && g.tile_stride <= kTilesPerWg
                      : g.tile_stride == g.n_wg * kTilesPerWg) &&
         g.rep * 64 * ((g.max_s + 15) / 16) <= kWsThreads && g.max_s <= g.n_s && g.max_s <= kMaxSplitShells &&
         bf16x3_lds_bytes(g.max_s, g.rep) <= kWsLdsMax && g.n_vox % kC2 == 0 && g.n_krange % 8 == 0 &&
         g.block0 % 8 == 0 && g.n_wg >= 1;
}

hipError_t launch_contract_bf16x3(const float* F, double* partial, const WsGroup* groups_dev, int n_groups,
                                  size_t lds_bytes, int n_blocks, hipStream_t st) {
  if (n_groups < 1 || n_blocks < 1 || lds_bytes > kWsLdsMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_contract_bf16x3, dim3((unsigned)n_blocks), dim3(kWsThreads), lds_bytes, st, F, partial,
                     groups_dev, n_groups);
  return hipGetLastError();
}

hipError_t launch_gbuild(const float* F, const double* gB, const double* norm, const int4* terms, long long n_terms,
                        const int32_t* term_off, int n_s, long long n_vox, double* w, float* G, hipStream_t st) {
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

long long reduce_blocks(long long n_tri) { return (n_tri + kRedTri - 1) / kRedTri; }

hipError_t launch_reduce_grouped(const RedGroup* groups_dev, int n_groups, int n_blocks, double* B, hipStream_t st) {
  if (n_groups < 1 || n_blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_grouped, dim3((unsigned)n_blocks), dim3(kRedTri * kRedPart), 0, st, groups_dev, n_groups,
                     B);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int n_krange, long long stride, long long n_tri, const int32_t* slot,
                         const double* norm, const int32_t* out_idx, double* out, hipStream_t st, bool accumulate) {
  if (n_tri <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_tri + kRedTri - 1) / kRedTri);
  hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(kRedTri * kRedPart), 0, st, partial, n_krange, stride, n_tri, slot,
                     norm, out_idx, out, accumulate ? 1 : 0);
  return hipGetLastError();
}

}  // namespace bispec
