// FFT pass kernels of the estimator (steps a, b and b2), templated on the line
// length so every index computation is compile-time.  Instantiated for the
// supported grid sizes by fft_forward.hip, fft_inv_x.hip, fft_inv_y.hip and
// fft_c2r.hip.
//
// Two grids: the input grid N (delta and its half spectrum) and the estimator
// grid G <= N on which the shell fields live.  Every shell mode has
// |m_i| < G/2, so a mode sits at the same signed frequency on both grids, and
// the triple sums over G^3 points pick exactly the closed triangles when
// G > 3 max|m_i| (the aliasing argument of Section 2.2 applied to G).
//
// Layouts (all C order, z fastest):
//   delta  float32 [N][N][N]
//   spec   complex [N (kx)][N (ky)][spec_row(N) (kz)]        (half spectrum, in place;
//                                                             kz <= N/2 used)
//   A1_n   complex [G (x)][2R+1 (ky + R)][wrow (kz)]         (shell n after the x pass)
//   A2_n   complex [G (x)][G (y)][wrow (kz)]                 (shell n after the y pass)
//   F_n    real, voxel-blocked (vox_index) over G^3          (shell field)
// The kz rows are padded to 128 bytes (spec_row, shell_row = wrow >= R + 1),
// so strided tiles of whole 128-byte pieces read and write whole cache lines.
// R = rad[n] is the largest |m_y| of any mode of shell n, so the inverse
// passes of shell n only touch the ball |m| <= R: the x pass runs only the
// (ky, kz) columns inside the disc ky^2 + kz^2 < hi2[n], the y pass only the
// kz <= R planes, and the z pass reads R+1 of the G/2+1 half-spectrum planes.
//
// Strided passes stage a tile of TW consecutive kz columns times the whole
// line in LDS (interleaved layout); contiguous passes stage whole lines.
//
// Cohorts: every pass also runs several identical problems in one launch
// (realisations of one configuration): blockIdx.y is the member, whose input
// and output sit at blockIdx.y times the given element strides (0 and one
// member for a single problem).
#pragma once

#include "fft_core.h"
#include "kernels.h"

namespace bispec {
namespace fftk {

constexpr int kThrAxis = 512;  // threads of a strided-pass block
constexpr int kThrZ = 256;     // threads of a contiguous-pass block

// Forward strided passes (k_fft_axis): columns per block, and the dynamic LDS
// bytes of the sizes whose tile does not fit the 64 KB of static LDS.
__host__ __device__ constexpr int fwd_tile_cols(int n) { return n >= 128 ? 16 : fft_tile_cols(n, false); }
__host__ __device__ constexpr unsigned fwd_dyn_lds(int n) {
  return n >= 512 ? (unsigned)(n * fwd_tile_cols(n) + n) * 8u : 0u;
}

// Shell of block b from the per-shell block prefix sums off[0 .. n_shells]:
// every thread tests a few entries (one coalesced read instead of a chain of
// dependent reads in a binary search).  Uniform over the block; contains a
// barrier, so every thread of the block must call it.
__device__ __forceinline__ int block_shell(const long long* __restrict__ off, int n_shells, long long b) {
  __shared__ int s_shell;
  for (int t = threadIdx.x; t < n_shells; t += blockDim.x)
    if (off[t] <= b && b < off[t + 1]) s_shell = t;
  __syncthreads();
  return s_shell;
}

__device__ __forceinline__ int freq(int q, int n) { return q < n / 2 ? q : q - n; }

// the N-entry twiddle table into LDS (twiddle reads of every pass then stay on chip)
template <int N, int NT, typename T>
__device__ __forceinline__ void stage_twiddles(V2<T>* twl, const V2<T>* __restrict__ tw) {
  staged_copy<N, NT, V2<T>>([&](int e) { return tw[e]; }, [&](int e, V2<T> v) { twl[e] = v; });
}

// ---- (a) forward: real z lines -> half spectrum ------------------------------
// Two real samples per complex slot: z_m = x_{2m} + i x_{2m+1}, M-point FFT,
// then X_k = (Z_k + Z*_{M-k})/2 + W_N^k (Z_k - Z*_{M-k})/(2i), k = 0..M.
template <int N>
__global__ void __launch_bounds__(kThrZ) k_r2c_z(const float* __restrict__ in, float2* __restrict__ out,
                                                 const float2* __restrict__ tw, float scale, long long in_stride,
                                                 long long out_stride) {
  in += blockIdx.y * in_stride;
  out += blockIdx.y * out_stride;
  constexpr int M = N / 2;
  constexpr int NL = fft_z_lines(M, false);
  constexpr int LS = M + 1;
  __shared__ float2 buf[NL * LS];
  __shared__ float2 twl[N];
  const long long n_lines = (long long)N * N;
  const long long line0 = (long long)blockIdx.x * NL;
  const int lines = (int)min((long long)NL, n_lines - line0);
  const float2* src = reinterpret_cast<const float2*>(in) + line0 * M;
  staged_copy<NL * M, kThrZ, float2>(
      [&](int e) { return e / M < lines ? src[(long long)e] : mk<float>(0.f, 0.f); },
      [&](int e, float2 v) { buf[(e / M) * LS + e % M] = v; });
  stage_twiddles<N, kThrZ, float>(twl, tw);
  __syncthreads();
  ct_fft<float, M, NL, kThrZ, false, LS, 2>(buf, twl, -1.0f);
  constexpr long long P = spec_row(N);
  float2* dst = out + line0 * P;
  for (int e = threadIdx.x; e < NL * (M + 1); e += kThrZ) {
    const int c = e / (M + 1), k = e % (M + 1);
    if (c >= lines) continue;
    const float2 zk = buf[c * LS + (k == M ? 0 : k)];
    const float2 zc = conjv<float>(buf[c * LS + (k == 0 ? 0 : M - k)]);
    const float2 a = scl<float>(add<float>(zk, zc), 0.5f);
    const float2 d = scl<float>(sub<float>(zk, zc), 0.5f);  // (Z_k - Z*_{M-k}) / 2
    const float2 w = twl[k];
    const float2 bi = mk<float>(d.y, -d.x);                 // d / i
    dst[(long long)c * P + k] = scl<float>(add<float>(a, mul<float>(w, bi)), scale);
  }
}

// ---- (a) forward: strided complex axis, in place -----------------------------
// Lines along an axis of length N with element stride `stride`; n_cols
// consecutive columns; planes at outer_stride.  rsd_pass (the final x pass):
// multiply by 1 + beta kz^2/|m|^2.
// The tile takes fwd_tile_cols(N) columns: 16 for N >= 128 (128-byte row
// pieces; the half-spectrum rows are padded to spec_row(N), so every piece is
// one cache line), in dynamic LDS (fwd_dyn_lds(N) bytes, above the 64 KB of
// static LDS) for N >= 512.
template <int N>
__global__ void __launch_bounds__(kThrAxis) k_fft_axis(float2* __restrict__ data, long long stride, int n_cols,
                                                       long long outer_stride, const float2* __restrict__ tw,
                                                       float sign, float scale, int rsd_pass, float beta,
                                                       long long m_stride) {
  data += blockIdx.y * m_stride;
  constexpr int TW = fwd_tile_cols(N);
  constexpr bool kDyn = fwd_dyn_lds(N) > 0;
  __shared__ float2 sbuf[kDyn ? 1 : N * TW];
  __shared__ float2 stwl[kDyn ? 1 : N];
  extern __shared__ float2 dlds[];
  float2* buf = kDyn ? dlds : sbuf;
  float2* twl = kDyn ? dlds + N * TW : stwl;
  const int n_ct = (n_cols + TW - 1) / TW;
  const int o = blockIdx.x / n_ct;
  const int c0 = (blockIdx.x % n_ct) * TW;
  const int cols = min(TW, n_cols - c0);
  float2* base = data + (long long)o * outer_stride + c0;
  staged_copy<N * TW, kThrAxis, float2>(
      [&](int e) { return e % TW < cols ? base[(long long)(e / TW) * stride + e % TW] : mk<float>(0.f, 0.f); },
      [&](int e, float2 v) { buf[e] = v; });
  stage_twiddles<N, kThrAxis, float>(twl, tw);
  __syncthreads();
  ct_fft<float, N, TW, kThrAxis, true, 1, 1>(buf, twl, sign);
  for (int e = threadIdx.x; e < N * TW; e += kThrAxis) {
    const int q = e / TW, c = e % TW;
    if (c >= cols) continue;
    float f = scale;
    if (rsd_pass) {
      // data layout [kx][ky][kz]: this pass runs along kx (q), o = ky, column = kz
      const long long mx = freq(q, N), my = freq(o, N), mz = c0 + c;
      const long long m2 = mx * mx + my * my + mz * mz;
      if (m2 > 0) f *= 1.0f + beta * (float)((double)(mz * mz) / (double)m2);
    }
    base[(long long)q * stride + c] = scl<float>(buf[e], f);
  }
}

// ---- (b) inverse x pass of every shell ----------------------------------------
// Tile (shell, ky, kz0) of TW columns: Delta (or 1 for the unit shells) on the
// modes of shell n in those columns, inverse FFT along x, into A1_n.
template <typename T, bool UNIT, int N>
__global__ void __launch_bounds__(kThrAxis) k_inv_x(const float2* __restrict__ spec, int spec_n,
                                                    V2<T>* __restrict__ a1, const int4* __restrict__ tiles,
                                                    const ShellDev* __restrict__ sh, const V2<T>* __restrict__ tw,
                                                    long long spec_stride, long long a1_stride) {
  if (spec) spec += blockIdx.y * spec_stride;
  a1 += blockIdx.y * a1_stride;
  constexpr int TW = fft_tile_cols(N, sizeof(T) == 8);
  __shared__ V2<T> buf[N * TW];
  __shared__ V2<T> twl[N];
  const int4 td = tiles[blockIdx.x];
  const int sn = td.x, ky = td.y, kz0 = td.z;
  const ShellDev d = sh[sn];
  const int R = d.rad;
  const int cols = min(TW, R + 1 - kz0);
  const int yrow = ky < 0 ? ky + spec_n : ky;
  const long long ky2 = (long long)ky * ky;
  staged_copy<N * TW, kThrAxis, V2<T>>(
      [&](int e) {
        const int q = e / TW, c = e % TW;
        V2<T> v = mk<T>((T)0, (T)0);
        if (c < cols) {
          const long long mx = freq(q, N), kz = kz0 + c;
          const long long m2 = mx * mx + ky2 + kz * kz;
          if (m2 >= d.lo2 && m2 < d.hi2) {
            if (UNIT) {
              v = mk<T>((T)1, (T)0);
            } else {
              const long long xrow = mx < 0 ? mx + spec_n : mx;
              const float2 x = spec[(xrow * spec_n + yrow) * spec_row(spec_n) + kz];
              v = mk<T>((T)x.x, (T)x.y);
              if (d.ell) {  // Legendre weight L_ell(mu), mu^2 = m_z^2 / |m|^2 (line of sight z)
                const T u = (T)((double)(kz * kz) / (double)m2);
                const T wl = d.ell == 2 ? (T)1.5 * u - (T)0.5 : ((T)35 * u * u - (T)30 * u + (T)3) / (T)8;
                v = mk<T>(v.x * wl, v.y * wl);
              }
            }
          }
        }
        return v;
      },
      [&](int e, V2<T> v) { buf[e] = v; });
  stage_twiddles<N, kThrAxis, T>(twl, tw);
  __syncthreads();
  ct_fft<T, N, TW, kThrAxis, true, 1, 1>(buf, twl, (T)1);
  V2<T>* dst = a1 + d.a1_off;
  const int wy = 2 * R + 1, wz = d.wrow;  // row stride (padded)
  for (int e = threadIdx.x; e < N * TW; e += kThrAxis) {
    const int q = e / TW, c = e % TW;
    if (c < cols) dst[((long long)q * wy + (ky + R)) * wz + kz0 + c] = buf[e];
  }
}

// ---- (b) inverse y pass of every shell ----------------------------------------
// Block -> (shell, x, kz tile) through the per-shell prefix sums tile_off, for
// the planes x0 + x < x_end of a slab (x local to the slab: A2 holds the
// slab's planes; blocks beyond x_end, in a slab shorter than the tables', do
// nothing).
template <typename T, int N>
__global__ void __launch_bounds__(kThrAxis) k_inv_y(const V2<T>* __restrict__ a1, V2<T>* __restrict__ a2,
                                                    const long long* __restrict__ tile_off, int n_shells,
                                                    const ShellDev* __restrict__ sh, const V2<T>* __restrict__ tw,
                                                    int x0, int x_end, long long a1_stride, long long a2_stride) {
  a1 += blockIdx.y * a1_stride;
  a2 += blockIdx.y * a2_stride;
  constexpr int TW = fft_tile_cols(N, sizeof(T) == 8);
  __shared__ V2<T> buf[N * TW];
  __shared__ V2<T> twl[N];
  const long long b = blockIdx.x;
  const int sn = block_shell(tile_off, n_shells, b);  // tile_off[sn] <= b < tile_off[sn + 1]
  const ShellDev d = sh[sn];
  const int R = d.rad;
  const int n_ct = (R + 1 + TW - 1) / TW;
  const long long local = b - tile_off[sn];
  const int x = (int)(local / n_ct);
  if (x0 + x >= x_end) return;  // uniform over the block, before any barrier
  const int kz0 = (int)(local % n_ct) * TW;
  const int cols = min(TW, R + 1 - kz0);
  const int wy = 2 * R + 1, wz = d.wrow;  // row stride (padded)
  const V2<T>* src = a1 + d.a1_off + (long long)(x0 + x) * wy * wz;
  staged_copy<N * TW, kThrAxis, V2<T>>(
      [&](int e) {
        const int q = e / TW, c = e % TW;
        V2<T> v = mk<T>((T)0, (T)0);
        if (c < cols) {
          const long long my = freq(q, N), kz = kz0 + c;
          if (my >= -R && my <= R && my * my + kz * kz < d.hi2) v = src[(my + R) * wz + kz];
        }
        return v;
      },
      [&](int e, V2<T> v) { buf[e] = v; });
  stage_twiddles<N, kThrAxis, T>(twl, tw);
  __syncthreads();
  ct_fft<T, N, TW, kThrAxis, true, 1, 1>(buf, twl, (T)1);
  V2<T>* dst = a2 + d.a2_off + (long long)x * N * wz;
  for (int e = threadIdx.x; e < N * TW; e += kThrAxis) {
    const int q = e / TW, c = e % TW;
    if (c < cols) dst[(long long)q * wz + kz0 + c] = buf[e];
  }
}

// ---- (b) inverse z pass (C2R) of every shell -----------------------------------
// Per (x, y) line: X_k (k = 0..M, zero beyond R), Z'_k = (X_k + X*_{M-k})
// + i W_N^{-k} (X_k - X*_{M-k}) for k < M, M-point inverse FFT; the
// unnormalised real line is (Re z_m, Im z_m) at (2m, 2m+1), written
// voxel-blocked.  Every shell has n_lines lines (N^2, or the lines of an
// x-slab: its voxels are then numbered from the slab's first), hence the same
// number of blocks (blk_off[sn] = sn * blocks per shell; the table is not
// read).
template <typename T, typename OutT, int N>
__global__ void __launch_bounds__(kThrZ) k_c2r_z(const V2<T>* __restrict__ a2, OutT* __restrict__ out,
                                                 const long long* __restrict__ blk_off, int n_shells,
                                                 const ShellDev* __restrict__ sh, const V2<T>* __restrict__ tw,
                                                 long long n_lines, long long a2_stride, long long out_stride) {
  a2 += blockIdx.y * a2_stride;
  out += blockIdx.y * out_stride;
  constexpr int M = N / 2;
  constexpr int NL = fft_z_lines(M, sizeof(T) == 8);
  constexpr int LS = M + 1;
  __shared__ V2<T> buf[NL * LS];
  __shared__ V2<T> twl[N];
  // every shell has the same n_lines lines, so the same number of blocks;
  // the shell runs fastest, so blocks in flight together write neighbouring
  // 128-byte pieces of the same voxel blocks (DRAM pages) instead of one
  // piece per 12.8 KB of the field
  const long long b = blockIdx.x;
  const int sn = (int)(b % n_shells);
  const ShellDev d = sh[sn];
  const int wz = d.rad + 1, ws = d.wrow;  // used kz columns, row stride
  const long long line0 = (b / n_shells) * NL;
  const int lines = (int)min((long long)NL, n_lines - line0);
  const V2<T>* src = a2 + d.a2_off + line0 * ws;
  staged_copy<NL * LS, kThrZ, V2<T>>(
      [&](int e) {
        const int c = e / LS, k = e % LS;
        return (c < lines && k < wz) ? src[(long long)c * ws + k] : mk<T>((T)0, (T)0);
      },
      [&](int e, V2<T> v) { buf[e] = v; });
  stage_twiddles<N, kThrZ, T>(twl, tw);
  __syncthreads();
  // pairs (k, M-k), k = 0..M/2, one thread each, in place
  constexpr int HALF = M / 2 + 1;
  for (int e = threadIdx.x; e < NL * HALF; e += kThrZ) {
    const int c = e / HALF, k = e % HALF;
    V2<T>* L = buf + c * LS;
    const V2<T> xk = L[k], xmk = L[M - k];
    const V2<T> sp = add<T>(xk, conjv<T>(xmk));
    const V2<T> t = mul<T>(conjv<T>(twl[k]), sub<T>(xk, conjv<T>(xmk)));
    if (k > 0 && k < M - k) {
      const V2<T> sp2 = add<T>(xmk, conjv<T>(xk));
      const V2<T> t2 = mul<T>(conjv<T>(twl[M - k]), sub<T>(xmk, conjv<T>(xk)));
      L[M - k] = mk<T>(sp2.x - t2.y, sp2.y + t2.x);
    }
    if (k < M) L[k] = mk<T>(sp.x - t.y, sp.y + t.x);
  }
  __syncthreads();
  ct_fft<T, M, NL, kThrZ, false, LS, 2>(buf, twl, (T)1);
  for (int e = threadIdx.x; e < NL * M; e += kThrZ) {
    const int c = e / M, q = e % M;
    if (c >= lines) continue;
    const V2<T> z = buf[c * LS + q];
    const OutT x0 = (OutT)z.x, x1 = (OutT)z.y;
    const long long at = vox_index((line0 + c) * N + 2 * q, sn, n_shells);  // even: pair stays in one block
    *reinterpret_cast<V2<OutT>*>(out + at) = mk<OutT>(x0, x1);
  }
}

}  // namespace fftk
}  // namespace bispec

// X-macro over the supported grid sizes N = 2^a * {1, 3, 5}, 8 <= N <= 1024.
#define BISPEC_FOR_EACH_N(X) \
  X(8) X(16) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512) X(640) \
  X(768) X(1024)

// ============================================================================
// Adjoint passes (gradient of sum_t gB_t B_t): the forward transform of every
// G_n, pruned to the modes of shell n, scattered into one half spectrum S.
// They mirror the inverse passes: z (R2C, keep kz <= R) -> A2_n, y (keep
// |ky| <= R) -> A1_n, x (keep the modes of shell n) -> S.
// ============================================================================
namespace bispec {
namespace fftk {

// z: G_n line (x, y) (voxel-blocked) -> A2_n[x][y][0..R] (forward R2C, unnormalised)
template <int N>
__global__ void __launch_bounds__(kThrZ) k_g_r2c_z(const float* __restrict__ G, float2* __restrict__ a2,
                                                   const long long* __restrict__ blk_off, int n_shells,
                                                   const ShellDev* __restrict__ sh, const float2* __restrict__ tw) {
  constexpr int M = N / 2;
  constexpr int NL = fft_z_lines(M, false);
  constexpr int LS = M + 1;
  __shared__ float2 buf[NL * LS];
  __shared__ float2 twl[N];
  // every shell has the same N^2 lines, so the same number of blocks
  const long long n_lines = (long long)N * N;
  constexpr long long kBps = ((long long)N * N + NL - 1) / NL;
  const long long b = blockIdx.x;
  const int sn = (int)(b / kBps);
  const ShellDev d = sh[sn];
  const int wz = d.rad + 1, ws = d.wrow;  // used kz columns, row stride
  const long long line0 = (b - sn * kBps) * NL;
  const int lines = (int)min((long long)NL, n_lines - line0);
  staged_copy<NL * M, kThrZ, float2>(
      [&](int e) {
        const int c = e / M, q = e % M;
        if (c >= lines) return mk<float>(0.f, 0.f);
        const long long at = vox_index((line0 + c) * N + 2 * q, sn, n_shells);
        return *reinterpret_cast<const float2*>(G + at);
      },
      [&](int e, float2 v) { buf[(e / M) * LS + e % M] = v; });
  stage_twiddles<N, kThrZ, float>(twl, tw);
  __syncthreads();
  ct_fft<float, M, NL, kThrZ, false, LS, 2>(buf, twl, -1.0f);
  float2* dst = a2 + d.a2_off + line0 * ws;
  for (int e = threadIdx.x; e < NL * wz; e += kThrZ) {
    const int c = e / wz, k = e % wz;
    if (c >= lines) continue;
    const float2 zk = buf[c * LS + (k == M ? 0 : k)];
    const float2 zc = conjv<float>(buf[c * LS + (k == 0 ? 0 : M - k)]);
    const float2 a = scl<float>(add<float>(zk, zc), 0.5f);
    const float2 dd = scl<float>(sub<float>(zk, zc), 0.5f);
    const float2 bi = mk<float>(dd.y, -dd.x);
    dst[(long long)c * ws + k] = add<float>(a, mul<float>(twl[k], bi));
  }
}

// y: A2_n[x][.][kz] (kz <= R) -> forward FFT along y -> A1_n[x][ky + R][kz], |ky| <= R
template <int N>
__global__ void __launch_bounds__(kThrAxis) k_g_fwd_y(const float2* __restrict__ a2, float2* __restrict__ a1,
                                                      const long long* __restrict__ tile_off, int n_shells,
                                                      const ShellDev* __restrict__ sh,
                                                      const float2* __restrict__ tw) {
  constexpr int TW = fft_tile_cols(N, false);
  __shared__ float2 buf[N * TW];
  __shared__ float2 twl[N];
  const long long b = blockIdx.x;
  const int sn = block_shell(tile_off, n_shells, b);  // tile_off[sn] <= b < tile_off[sn + 1]
  const ShellDev d = sh[sn];
  const int R = d.rad;
  const int n_ct = (R + 1 + TW - 1) / TW;
  const long long local = b - tile_off[sn];
  const int x = (int)(local / n_ct);
  const int kz0 = (int)(local % n_ct) * TW;
  const int cols = min(TW, R + 1 - kz0);
  const int wy = 2 * R + 1, wz = d.wrow;  // row stride (padded)
  const float2* src = a2 + d.a2_off + (long long)x * N * wz;
  staged_copy<N * TW, kThrAxis, float2>(
      [&](int e) { return e % TW < cols ? src[(long long)(e / TW) * wz + kz0 + e % TW] : mk<float>(0.f, 0.f); },
      [&](int e, float2 v) { buf[e] = v; });
  stage_twiddles<N, kThrAxis, float>(twl, tw);
  __syncthreads();
  ct_fft<float, N, TW, kThrAxis, true, 1, 1>(buf, twl, -1.0f);
  float2* dst = a1 + d.a1_off + (long long)x * wy * wz;
  for (int e = threadIdx.x; e < wy * TW; e += kThrAxis) {
    const int ky = e / TW - R, c = e % TW;
    if (c < cols) dst[(long long)(ky + R) * wz + kz0 + c] = buf[(ky < 0 ? ky + N : ky) * TW + c];
  }
}

// x: tile (shell, ky, kz0): A1_n[.][ky + R][kz] -> forward FFT along x -> for the
// modes of shell n: S[kx][ky][kz] += scale * Z(k) * value (the shells of one
// launch are disjoint; launches of several grids add into the same modes);
// S is the half spectrum of the spec_n grid
template <int N>
__global__ void __launch_bounds__(kThrAxis) k_g_fwd_x(const float2* __restrict__ a1, float2* __restrict__ S,
                                                      int spec_n, const int4* __restrict__ tiles,
                                                      const ShellDev* __restrict__ sh,
                                                      const float2* __restrict__ tw, float scale, float beta) {
  constexpr int TW = fft_tile_cols(N, false);
  __shared__ float2 buf[N * TW];
  __shared__ float2 twl[N];
  const int4 td = tiles[blockIdx.x];
  const int sn = td.x, ky = td.y, kz0 = td.z;
  const ShellDev d = sh[sn];
  const int R = d.rad;
  const int cols = min(TW, R + 1 - kz0);
  const int wy = 2 * R + 1, wz = d.wrow;  // row stride (padded)
  const float2* src = a1 + d.a1_off;
  staged_copy<N * TW, kThrAxis, float2>(
      [&](int e) {
        return e % TW < cols ? src[((long long)(e / TW) * wy + (ky + R)) * wz + kz0 + e % TW] : mk<float>(0.f, 0.f);
      },
      [&](int e, float2 v) { buf[e] = v; });
  stage_twiddles<N, kThrAxis, float>(twl, tw);
  __syncthreads();
  ct_fft<float, N, TW, kThrAxis, true, 1, 1>(buf, twl, -1.0f);
  const int yrow = ky < 0 ? ky + spec_n : ky;
  const long long ky2 = (long long)ky * ky;
  for (int e = threadIdx.x; e < N * TW; e += kThrAxis) {
    const int q = e / TW, c = e % TW;
    if (c >= cols) continue;
    const long long mx = freq(q, N), kz = kz0 + c;
    const long long m2 = mx * mx + ky2 + kz * kz;
    if (m2 < d.lo2 || m2 >= d.hi2) continue;
    const float z = 1.0f + beta * (float)((double)(kz * kz) / (double)m2);
    const long long xrow = mx < 0 ? mx + spec_n : mx;
    float2& o = S[(xrow * spec_n + yrow) * spec_row(spec_n) + kz];
    o = add<float>(o, scl<float>(buf[e], scale * z));
  }
}

}  // namespace fftk
}  // namespace bispec
