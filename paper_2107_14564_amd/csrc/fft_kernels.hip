// FFT passes of the estimator (steps a and b/b2), hand-written for gfx950.
//
// Grid layout (all C order, z fastest):
//   delta  float32 [N][N][N]
//   spec   complex [N (kx)][N (ky)][M+1 (kz)], M = N/2     (half spectrum, in place)
//   A1_n   complex [N (x)][2R+1 (ky + R)][R+1 (kz)]        (shell n after the x pass)
//   A2_n   complex [N (x)][N (y)][R+1 (kz)]                (shell n after the y pass)
//   F_n    real    [N][N][N]                               (shell field)
// R = rad[n] is the largest |m_y| of any mode of shell n, so the inverse
// passes of shell n only touch the ball |m| <= R: the x pass runs only the
// (ky, kz) columns inside the disc ky^2 + kz^2 < hi2[n], the y pass only the
// kz <= R planes, and the z pass reads R+1 of the M+1 half-spectrum planes.
//
// Strided passes stage a tile of TW consecutive kz columns times the whole
// line in LDS (TW * 8 B or TW * 16 B contiguous per row), contiguous passes
// stage whole lines.  All lines of one work group are transformed together by
// lds_fft.
#include "fft_core.h"
#include "kernels.h"

namespace bispec {

namespace {

template <typename T> struct FftCfg;
template <> struct FftCfg<float> { static constexpr int E = kFftElemsF32; };
template <> struct FftCfg<double> { static constexpr int E = kFftElemsF64; };
constexpr int NT = kFftThreads;

__device__ __forceinline__ int freq(int q, int n) { return q < n / 2 ? q : q - n; }

// ---- (a) forward: real z lines -> half spectrum --------------------------------

// Two real samples per complex slot: z_m = x_{2m} + i x_{2m+1}, M-point FFT,
// then X_k = (Z_k + Z*_{M-k})/2 + W_N^k (Z_k - Z*_{M-k})/(2i), k = 0..M.
__global__ void __launch_bounds__(NT) k_r2c_z(const float* __restrict__ in, float2* __restrict__ out, int n,
                                              long long n_lines, FftSched s, const float2* __restrict__ tw,
                                              float scale) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* buf = reinterpret_cast<float2*>(smem_raw);
  const int m = n / 2;
  const int nl = fft_tile_lines(m, false);
  const int ls = m + 1;  // one padding slot per line
  const long long line0 = (long long)blockIdx.x * nl;
  const int lines = (int)min((long long)nl, n_lines - line0);
  const float2* src = reinterpret_cast<const float2*>(in) + line0 * m;
  for (int e = threadIdx.x; e < lines * m; e += NT) {
    const int c = e / m, q = e % m;
    buf[c * ls + q] = src[(long long)c * m + q];
  }
  __syncthreads();
  lds_fft<float, FftCfg<float>::E, NT>(buf, s, lines, 1, ls, false, tw, -1.0f);
  float2* dst = out + line0 * (m + 1);
  for (int e = threadIdx.x; e < lines * (m + 1); e += NT) {
    const int c = e / (m + 1), k = e % (m + 1);
    const float2 zk = buf[c * ls + (k == m ? 0 : k)];
    const float2 zc = conjv<float>(buf[c * ls + (k == 0 ? 0 : m - k)]);
    const float2 a = scl<float>(add<float>(zk, zc), 0.5f);
    const float2 d = scl<float>(sub<float>(zk, zc), 0.5f);  // (Zk - Z*_{M-k}) / 2
    // W^k d / i = W^k * (-i d)
    const float2 w = tw[k];
    const float2 bi = mk<float>(d.y, -d.x);
    const float2 x = add<float>(a, mul<float>(w, bi));
    dst[(long long)c * (m + 1) + k] = scl<float>(x, scale);
  }
}

// ---- (a) forward: strided complex axis, in place -------------------------------
// Lines along an axis of length n with element stride `stride`; columns are
// n_cols consecutive elements; `outer` independent planes at outer_stride.
// With rsd != 0 (final x pass): multiply by 1 + beta kz^2/|m|^2.
__global__ void __launch_bounds__(NT) k_fft_axis(float2* __restrict__ data, FftSched s, long long stride,
                                                 int n_cols, long long outer_stride, const float2* __restrict__ tw,
                                                 float sign, float scale, int rsd_pass, float beta) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* buf = reinterpret_cast<float2*>(smem_raw);
  const int n = s.n;
  const int tw_cols = fft_tile_cols(n, false);  // tile width
  const int n_ct = (n_cols + tw_cols - 1) / tw_cols;
  const int o = blockIdx.x / n_ct;
  const int c0 = (blockIdx.x % n_ct) * tw_cols;
  const int cols = min(tw_cols, n_cols - c0);
  float2* base = data + (long long)o * outer_stride + c0;
  for (int e = threadIdx.x; e < n * tw_cols; e += NT) {
    const int q = e / tw_cols, c = e % tw_cols;
    if (c < cols) buf[q * tw_cols + c] = base[(long long)q * stride + c];
  }
  __syncthreads();
  lds_fft<float, FftCfg<float>::E, NT>(buf, s, tw_cols, tw_cols, 1, true, tw, sign);
  for (int e = threadIdx.x; e < n * tw_cols; e += NT) {
    const int q = e / tw_cols, c = e % tw_cols;
    if (c >= cols) continue;
    float f = scale;
    if (rsd_pass) {
      // data layout [kx][ky][kz]: this pass runs along kx (q), o = ky, column = kz
      const long long mx = freq(q, n), my = freq(o, n), mz = c0 + c;
      const long long m2 = mx * mx + my * my + mz * mz;
      if (m2 > 0) f *= 1.0f + beta * (float)((double)(mz * mz) / (double)m2);
    }
    base[(long long)q * stride + c] = scl<float>(buf[q * tw_cols + c], f);
  }
}

// ---- (b) inverse x pass of every shell -------------------------------------------
// Tile (shell, ky, kz0) of TW columns.  Loads Delta (or 1 for the unit shells)
// of the modes of shell n in those columns, inverse FFT along x, writes A1_n.
template <typename T, bool UNIT>
__global__ void __launch_bounds__(NT) k_inv_x(const float2* __restrict__ spec, V2<T>* __restrict__ a1,
                                              const int4* __restrict__ tiles, const ShellDev* __restrict__ sh,
                                              FftSched s, int m, const V2<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
  const int n = s.n;
  const int tw_cols = fft_tile_cols(n, sizeof(T) == 8);
  const int4 td = tiles[blockIdx.x];
  const int sn = td.x, ky = td.y, kz0 = td.z;
  const ShellDev d = sh[sn];
  const int R = d.rad;
  const int cols = min(tw_cols, R + 1 - kz0);
  const int yrow = ky < 0 ? ky + n : ky;
  for (int e = threadIdx.x; e < n * tw_cols; e += NT) {
    const int q = e / tw_cols, c = e % tw_cols;
    V2<T> v = mk<T>((T)0, (T)0);
    if (c < cols) {
      const long long mx = freq(q, n), kz = kz0 + c;
      const long long m2 = mx * mx + (long long)ky * ky + kz * kz;
      if (m2 >= d.lo2 && m2 < d.hi2) {
        if (UNIT) {
          v = mk<T>((T)1, (T)0);
        } else {
          const float2 x = spec[((long long)q * n + yrow) * (m + 1) + kz];
          v = mk<T>((T)x.x, (T)x.y);
        }
      }
    }
    buf[q * tw_cols + c] = v;
  }
  __syncthreads();
  lds_fft<T, FftCfg<T>::E, NT>(buf, s, tw_cols, tw_cols, 1, true, tw, (T)1);
  V2<T>* dst = a1 + d.a1_off;
  const int wy = 2 * R + 1, wz = R + 1;
  for (int e = threadIdx.x; e < n * tw_cols; e += NT) {
    const int q = e / tw_cols, c = e % tw_cols;
    if (c < cols) dst[((long long)q * wy + (ky + R)) * wz + kz0 + c] = buf[q * tw_cols + c];
  }
}

// ---- (b) inverse y pass of every shell -------------------------------------------
// Block -> (shell, x, kz tile) through the per-shell prefix sums tile_off.
template <typename T>
__global__ void __launch_bounds__(NT) k_inv_y(const V2<T>* __restrict__ a1, V2<T>* __restrict__ a2,
                                              const long long* __restrict__ tile_off, int n_shells,
                                              const ShellDev* __restrict__ sh, FftSched s,
                                              const V2<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
  const int n = s.n;
  const int tw_cols = fft_tile_cols(n, sizeof(T) == 8);
  const long long b = blockIdx.x;
  int lo = 0, hi = n_shells;  // find sn with tile_off[sn] <= b < tile_off[sn+1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (tile_off[mid] <= b) lo = mid; else hi = mid;
  }
  const int sn = lo;
  const ShellDev d = sh[sn];
  const int R = d.rad;
  const int n_ct = (R + 1 + tw_cols - 1) / tw_cols;
  const long long local = b - tile_off[sn];
  const int x = (int)(local / n_ct);
  const int kz0 = (int)(local % n_ct) * tw_cols;
  const int cols = min(tw_cols, R + 1 - kz0);
  const int wy = 2 * R + 1, wz = R + 1;
  const V2<T>* src = a1 + d.a1_off + (long long)x * wy * wz;
  for (int e = threadIdx.x; e < n * tw_cols; e += NT) {
    const int q = e / tw_cols, c = e % tw_cols;
    V2<T> v = mk<T>((T)0, (T)0);
    if (c < cols) {
      const long long my = freq(q, n), kz = kz0 + c;
      if (my * my + kz * kz < d.hi2 && my >= -R && my <= R) v = src[(my + R) * wz + kz];
    }
    buf[q * tw_cols + c] = v;
  }
  __syncthreads();
  lds_fft<T, FftCfg<T>::E, NT>(buf, s, tw_cols, tw_cols, 1, true, tw, (T)1);
  V2<T>* dst = a2 + d.a2_off + (long long)x * n * wz;
  for (int e = threadIdx.x; e < n * tw_cols; e += NT) {
    const int q = e / tw_cols, c = e % tw_cols;
    if (c < cols) dst[(long long)q * wz + kz0 + c] = buf[q * tw_cols + c];
  }
}

// ---- (b) inverse z pass (C2R) of every shell --------------------------------------
// For each (x, y) line: X_k (k = 0..M, zero beyond R), Z'_k = (X_k + X*_{M-k})
// + i W_N^{-k} (X_k - X*_{M-k}) for k < M, M-point inverse FFT, and the
// unnormalised real line is (Re z_m, Im z_m) at (2m, 2m+1).
template <typename T, typename OutT>
__global__ void __launch_bounds__(NT) k_c2r_z(const V2<T>* __restrict__ a2, OutT* __restrict__ out,
                                              long long field_stride, const long long* __restrict__ blk_off,
                                              int n_shells, const ShellDev* __restrict__ sh, FftSched s, int n,
                                              const V2<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
  const int m = n / 2;
  const int nl = fft_tile_lines(m, sizeof(T) == 8);
  const int ls = m + 1;
  const long long b = blockIdx.x;
  int lo = 0, hi = n_shells;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (blk_off[mid] <= b) lo = mid; else hi = mid;
  }
  const int sn = lo;
  const ShellDev d = sh[sn];
  const int R = d.rad;
  const int wz = R + 1;
  const long long n_lines = (long long)n * n;
  const long long line0 = (b - blk_off[sn]) * nl;
  const int lines = (int)min((long long)nl, n_lines - line0);
  const V2<T>* src = a2 + d.a2_off + line0 * wz;
  for (int e = threadIdx.x; e < lines * ls; e += NT) {
    const int c = e / ls, k = e % ls;
    buf[c * ls + k] = k < wz ? src[(long long)c * wz + k] : mk<T>((T)0, (T)0);
  }
  __syncthreads();
  // pairs (k, M-k), k = 0..M/2, handled by one thread each: in place
  const int half = m / 2 + 1;
  for (int e = threadIdx.x; e < lines * half; e += NT) {
    const int c = e / half, k = e % half;
    V2<T>* L = buf + c * ls;
    const V2<T> xk = L[k], xmk = L[m - k];
    // Z'_k from X_k, X_{M-k}
    {
      const V2<T> sp = add<T>(xk, conjv<T>(xmk));
      const V2<T> df = sub<T>(xk, conjv<T>(xmk));
      const V2<T> wc = conjv<T>(tw[k]);          // W_N^{-k}
      const V2<T> t = mul<T>(wc, df);
      const V2<T> zk = mk<T>(sp.x - t.y, sp.y + t.x);  // sp + i t
      if (k > 0 && k < m - k) {
        const int k2 = m - k;  // Z'_{M-k} from X_{M-k}, X_k
        const V2<T> sp2 = add<T>(xmk, conjv<T>(xk));
        const V2<T> df2 = sub<T>(xmk, conjv<T>(xk));
        const V2<T> t2 = mul<T>(conjv<T>(tw[k2]), df2);
        L[k2] = mk<T>(sp2.x - t2.y, sp2.y + t2.x);
      }
      if (k < m) L[k] = zk;
    }
  }
  __syncthreads();
  lds_fft<T, FftCfg<T>::E, NT>(buf, s, lines, 1, ls, false, tw, (T)1);
  // (x_{2q}, x_{2q+1}) = (Re z_q, Im z_q): one paired store per output slot
  V2<OutT>* dst = reinterpret_cast<V2<OutT>*>(out + (long long)sn * field_stride + line0 * n);
  for (int e = threadIdx.x; e < lines * m; e += NT) {
    const int c = e / m, q = e % m;
    const V2<T> z = buf[c * ls + q];
    dst[(long long)c * m + q] = mk<OutT>((OutT)z.x, (OutT)z.y);
  }
}

FftSched sched(int n, int tw_stride) {
  FftSched s{};
  s.n = n;
  std::vector<int> r = fft_radices(n);
  s.npass = (int)r.size();
  for (int p = 0; p < s.npass; ++p) s.r[p] = r[p];
  s.tw_stride = tw_stride;
  return s;
}

}  // namespace

void plan_shell_passes(const ShellGeometry& g, bool f64, ShellPassPlan& p) {
  const int n = g.n_g;
  const int twc = fft_tile_cols(n, f64);
  const int nl = fft_tile_lines(n / 2, f64);
  p.shells.resize(g.n_s);
  p.x_tiles.clear();
  p.y_off.assign(1, 0);
  p.z_off.assign(1, 0);
  long long a1 = 0, a2 = 0;
  for (int sn = 0; sn < g.n_s; ++sn) {
    ShellDev& d = p.shells[sn];
    d.lo2 = g.lo2[sn];
    d.hi2 = g.hi2[sn];
    d.rad = g.rad[sn];
    d.pad = 0;
    const long long R = d.rad;
    d.a1_off = a1;
    d.a2_off = a2;
    a1 += (long long)n * (2 * R + 1) * (R + 1);
    a2 += (long long)n * n * (R + 1);
    for (long long ky = -R; ky <= R; ++ky)
      for (long long kz0 = 0; kz0 <= R; kz0 += twc)
        if (ky * ky + kz0 * kz0 < d.hi2) p.x_tiles.push_back(make_int4(sn, (int)ky, (int)kz0, 0));
    const long long n_ct = (R + 1 + twc - 1) / twc;
    p.y_off.push_back(p.y_off.back() + (long long)n * n_ct);
    p.z_off.push_back(p.z_off.back() + ((long long)n * n + nl - 1) / nl);
  }
  p.a1_elems = a1;
  p.a2_elems = a2;
}

hipError_t launch_forward(const float* delta, float2* spec, int n, float beta, const float2* tw, hipStream_t st) {
  const int m = n / 2;
  const float axis_scale = 1.0f / sqrtf((float)n);  // unitary overall: N^{-3/2}
  // z: real -> half spectrum
  {
    const int nl = fft_tile_lines(m, false);
    const long long n_lines = (long long)n * n;
    const unsigned blocks = (unsigned)((n_lines + nl - 1) / nl);
    const size_t lds = (size_t)nl * (m + 1) * sizeof(float2);
    hipLaunchKernelGGL(k_r2c_z, dim3(blocks), dim3(NT), lds, st, delta, spec, n, n_lines, sched(m, 2), tw, axis_scale);
  }
  const int twc = fft_tile_cols(n, false);
  const int n_ct = (m + 1 + twc - 1) / twc;
  const size_t lds = (size_t)n * twc * sizeof(float2);
  // y: lines [x][.][kz], stride M+1, outer x
  hipLaunchKernelGGL(k_fft_axis, dim3(n * n_ct), dim3(NT), lds, st, spec, sched(n, 1), (long long)(m + 1), m + 1,
                     (long long)n * (m + 1), tw, -1.0f, axis_scale, 0, 0.0f);
  // x: lines [.][ky][kz], stride N(M+1), outer ky; RSD factor applied here
  hipLaunchKernelGGL(k_fft_axis, dim3(n * n_ct), dim3(NT), lds, st, spec, sched(n, 1), (long long)n * (m + 1), m + 1,
                     (long long)(m + 1), tw, -1.0f, axis_scale, beta != 0.0f ? 1 : 0, beta);
  return hipGetLastError();
}

template <typename T, bool UNIT, typename OutT>
static hipError_t launch_shells_impl(const float2* spec, V2<T>* a1, V2<T>* a2, OutT* out, long long field_stride,
                                     const ShellLaunch& L, int n, const V2<T>* tw, hipStream_t st) {
  const bool f64 = sizeof(T) == 8;
  const int twc = fft_tile_cols(n, f64);
  const size_t lds_axis = (size_t)n * twc * sizeof(V2<T>);
  if (L.n_x_tiles > 0)
    hipLaunchKernelGGL((k_inv_x<T, UNIT>), dim3((unsigned)L.n_x_tiles), dim3(NT), lds_axis, st, spec, a1, L.x_tiles,
                       L.shells, sched(n, 1), n / 2, tw);
  if (L.n_y_blocks > 0)
    hipLaunchKernelGGL((k_inv_y<T>), dim3((unsigned)L.n_y_blocks), dim3(NT), lds_axis, st, a1, a2, L.y_off, L.n_shells,
                       L.shells, sched(n, 1), tw);
  const int m = n / 2;
  const int nl = fft_tile_lines(m, f64);
  const size_t lds_z = (size_t)nl * (m + 1) * sizeof(V2<T>);
  if (L.n_z_blocks > 0)
    hipLaunchKernelGGL((k_c2r_z<T, OutT>), dim3((unsigned)L.n_z_blocks), dim3(NT), lds_z, st, a2, out, field_stride,
                       L.z_off, L.n_shells, L.shells, sched(m, 2), n, tw);
  return hipGetLastError();
}

hipError_t launch_data_shells(const float2* spec, float2* a1, float2* a2, float* F, long long field_stride,
                              const ShellLaunch& L, int n, const float2* tw, hipStream_t st) {
  return launch_shells_impl<float, false, float>(spec, a1, a2, F, field_stride, L, n, tw, st);
}

hipError_t launch_unit_shells(double2* a1, double2* a2, double* I, long long field_stride, const ShellLaunch& L, int n,
                              const double2* tw, hipStream_t st) {
  return launch_shells_impl<double, true, double>(nullptr, a1, a2, I, field_stride, L, n, tw, st);
}

}  // namespace bispec
