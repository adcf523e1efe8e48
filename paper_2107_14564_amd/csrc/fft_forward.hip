// Forward transform (step a) and the composition of the per-shell inverse
// passes; also the host planning of the shell passes and the field unblocking.
#include "fft_kernels_impl.h"

namespace bispec {

using namespace fftk;

namespace {

template <int N>
hipError_t forward_n(const float* delta, float2* spec, float beta, const float2* tw, hipStream_t st, int members,
                     long long delta_stride, long long spec_stride) {
  constexpr int M = N / 2;
  const float axis_scale = 1.0f / sqrtf((float)N);  // unitary overall: N^{-3/2}
  {
    constexpr int NL = fft_z_lines(M, false);
    const long long n_lines = (long long)N * N;
    const unsigned blocks = (unsigned)((n_lines + NL - 1) / NL);
    hipLaunchKernelGGL(k_r2c_z<N>, dim3(blocks, members), dim3(kThrZ), 0, st, delta, spec, tw, axis_scale,
                       delta_stride, spec_stride);
  }
  constexpr int TW = fwd_tile_cols(N);
  constexpr unsigned kLds = fwd_dyn_lds(N);
  const int n_ct = (M + 1 + TW - 1) / TW;
  // y: lines [x][.][kz], stride P = spec_row(N), planes x
  constexpr long long P = spec_row(N);
  hipLaunchKernelGGL(k_fft_axis<N>, dim3(N * n_ct, members), dim3(kThrAxis), kLds, st, spec, P, M + 1, (long long)N * P,
                     tw, -1.0f, axis_scale, 0, 0.0f, spec_stride);
  // x: lines [.][ky][kz], stride N P, planes ky; RSD factor applied here
  hipLaunchKernelGGL(k_fft_axis<N>, dim3(N * n_ct, members), dim3(kThrAxis), kLds, st, spec, (long long)N * P, M + 1, P,
                     tw, -1.0f, axis_scale, beta != 0.0f ? 1 : 0, beta, spec_stride);
  return hipGetLastError();
}

__global__ void k_unblock(const float* __restrict__ F, int shell, int n_s, long long n_vox, float* __restrict__ dst) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n_vox) dst[v] = F[vox_index(v, shell, n_s)];
}

}  // namespace

// Raises the dynamic LDS limit of the forward strided pass where its tile
// needs it (N >= 512); done at plan time so launches stay capture-safe.
hipError_t prepare_forward() {
  hipError_t e = hipFuncSetAttribute((const void*)k_fft_axis<512>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)fwd_dyn_lds(512));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_fft_axis<640>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fwd_dyn_lds(640));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_fft_axis<768>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fwd_dyn_lds(768));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_fft_axis<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fwd_dyn_lds(1024));
  return e;
}

hipError_t launch_forward(const float* delta, float2* spec, int n, float beta, const float2* tw, hipStream_t st,
                          int members, long long delta_stride, long long spec_stride) {
  if (members < 1) return hipErrorInvalidValue;
  switch (n) {
#define BISPEC_CASE(NN) \
  case NN: return forward_n<NN>(delta, spec, beta, tw, st, members, delta_stride, spec_stride);
    BISPEC_FOR_EACH_N(BISPEC_CASE)
#undef BISPEC_CASE
    default: return hipErrorInvalidValue;
  }
}

void plan_shell_passes(const ShellGeometry& g, int n, bool f64, ShellPassPlan& p, int nx) {
  if (nx <= 0 || nx > n) nx = n;
  const int twc = fft_tile_cols(n, f64);
  const int nl = fft_z_lines(n / 2, f64);
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
    d.wrow = shell_row(d.rad, f64);
    d.ell = g.ell.empty() ? 0 : g.ell[sn];
    d.pad_ = 0;
    const long long R = d.rad;
    d.a1_off = a1;
    d.a2_off = a2;
    a1 += (long long)n * (2 * R + 1) * d.wrow;
    a2 += (long long)nx * n * d.wrow;
    for (long long ky = -R; ky <= R; ++ky)
      for (long long kz0 = 0; kz0 <= R; kz0 += twc)
        if (ky * ky + kz0 * kz0 < d.hi2) p.x_tiles.push_back(make_int4(sn, (int)ky, (int)kz0, 0));
    const long long n_ct = (R + 1 + twc - 1) / twc;
    p.y_off.push_back(p.y_off.back() + (long long)nx * n_ct);
    p.z_off.push_back(p.z_off.back() + ((long long)nx * n + nl - 1) / nl);
  }
  p.a1_elems = a1;
  p.a2_elems = a2;
}

hipError_t launch_data_shells(const float2* spec, float2* a1, float2* a2, float* F, const ShellLaunch& L, int n,
                              const float2* tw, hipStream_t st) {
  hipError_t e = launch_inv_x_f32(spec, a1, L, n, tw, st);
  if (e == hipSuccess) e = launch_inv_y_f32(a1, a2, L, n, tw, st);
  if (e == hipSuccess) e = launch_c2r_f32(a2, F, L, n, tw, st);
  return e;
}

hipError_t launch_unit_shells(double2* a1, double2* a2, double* I, const ShellLaunch& L, int n, const double2* tw,
                              hipStream_t st) {
  hipError_t e = launch_inv_x_unit_f64(a1, L, n, tw, st);
  if (e == hipSuccess) e = launch_inv_y_f64(a1, a2, L, n, tw, st);
  if (e == hipSuccess) e = launch_c2r_f64(a2, I, L, n, tw, st);
  return e;
}

hipError_t launch_unblock(const float* F, int shell, int n_s, long long n_vox, float* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_unblock, dim3((unsigned)((n_vox + 255) / 256)), dim3(256), 0, st, F, shell, n_s, n_vox, dst);
  return hipGetLastError();
}

}  // namespace bispec
