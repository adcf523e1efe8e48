// Adjoint transform of the per-shell fields (gradient, step g): pruned forward
// passes of every G_n scattered into one half spectrum.
#include "fft_kernels_impl.h"

namespace bispec {

using namespace fftk;

namespace {

__global__ void k_zero(float2* __restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_float2(0.f, 0.f);
}

template <int N>
hipError_t adjoint_n(const float* G, float2* a1, float2* a2, float2* S, const ShellLaunch& L, const float2* tw,
                     float scale, float beta, bool zero_first, hipStream_t st) {
  const long long sn = L.spec_n;
  const long long n_spec = sn * sn * spec_row((int)sn);
  if (zero_first) hipLaunchKernelGGL(k_zero, dim3((unsigned)((n_spec + 255) / 256)), dim3(256), 0, st, S, n_spec);
  if (L.n_z_blocks > 0)
    hipLaunchKernelGGL(k_g_r2c_z<N>, dim3((unsigned)L.n_z_blocks), dim3(kThrZ), 0, st, G, a2, L.z_off, L.n_shells,
                       L.shells, tw);
  if (L.n_y_blocks > 0)
    hipLaunchKernelGGL(k_g_fwd_y<N>, dim3((unsigned)L.n_y_blocks), dim3(kThrAxis), 0, st, a2, a1, L.y_off,
                       L.n_shells, L.shells, tw);
  if (L.n_x_tiles > 0)
    hipLaunchKernelGGL(k_g_fwd_x<N>, dim3((unsigned)L.n_x_tiles), dim3(kThrAxis), 0, st, a1, S, L.spec_n, L.x_tiles,
                       L.shells, tw, scale, beta);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_shells(const float* G, float2* a1, float2* a2, float2* S, const ShellLaunch& L, int n,
                                 const float2* tw, float scale, float beta, bool zero_first, hipStream_t st) {
  switch (n) {
#define BISPEC_CASE(NN) \
  case NN: return adjoint_n<NN>(G, a1, a2, S, L, tw, scale, beta, zero_first, st);
    BISPEC_FOR_EACH_N(BISPEC_CASE)
#undef BISPEC_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bispec
