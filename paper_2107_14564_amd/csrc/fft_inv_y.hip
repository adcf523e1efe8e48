// Inverse y pass of every shell (fp32 data shells, fp64 unit shells).
#include "fft_kernels_impl.h"

namespace bispec {

using namespace fftk;

template <typename T>
static hipError_t inv_y(const V2<T>* a1, V2<T>* a2, const ShellLaunch& L, int n, const V2<T>* tw, hipStream_t st) {
  if (L.n_y_blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)L.n_y_blocks, (unsigned)L.n_members);
  switch (n) {
#define BISPEC_CASE(NN)                                                                                    \
  case NN:                                                                                                 \
    hipLaunchKernelGGL((k_inv_y<T, NN>), grid, dim3(kThrAxis), 0, st, a1, a2, L.y_off, L.n_shells, L.shells, tw, \
                       L.x0, L.x_end > 0 ? L.x_end : n, L.a1_stride, L.a2_stride);                              \
    break;
    BISPEC_FOR_EACH_N(BISPEC_CASE)
#undef BISPEC_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_inv_y_f32(const float2* a1, float2* a2, const ShellLaunch& L, int n, const float2* tw,
                            hipStream_t st) {
  return inv_y<float>(a1, a2, L, n, tw, st);
}

hipError_t launch_inv_y_f64(const double2* a1, double2* a2, const ShellLaunch& L, int n, const double2* tw,
                            hipStream_t st) {
  return inv_y<double>(a1, a2, L, n, tw, st);
}

}  // namespace bispec
