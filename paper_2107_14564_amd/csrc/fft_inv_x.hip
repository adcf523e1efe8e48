// Inverse x pass of every shell (step b: data shells in fp32; step b2: unit shells in fp64).
#include "fft_kernels_impl.h"

namespace bispec {

using namespace fftk;

template <typename T, bool UNIT>
static hipError_t inv_x(const float2* spec, V2<T>* a1, const ShellLaunch& L, int n, const V2<T>* tw,
                        hipStream_t st) {
  if (L.n_x_tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)L.n_x_tiles, (unsigned)L.n_members);
  switch (n) {
#define BISPEC_CASE(NN)                                                                                     \
  case NN:                                                                                                  \
    hipLaunchKernelGGL((k_inv_x<T, UNIT, NN>), grid, dim3(kThrAxis), 0, st, spec, L.spec_n, a1, L.x_tiles, L.shells, tw, \
                       L.spec_stride, L.a1_stride);                                                        \
    break;
    BISPEC_FOR_EACH_N(BISPEC_CASE)
#undef BISPEC_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_inv_x_f32(const float2* spec, float2* a1, const ShellLaunch& L, int n, const float2* tw,
                            hipStream_t st) {
  return inv_x<float, false>(spec, a1, L, n, tw, st);
}

hipError_t launch_inv_x_unit_f64(double2* a1, const ShellLaunch& L, int n, const double2* tw, hipStream_t st) {
  return inv_x<double, true>(nullptr, a1, L, n, tw, st);
}

}  // namespace bispec
