// Inverse z pass (C2R) of every shell, writing the voxel-blocked shell fields.
#include "fft_kernels_impl.h"

namespace bispec {

using namespace fftk;

template <typename T, typename OutT>
static hipError_t c2r(const V2<T>* a2, OutT* out, const ShellLaunch& L, int n, const V2<T>* tw, hipStream_t st) {
  if (L.n_z_blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)L.n_z_blocks, (unsigned)L.n_members);
  switch (n) {
#define BISPEC_CASE(NN)                                                                                        \
  case NN:                                                                                                     \
    hipLaunchKernelGGL((k_c2r_z<T, OutT, NN>), grid, dim3(kThrZ), 0, st, a2, out, L.z_off, L.n_shells, \
                       L.shells, tw, L.n_lines > 0 ? L.n_lines : (long long)n * n, L.a2_stride, L.f_stride); \
    break;
    BISPEC_FOR_EACH_N(BISPEC_CASE)
#undef BISPEC_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_c2r_f32(const float2* a2, float* F, const ShellLaunch& L, int n, const float2* tw,
                          hipStream_t st) {
  return c2r<float, float>(a2, F, L, n, tw, st);
}

hipError_t launch_c2r_f64(const double2* a2, double* I, const ShellLaunch& L, int n, const double2* tw,
                          hipStream_t st) {
  return c2r<double, double>(a2, I, L, n, tw, st);
}

}  // namespace bispec
