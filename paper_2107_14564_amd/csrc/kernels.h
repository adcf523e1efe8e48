// Launch interface between the plan runtime (api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "geometry.h"

namespace bispec {

constexpr int kFftThreads = 256;
constexpr int kFftElemsF32 = 32;  // LDS tile of an fp32 FFT block = 32 * 256 complex (64 KB)
constexpr int kFftElemsF64 = 16;  // LDS tile of an fp64 FFT block = 16 * 256 complex (64 KB)

// columns per block of a strided pass over lines of length n
__host__ __device__ inline int fft_tile_cols(int n, bool f64) {
  return (kFftThreads * (f64 ? kFftElemsF64 : kFftElemsF32)) / n;
}
// lines per block of a contiguous pass over lines of length len (LDS stride len + 1)
__host__ __device__ inline int fft_tile_lines(int len, bool f64) {
  return (kFftThreads * (f64 ? kFftElemsF64 : kFftElemsF32)) / (len + 1);
}

struct ShellDev {
  long long lo2, hi2;   // shell holds lo2 <= |m|^2 < hi2
  long long a1_off;     // element offset of A1_n
  long long a2_off;     // element offset of A2_n
  int rad;              // R = floor(sqrt(hi2 - 1))
  int pad;
};

struct ShellLaunch {
  int n_shells = 0;
  const ShellDev* shells = nullptr;   // device [n_shells]
  const int4* x_tiles = nullptr;      // device (shell, ky, kz0, 0)
  long long n_x_tiles = 0;
  const long long* y_off = nullptr;   // device prefix sums [n_shells + 1]
  long long n_y_blocks = 0;
  const long long* z_off = nullptr;   // device prefix sums [n_shells + 1]
  long long n_z_blocks = 0;
};

// host-side description of the shell passes; device arrays are uploaded by the caller
struct ShellPassPlan {
  std::vector<ShellDev> shells;
  std::vector<int4> x_tiles;
  std::vector<long long> y_off, z_off;
  long long a1_elems = 0, a2_elems = 0;
};
void plan_shell_passes(const ShellGeometry& g, bool f64, ShellPassPlan& p);

hipError_t launch_forward(const float* delta, float2* spec, int n, float beta, const float2* tw, hipStream_t st);
hipError_t launch_data_shells(const float2* spec, float2* a1, float2* a2, float* F, long long field_stride,
                              const ShellLaunch& L, int n, const float2* tw, hipStream_t st);
hipError_t launch_unit_shells(double2* a1, double2* a2, double* I, long long field_stride, const ShellLaunch& L, int n,
                              const double2* tw, hipStream_t st);

// ---- contraction ---------------------------------------------------------------
struct ContractArgs {
  const RowBlock* rows = nullptr;   // device
  const Tile* tiles = nullptr;      // device, task-major
  const int32_t* task_off = nullptr;  // device [n_tasks + 1] (task grouping of the kernel launched)
  int n_tasks = 0;
  const int32_t* tri_index = nullptr; // device [n_s^3]: (i-1, j-1, l-1) -> triangle or -1
  int n_s = 0;
  long long n_vox = 0;               // voxels per field
  int n_krange = 0;                  // voxel ranges (multiple of 8)
  double* partial = nullptr;         // device [n_krange][n_tri]
  long long n_tri = 0;
};

hipError_t launch_contract_fp32(const float* F, const ContractArgs& a, hipStream_t st);
hipError_t launch_contract_fp64(const double* F, const ContractArgs& a, hipStream_t st);
hipError_t launch_contract_bf16x3(const float* F, const ContractArgs& a, hipStream_t st);
// B[t] = norm[t] * sum_k partial[k][t] (fixed order, float64)
hipError_t launch_reduce(const double* partial, int n_krange, long long n_tri, const double* norm, double* out,
                         hipStream_t st);

}  // namespace bispec
