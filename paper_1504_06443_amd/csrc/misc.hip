// Elementwise helpers: copies, symmetrisation and fills (HBM-bound, coalesced
// along columns; 2D grid of 64 x 4 thread blocks walking a column-major matrix).
#include "common.h"

namespace gep {
namespace {

constexpr int TX = 64, TY = 4, COLS_PER = 16;

__global__ void copy_kernel(int64_t m, int64_t n, const double* __restrict__ src, int64_t lds,
                            double* __restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * TX + threadIdx.x;
  if (i >= m) return;
  const int64_t j0 = ((int64_t)blockIdx.y * TY + threadIdx.y) * COLS_PER;
  for (int c = 0; c < COLS_PER; ++c) {
    const int64_t j = j0 + c;
    if (j >= n) break;
    dst[i + j * ldd] = src[i + j * lds];
  }
}

__global__ void symm_kernel(int64_t n, const double* __restrict__ src, int64_t lds,
                            double* __restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * TX + threadIdx.x;
  if (i >= n) return;
  const int64_t j0 = ((int64_t)blockIdx.y * TY + threadIdx.y) * COLS_PER;
  for (int c = 0; c < COLS_PER; ++c) {
    const int64_t j = j0 + c;
    if (j >= n) break;
    dst[i + j * ldd] = (i >= j) ? src[i + j * lds] : src[j + i * lds];
  }
}

__global__ void set_kernel(int64_t m, int64_t n, double off, double diag, double* __restrict__ dst,
                           int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * TX + threadIdx.x;
  if (i >= m) return;
  const int64_t j0 = ((int64_t)blockIdx.y * TY + threadIdx.y) * COLS_PER;
  for (int c = 0; c < COLS_PER; ++c) {
    const int64_t j = j0 + c;
    if (j >= n) break;
    dst[i + j * ldd] = (i == j) ? diag : off;
  }
}

__global__ void zero_upper_kernel(int64_t n, double* __restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * TX + threadIdx.x;
  if (i >= n) return;
  const int64_t j0 = ((int64_t)blockIdx.y * TY + threadIdx.y) * COLS_PER;
  for (int c = 0; c < COLS_PER; ++c) {
    const int64_t j = j0 + c;
    if (j >= n) break;
    if (i < j) dst[i + j * ldd] = 0.0;
  }
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// info <- code when the flag is set and info still reads success (an earlier
// failure keeps its code).
__global__ void flag_to_info_kernel(const int32_t* flag, int32_t* info, int32_t code) {
  if (*flag != 0) atomicCAS(info, 0, code);
}
__global__ void info_if_zero_kernel(int32_t* info, int32_t code) { atomicCAS(info, 0, code); }

dim3 grid2(int64_t m, int64_t n) {
  return dim3((unsigned)cdiv(m, TX), (unsigned)cdiv(cdiv(n, COLS_PER), TY));
}

}  // namespace

void copy_matrix(int64_t m, int64_t n, const double* src, int64_t lds, double* dst, int64_t ldd,
                 hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(copy_kernel, grid2(m, n), dim3(TX, TY), 0, s, m, n, src, lds, dst, ldd);
  GEP_LAUNCH_CHECK();
}

void symmetrize_from_lower(int64_t n, const double* src, int64_t lds, double* dst, int64_t ldd,
                           hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(symm_kernel, grid2(n, n), dim3(TX, TY), 0, s, n, src, lds, dst, ldd);
  GEP_LAUNCH_CHECK();
}

void set_matrix(int64_t m, int64_t n, double off, double diag, double* dst, int64_t ldd,
                hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(set_kernel, grid2(m, n), dim3(TX, TY), 0, s, m, n, off, diag, dst, ldd);
  GEP_LAUNCH_CHECK();
}

void zero_upper(int64_t n, double* dst, int64_t ldd, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_upper_kernel, grid2(n, n), dim3(TX, TY), 0, s, n, dst, ldd);
  GEP_LAUNCH_CHECK();
}

void fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, p, n, v);
  GEP_LAUNCH_CHECK();
}

void fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, p, n, v);
  GEP_LAUNCH_CHECK();
}

void raise_info(int32_t* info, int32_t code, hipStream_t s) {
  if (!info) return;
  hipLaunchKernelGGL(info_if_zero_kernel, dim3(1), dim3(1), 0, s, info, code);
  GEP_LAUNCH_CHECK();
}

void raise_info_if(const int32_t* flag, int32_t* info, int32_t code, hipStream_t s) {
  if (!flag || !info) return;
  hipLaunchKernelGGL(flag_to_info_kernel, dim3(1), dim3(1), 0, s, flag, info, code);
  GEP_LAUNCH_CHECK();
}

}  // namespace gep
