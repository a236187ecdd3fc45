// Calibration kernels: what the device sustains for the two resources the
// solver is bound by (FP64 vector FMA issue, HBM streaming writes), and a
// plain copy of known size, the reference against which hardware traffic
// counters are scaled; and the solver's three reciprocals, whose accuracy
// its error reasoning relies on.  They touch only the buffers they are given.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/arrow.h"
#include "solver.hpp"

namespace {

constexpr int PROBE_BLOCK = 256;
constexpr int FMA_CHAINS = 8;
typedef double v2d __attribute__((ext_vector_type(2)));

// FMA_CHAINS independent chains per lane, `iters` dependent FMAs each; the
// sum of the chains is stored so that nothing is optimised away.
__global__ __launch_bounds__(PROBE_BLOCK) void k_probe_fma(double* out, int iters, double a, double b) {
  double x[FMA_CHAINS];
#pragma unroll
  for (int c = 0; c < FMA_CHAINS; ++c) x[c] = (double)(threadIdx.x + c);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < FMA_CHAINS; ++c) x[c] = fma(x[c], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < FMA_CHAINS; ++c) s += x[c];
  out[(size_t)blockIdx.x * PROBE_BLOCK + threadIdx.x] = s;
}

// grid-stride 16-byte streaming stores
__global__ __launch_bounds__(PROBE_BLOCK) void k_probe_fill(v2d* dst, int64_t n2, double v) {
  const int64_t stride = (int64_t)gridDim.x * PROBE_BLOCK;
  const v2d val = {v, v};
  for (int64_t i = (int64_t)blockIdx.x * PROBE_BLOCK + threadIdx.x; i < n2; i += stride)
    __builtin_nontemporal_store(val, dst + i);
}

__global__ __launch_bounds__(PROBE_BLOCK) void k_probe_copy(v2d* dst, const v2d* src, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * PROBE_BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * PROBE_BLOCK + threadIdx.x; i < n2; i += stride) dst[i] = src[i];
}

// the solver's reciprocals of x[i]: out[i] the bare estimate, out[n + i] one
// Newton step, out[2n + i] two
__global__ __launch_bounds__(PROBE_BLOCK) void k_probe_rcp(const double* x, double* out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * PROBE_BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * PROBE_BLOCK + threadIdx.x; i < n; i += stride) {
    const double v = x[i];
    out[i] = ahd::recip_est(v);
    out[n + i] = ahd::recip1(v);
    out[2 * n + i] = ahd::recip(v);
  }
}

int grid_for(int64_t items, int cap) {
  const int64_t g = (items + PROBE_BLOCK - 1) / PROBE_BLOCK;
  return (int)(g < cap ? (g > 0 ? g : 1) : cap);
}

}  // namespace

extern "C" {

int arrow_probe_fma(double* out, int64_t blocks, int iters, void* stream) {
  if (!out) return -1;
  if (blocks < 1 || blocks > (1 << 24)) return -2;
  if (iters < 1) return -3;
  hipLaunchKernelGGL(k_probe_fma, dim3((unsigned)blocks), dim3(PROBE_BLOCK), 0, (hipStream_t)stream, out, iters,
                     0.999999999, 1e-9);
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

int arrow_probe_fill(double* dst, int64_t bytes, double value, void* stream) {
  if (!dst || ((uintptr_t)dst & 15)) return -1;
  if (bytes < 16 || (bytes & 15)) return -2;
  const int64_t n2 = bytes / 16;
  hipLaunchKernelGGL(k_probe_fill, dim3((unsigned)grid_for(n2, 1 << 16)), dim3(PROBE_BLOCK), 0, (hipStream_t)stream,
                     (v2d*)dst, n2, value);
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

int arrow_probe_copy(double* dst, const double* src, int64_t bytes, void* stream) {
  if (!dst || ((uintptr_t)dst & 15)) return -1;
  if (!src || ((uintptr_t)src & 15)) return -2;
  if (bytes < 16 || (bytes & 15)) return -3;
  const int64_t n2 = bytes / 16;
  hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)grid_for(n2, 1 << 16)), dim3(PROBE_BLOCK), 0, (hipStream_t)stream,
                     (v2d*)dst, (const v2d*)src, n2);
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

int arrow_probe_rcp(const double* x, double* out, int64_t n, void* stream) {
  if (!x) return -1;
  if (!out) return -2;
  if (n < 1) return -3;
  hipLaunchKernelGGL(k_probe_rcp, dim3((unsigned)grid_for(n, 1 << 16)), dim3(PROBE_BLOCK), 0, (hipStream_t)stream, x,
                     out, n);
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

}  // extern "C"
