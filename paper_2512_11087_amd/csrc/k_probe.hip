// Peak probes for roofline denominators measured on the device itself (beside
// the published peaks): a streaming copy for HBM bandwidth and a loop of
// independent float64 matrix-core operations for the FP64 MFMA rate.
#include "cv_common.h"
#include "cv_internal.h"

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

// dst = src over n16 16-byte elements, grid-stride, four 16-byte
// non-temporal loads in flight per thread before their stores (the fastest
// of the forms measured on the device).
typedef float f4v __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_probe_copy(const f4v* __restrict__ src,
                                                    f4v* __restrict__ dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    f4v v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Each wave issues `iters` (a multiple of 8) rounds of four independent
// v_mfma_f64_16x16x4_f64 (2048 flops each) on register operands, unrolled by
// 8 so the accumulators stay in the registers the matrix cores write; the
// accumulators are written out so the work is kept.
__global__ __launch_bounds__(256, 2) void k_probe_mfma(int iters, double* out) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + 1e-9 * lane, b = 1.0 - 1e-9 * lane;
  d4_t c0 = {0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
#pragma unroll 1
  for (int i = 0; i < iters; i += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
    }
  }
  const double s = (c0.x + c1.y) + (c2.z + c3.w);
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t launch_probe_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  hipLaunchKernelGGL(k_probe_copy, dim3(16384), dim3(256), 0, s, (const f4v*)src, (f4v*)dst, n16);
  return hipGetLastError();
}

hipError_t launch_probe_mfma(int blocks, int iters, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(256), 0, s, iters, out);
  return hipGetLastError();
}
