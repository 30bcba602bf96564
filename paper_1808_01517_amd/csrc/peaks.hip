// Reference kernels for the roofline: a device-to-device copy (the HBM
// bandwidth this GPU actually delivers to a streaming kernel) and MFMA
// loops (the matrix-core rates it delivers), measured on the same GPU as
// the layers' kernels so that every roofline fraction can be given against
// the spec-sheet peak and against the measured one.  Measurement only: no
// layer calls these.
#include <hip/hip_runtime.h>

#include "gemm_common.h"
#include "internal.h"

namespace dlm {
namespace {

// One block per 8 KB chunk: each lane loads two 16-byte runs (256 lanes
// apart, so every load instruction covers 4 KB contiguously), then stores
// them.  Measured faster than grid-stride loops with deeper unrolling.
constexpr int kCopyUnroll = 2;
constexpr size_t kCopyChunk16 = size_t(kCopyUnroll) * 256;  // 16-byte runs per block

__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst) {
  const size_t base = (size_t)blockIdx.x * kCopyChunk16 + threadIdx.x;
  uint4 v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) v[u] = src[base + u * 256];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) dst[base + u * 256] = v[u];
}

__global__ void copy_tail(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, size_t n4) {
  const size_t i = (size_t)blockIdx.x * 64 + threadIdx.x;
  if (i < n4) dst[i] = src[i];
}

// Sixteen (FP32) or eight (BF16, 32 x 32 tiles) independent accumulator
// chains per wave: a 16 x 16 MFMA's result is ready for the next MFMA on
// the same accumulator only ~16 issue slots later, so fewer chains leave
// the matrix core idle (eight 16x16x4 chains measured 139 TFLOP/s, sixteen
// 155).  The operands depend on the lane and the result is stored, so
// nothing is folded away.
constexpr int kChainsF32 = 16, kChainsBf16 = 8;

__global__ __launch_bounds__(256) void mfma_f32_loop(int iters, float *out) {
  const int lane = threadIdx.x & 63;
  const float a = 1.0f + lane * 1e-3f, b = 0.5f - lane * 1e-3f;
  floatx4 acc[kChainsF32];
#pragma unroll
  for (int j = 0; j < kChainsF32; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChainsF32; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChainsF32; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void mfma_bf16_loop(int iters, float *out) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1.0f + (lane + e) * 1e-3f);
    b[e] = (__bf16)(0.5f - (lane + e) * 1e-3f);
  }
  floatx16 acc[kChainsBf16];
#pragma unroll
  for (int j = 0; j < kChainsBf16; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[j][e] = 0.f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChainsBf16; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChainsBf16; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[j][e];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace
}  // namespace dlm

extern "C" {

dlm_status dlm_peak_copy(const void *src, void *dst, size_t bytes, void *stream) {
  if (bytes == 0) return DLM_OK;
  if (!src || !dst) return dlm::report(DLM_EINVAL, "null device pointer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
    return dlm::report(DLM_EINVAL, "copy buffers must be 16-byte aligned");
  if (bytes % 4) return dlm::report(DLM_EINVAL, "bytes must be a multiple of 4");
  hipStream_t st = (hipStream_t)stream;
  // whole 8 KB chunks by the block kernel, the rest (< 8 KB) 4 bytes a lane
  const size_t blocks = bytes / (dlm::kCopyChunk16 * 16);
  if (blocks > 0x7fffffff) return dlm::report(DLM_EINVAL, "copy of %zu bytes is too large", bytes);
  if (blocks)
    hipLaunchKernelGGL(dlm::copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst));
  const size_t n16 = blocks * dlm::kCopyChunk16;
  const size_t n4 = (bytes - n16 * 16) / 4;
  if (n4)
    hipLaunchKernelGGL(dlm::copy_tail, dim3((unsigned)((n4 + 63) / 64)), dim3(64), 0, st,
                       reinterpret_cast<const uint32_t *>(static_cast<const char *>(src) + n16 * 16),
                       reinterpret_cast<uint32_t *>(static_cast<char *>(dst) + n16 * 16), n4);
  return hipGetLastError() == hipSuccess ? DLM_OK
                                         : dlm::report(DLM_EDEVICE, "kernel launch failed: %s",
                                                       hipGetErrorString(hipGetLastError()));
}

size_t dlm_peak_mfma_out_floats(int blocks) { return blocks > 0 ? size_t(blocks) * 256 : 0; }

double dlm_peak_mfma_flops(dlm_precision prec, int blocks, int iters) {
  const double per = prec == DLM_BF16 ? 2.0 * 32 * 32 * 16 * dlm::kChainsBf16 : 2.0 * 16 * 16 * 4 * dlm::kChainsF32;
  return blocks > 0 && iters > 0 ? double(blocks) * 4 * iters * per : 0.0;
}

dlm_status dlm_peak_mfma(dlm_precision prec, int blocks, int iters, float *out, void *stream) {
  if (prec != DLM_FP32 && prec != DLM_BF16) return dlm::report(DLM_EINVAL, "unknown precision %d", int(prec));
  if (blocks <= 0 || iters <= 0 || !out) return dlm::report(DLM_EINVAL, "blocks and iters must be > 0, out non-null");
  hipStream_t st = (hipStream_t)stream;
  if (prec == DLM_BF16)
    hipLaunchKernelGGL(dlm::mfma_bf16_loop, dim3(blocks), dim3(256), 0, st, iters, out);
  else
    hipLaunchKernelGGL(dlm::mfma_f32_loop, dim3(blocks), dim3(256), 0, st, iters, out);
  return hipGetLastError() == hipSuccess ? DLM_OK
                                         : dlm::report(DLM_EDEVICE, "kernel launch failed: %s",
                                                       hipGetErrorString(hipGetLastError()));
}

}  // extern "C"
