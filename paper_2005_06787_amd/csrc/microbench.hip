// Ceiling microbenchmarks of one MI355X, used to judge the stem kernels:
// streaming copy bandwidth (8- or 16-byte accesses per lane) and the dense
// matrix-core rates of the MFMA shapes the products use.

#include <hip/hip_runtime.h>

#include <string>

#include "stem_internal.h"

using namespace stem;

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T>
__global__ __launch_bounds__(256) void mb_copy_kernel(const T* __restrict__ src,
                                                      T* __restrict__ dst, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

// UNROLL loads in flight per lane before the stores; NT: non-temporal
// (streaming) loads and stores.
template <int UNROLL, int NT>
__global__ __launch_bounds__(256) void mb_copy_unrolled_kernel(const f32x4* __restrict__ src,
                                                               f32x4* __restrict__ dst,
                                                               uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (UNROLL - 1) * stride < n; i += UNROLL * stride) {
    f32x4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u)
      v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      if (NT)
        __builtin_nontemporal_store(v[u], dst + i + u * stride);
      else
        dst[i + u * stride] = v[u];
    }
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Every wave runs 8 independent accumulator chains of `iters` MFMAs each;
// the operands are lane values that the compiler cannot fold.
template <int KIND>
__global__ __launch_bounds__(256) void mb_mfma_kernel(int64_t iters, float* __restrict__ out) {
  const float x = (float)threadIdx.x * 1e-3f;
  f32x4 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (KIND == 0) {
    const float a = x, b = 1.f - x;
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  } else if (KIND == 1) {
    f16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a[i] = (_Float16)(x + i);
      b[i] = (_Float16)(1.f - x);
    }
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[c], 0, 0, 0);
  } else {
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a[i] = (__bf16)(x + i);
      b[i] = (__bf16)(1.f - x);
    }
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

stem_status mb_fail(const char* what, hipError_t e) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return STEM_EHIP;
}

}  // namespace

extern "C" {

stem_status stem_mb_copy(const void* src, void* dst, uint64_t bytes, int32_t vec_bytes,
                         int32_t blocks, void* stream) {
  if (!src || !dst) {
    set_error("null pointer");
    return STEM_EINVAL;
  }
  const bool unrolled = vec_bytes == 64 || vec_bytes == 65;
  if ((vec_bytes != 8 && vec_bytes != 16 && !unrolled) || bytes % 16 || blocks < 1) {
    set_error("vec_bytes must be 8, 16, 64 or 65 and bytes a multiple of 16; blocks >= 1");
    return STEM_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  if (vec_bytes == 64)
    hipLaunchKernelGGL((mb_copy_unrolled_kernel<4, 0>), dim3(blocks), dim3(256), 0, st,
                       (const f32x4*)src, (f32x4*)dst, bytes / 16);
  else if (vec_bytes == 65)
    hipLaunchKernelGGL((mb_copy_unrolled_kernel<4, 1>), dim3(blocks), dim3(256), 0, st,
                       (const f32x4*)src, (f32x4*)dst, bytes / 16);
  else if (vec_bytes == 16)
    hipLaunchKernelGGL(mb_copy_kernel<f32x4>, dim3(blocks), dim3(256), 0, st, (const f32x4*)src,
                       (f32x4*)dst, bytes / 16);
  else
    hipLaunchKernelGGL(mb_copy_kernel<float2>, dim3(blocks), dim3(256), 0, st,
                       (const float2*)src, (float2*)dst, bytes / 8);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STEM_OK : mb_fail("copy", e);
}

stem_status stem_mb_mfma(int32_t kind, int64_t iters, int32_t blocks, float* out, void* stream) {
  if (!out || iters < 1 || blocks < 1 || kind < 0 || kind > 2) {
    set_error("bad argument");
    return STEM_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  if (kind == 0)
    hipLaunchKernelGGL(mb_mfma_kernel<0>, dim3(blocks), dim3(256), 0, st, iters, out);
  else if (kind == 1)
    hipLaunchKernelGGL(mb_mfma_kernel<1>, dim3(blocks), dim3(256), 0, st, iters, out);
  else
    hipLaunchKernelGGL(mb_mfma_kernel<2>, dim3(blocks), dim3(256), 0, st, iters, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STEM_OK : mb_fail("mfma", e);
}

}  // extern "C"
