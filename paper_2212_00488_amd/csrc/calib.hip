// Peak-rate probes (include/stereo_calib.h): LDS read bandwidth, 32-bit
// integer VALU rate and device-memory copy bandwidth of the device.
#include "stereo_calib.h"

#include <hip/hip_runtime.h>

#include "stereo.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCalibThreads = 1024;
constexpr int kLdsWords = 64 * 1024 / 16;  // 64 KiB of 16-byte words

// Each wave's 16-byte load covers 1 KiB of consecutive LDS (lane l reads
// word base + l): every bank serves the same number of lanes.  The four
// loads of a step sit 16 KiB apart; a compiler barrier between steps makes
// every step reload.  Two 3-input adds fold each load into the sinks.
__global__ void __launch_bounds__(kCalibThreads) k_calib_lds(uint32_t* __restrict__ sink,
                                                             int iters) {
  __shared__ u32x4 buf[kLdsWords];
  const int t = threadIdx.x;
  for (int i = t; i < kLdsWords; i += kCalibThreads)
    buf[i] = u32x4{(uint32_t)i, (uint32_t)i * 3u, (uint32_t)i * 5u, (uint32_t)i * 7u};
  __syncthreads();
  uint32_t a = 0, b = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const u32x4 v = buf[t + (k & 3) * kCalibThreads];
      a += v.x + v.y;
      b += v.z + v.w;
      if ((k & 3) == 3) __asm__ volatile("" ::: "memory");
    }
  }
  sink[blockIdx.x * kCalibThreads + t] = a ^ b;
}

// 16 independent chains of a 32-bit add and a xor per step (the chains keep
// every SIMD issuing without a dependency stall).
__global__ void __launch_bounds__(kCalibThreads) k_calib_valu(uint32_t* __restrict__ sink,
                                                              int iters) {
  uint32_t x[16], y[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    x[j] = threadIdx.x + j;
    y[j] = blockIdx.x * 7u + j * 13u;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        x[j] += y[j];
        y[j] ^= x[j];
      }
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) s ^= x[j] + y[j];
  sink[blockIdx.x * kCalibThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_calib_copy(const u32x4* __restrict__ src,
                                                    u32x4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

int launched() { return hipGetLastError() == hipSuccess ? 0 : STEREO_EHIP; }

}  // namespace

extern "C" {

int stereo_calib_lds_read(uint32_t* sink, int blocks, int iters, hipStream_t stream) {
  if (!sink || blocks < 1 || iters < 1) return STEREO_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_calib_lds, dim3(blocks), dim3(kCalibThreads), 0, stream, sink, iters);
  return launched();
}

int stereo_calib_valu(uint32_t* sink, int blocks, int iters, hipStream_t stream) {
  if (!sink || blocks < 1 || iters < 1) return STEREO_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_calib_valu, dim3(blocks), dim3(kCalibThreads), 0, stream, sink, iters);
  return launched();
}

int stereo_calib_copy(const void* src, void* dst, size_t bytes, int blocks, hipStream_t stream) {
  if (!src || !dst || blocks < 1 || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
    return STEREO_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_calib_copy, dim3(blocks), dim3(256), 0, stream,
                     static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), bytes / 16);
  return launched();
}

}  // extern "C"
