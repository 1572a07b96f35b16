// Plain device copy of known size, used only to calibrate the hardware byte
// counters (FETCH_SIZE, WRITE_SIZE) against which the traffic of the
// method's kernels is reported.  Every lane moves one 4-byte word, the same
// access width as the method's kernels.  Not part of the time step.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

__global__ void __launch_bounds__(256) k_copy_words(const uint32_t *__restrict__ src,
                                                    uint32_t *__restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Copy n_words 4-byte words from src to dst (device pointers) on stream.
// Returns 0, -1 for a null pointer or a grid beyond 2^31 blocks, -4 if the
// launch failed.
extern "C" int fdlbm_calib_copy(const void *src, void *dst, size_t n_words, void *stream) {
  if (!src || !dst) return -1;
  const size_t blocks = (n_words + 255) / 256;
  if (blocks == 0) return 0;
  if (blocks > 0x7fffffffu) return -1;
  hipLaunchKernelGGL(k_copy_words, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     (const uint32_t *)src, (uint32_t *)dst, n_words);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
