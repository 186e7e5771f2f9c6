// probe.hip -- the measurement kernel bench.py runs beside the evaluator (not
// part of the evaluation path): the attainable integer-bitwise VALU rate of
// the device, the denominator check of the algorithmic fraction.
//
// k_valu_peak: every lane runs 8 independent chains of v_bitop3_b32 (each
// chain depends only on itself and on two loop-invariant operands), so the
// only limit is VALU issue.  fbg_probe_valu_peak launches it on `stream` and
// returns after queueing; the caller times it with events and reads nothing
// back but the checksum words (which keep the chains live).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__global__ __launch_bounds__(256) void k_valu_peak(uint32_t *out, uint32_t iters, uint32_t seed) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a0 = seed ^ tid, a1 = a0 * 3u, a2 = a0 * 5u, a3 = a0 * 7u;
  uint32_t a4 = a0 * 11u, a5 = a0 * 13u, a6 = a0 * 17u, a7 = a0 * 19u;
  const uint32_t b = seed * 0x9E3779B9u, c = seed ^ 0x85EBCA6Bu;
  for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
    for (int r = 0; r < 8; r++) {
      a0 = __builtin_amdgcn_bitop3_b32(a0, b, c, 0x96);
      a1 = __builtin_amdgcn_bitop3_b32(a1, b, c, 0xE8);
      a2 = __builtin_amdgcn_bitop3_b32(a2, b, c, 0x96);
      a3 = __builtin_amdgcn_bitop3_b32(a3, b, c, 0xE8);
      a4 = __builtin_amdgcn_bitop3_b32(a4, b, c, 0x96);
      a5 = __builtin_amdgcn_bitop3_b32(a5, b, c, 0xE8);
      a6 = __builtin_amdgcn_bitop3_b32(a6, b, c, 0x96);
      a7 = __builtin_amdgcn_bitop3_b32(a7, b, c, 0xE8);
    }
  }
  out[tid] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

}  // namespace

extern "C" {

// Queue one launch of `blocks` x 256 threads, each issuing 64 * iters
// v_bitop3_b32; `out` holds blocks * 256 uint32 words (device memory).
// Returns 0, or the HIP error code of the launch.
int fbg_probe_valu_peak(uint32_t *out, int32_t blocks, uint32_t iters, uint32_t seed, void *stream) {
  if (!out || blocks <= 0) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_valu_peak, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, out, iters, seed);
  return (int)hipGetLastError();
}

}  // extern "C"
