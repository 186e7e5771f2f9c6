// probe.hip -- measurement kernels used by bench.py beside the evaluator (not
// part of the evaluation path): the attainable integer-bitwise VALU rate of
// the device, the denominator check of the algorithmic fraction, and the
// write rate of the DNF write-out's store pattern alone, in three forms.
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

// The DNF write-out's store pattern without the evaluation, in three forms.
// A wave writes tiles of 32 x 64 words (8 KiB), striding over the tiles; NT
// selects non-temporal stores, as the evaluator uses.
//   FORM 0: word i of lane l at tile * 2048 + i * 64 + l: 32 stores of 4
//           bytes per lane (256 contiguous bytes per instruction), the
//           evaluator's register layout stored as it is;
//   FORM 1: the same 8 KiB as 8 stores of 16 bytes per lane (1 KiB
//           contiguous per instruction), values made in place;
//   FORM 3: FORM 0 with each wave writing `run` consecutive tiles in a row;
//   FORM 2: FORM 0's register layout turned into FORM 1's stores through
//           LDS: each half tile (16 rows, 4 KiB per wave) is written to LDS
//           row by row and read back as 16-byte columns.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// LDS written by the lanes of a wave is read by other lanes of the same wave
// only after this point (no code motion across it; no instruction emitted).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool NT, int FORM>
__global__ __launch_bounds__(256) void k_store_tiles(uint32_t *p, uint64_t ntiles, uint32_t run) {
  __shared__ uint32_t stage[FORM == 2 ? 4 * 1024 : 1];
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  uint32_t *ws = stage + (threadIdx.x >> 6) * 1024;
  auto rows_b32 = [&](uint64_t t) {
    uint32_t *dst = p + t * 2048 + lane;
#pragma unroll
    for (int i = 0; i < 32; i++) {
      const uint32_t v = (uint32_t)t ^ (uint32_t)i ^ lane;
      if (NT)
        __builtin_nontemporal_store(v, dst + i * 64);
      else
        dst[i * 64] = v;
    }
  };
  if (FORM == 3) {  // FORM 0's stores, `run` consecutive tiles per wave at a time
    for (uint64_t r = wave; r * run < ntiles; r += nw)
      for (uint64_t t = r * run; t < r * run + run && t < ntiles; t++) rows_b32(t);
    return;
  }
  for (uint64_t t = wave; t < ntiles; t += nw) {
    if (FORM == 0) {
      rows_b32(t);
    } else if (FORM == 1) {
      u32x4 *dst = (u32x4 *)(p + t * 2048) + lane;
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const uint32_t b = (uint32_t)t ^ (uint32_t)k ^ lane;
        const u32x4 v = {b, b + 1u, b + 2u, b + 3u};
        if (NT)
          __builtin_nontemporal_store(v, dst + k * 64);
        else
          dst[k * 64] = v;
      }
    } else {
      u32x4 *dst = (u32x4 *)(p + t * 2048) + lane;
#pragma unroll
      for (int h = 0; h < 2; h++) {
#pragma unroll
        for (int i = 0; i < 16; i++) ws[i * 64 + lane] = (uint32_t)t ^ (uint32_t)(16 * h + i) ^ lane;
        wave_lds_sync();
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const u32x4 v = ((const u32x4 *)ws)[k * 64 + lane];
          if (NT)
            __builtin_nontemporal_store(v, dst + (4 * h + k) * 64);
          else
            dst[(4 * h + k) * 64] = v;
        }
        wave_lds_sync();
      }
    }
  }
}

}  // namespace

extern "C" {

// Queue one launch writing ntiles x 2048 uint32 words of `out` (device
// memory of at least that size, 16-byte aligned) with the evaluator's tile
// pattern; flags bit 0 selects non-temporal stores, bits 1-2 the form (0:
// 4-byte stores, 1: 16-byte stores, 2: 4-byte rows turned into 16-byte
// stores through LDS, 3: form 0 in runs of `run` tiles per wave, run >= 1).
// Returns 0, or a HIP error code.
int fbg_probe_store_tiles(uint32_t *out, uint64_t ntiles, int32_t blocks, int32_t flags, uint32_t run,
                          void *stream) {
  if (!out || blocks <= 0 || flags < 0 || flags > 7 || run == 0 || ((uintptr_t)out & 15u))
    return (int)hipErrorInvalidValue;
  const dim3 g((unsigned)blocks), b(256);
  hipStream_t s = (hipStream_t)stream;
  switch (flags) {
    case 0: hipLaunchKernelGGL((k_store_tiles<false, 0>), g, b, 0, s, out, ntiles, run); break;
    case 1: hipLaunchKernelGGL((k_store_tiles<true, 0>), g, b, 0, s, out, ntiles, run); break;
    case 2: hipLaunchKernelGGL((k_store_tiles<false, 1>), g, b, 0, s, out, ntiles, run); break;
    case 3: hipLaunchKernelGGL((k_store_tiles<true, 1>), g, b, 0, s, out, ntiles, run); break;
    case 4: hipLaunchKernelGGL((k_store_tiles<false, 2>), g, b, 0, s, out, ntiles, run); break;
    case 5: hipLaunchKernelGGL((k_store_tiles<true, 2>), g, b, 0, s, out, ntiles, run); break;
    case 6: hipLaunchKernelGGL((k_store_tiles<false, 3>), g, b, 0, s, out, ntiles, run); break;
    default: hipLaunchKernelGGL((k_store_tiles<true, 3>), g, b, 0, s, out, ntiles, run); break;
  }
  return (int)hipGetLastError();
}


// Queue one launch of `blocks` x 256 threads, each issuing 64 * iters
// v_bitop3_b32; `out` holds blocks * 256 uint32 words (device memory).
// Returns 0, or the HIP error code of the launch.
int fbg_probe_valu_peak(uint32_t *out, int32_t blocks, uint32_t iters, uint32_t seed, void *stream) {
  if (!out || blocks <= 0) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_valu_peak, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, out, iters, seed);
  return (int)hipGetLastError();
}

}  // extern "C"
