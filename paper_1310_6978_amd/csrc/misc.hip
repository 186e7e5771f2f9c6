// misc.hip -- launches of the small kernels (stored-DNF scans, the exclusive
// scan of per-tile counts, fills) and the per-mode dispatch of the
// single-program evaluator (its kernels live in eval_*.hip).
#define FBG_DEVICE_MISC_KERNELS
#include "fbg_device.h"

namespace fbg {

hipError_t launch_eval_count(int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds, hipStream_t s);
hipError_t launch_eval_dnf(int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds, hipStream_t s);
hipError_t launch_eval_enum(int mode, int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds,
                            hipStream_t s);
int eval_occ_count(int log2w, int var, int block, size_t lds);
int eval_occ_dnf(int log2w, int var, int block, size_t lds);
int eval_occ_enum(int mode, int log2w, int var, int block, size_t lds);

hipError_t launch_eval(int mode, int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds,
                       hipStream_t s) {
  switch (mode) {
    case dev::MODE_COUNT: return launch_eval_count(log2w, var, a, grid, block, lds, s);
    case dev::MODE_DNF: return launch_eval_dnf(log2w, var, a, grid, block, lds, s);
    case dev::MODE_TILECNT:
    case dev::MODE_ENUM: return launch_eval_enum(mode, log2w, var, a, grid, block, lds, s);
  }
  return hipErrorInvalidValue;
}

int eval_blocks_per_cu(int mode, int log2w, int var, int block, size_t lds) {
  switch (mode) {
    case dev::MODE_COUNT: return eval_occ_count(log2w, var, block, lds);
    case dev::MODE_DNF: return eval_occ_dnf(log2w, var, block, lds);
    default: return eval_occ_enum(mode, log2w, var, block, lds);
  }
}

hipError_t launch_dnf_scan(int mode, const EvalArgs &a, int grid, int block, hipStream_t s) {
  if (mode == dev::MODE_TILECNT)
    hipLaunchKernelGGL((dev::k_dnf_scan<dev::MODE_TILECNT>), dim3(grid), dim3(block), 0, s, a);
  else if (mode == dev::MODE_ENUM)
    hipLaunchKernelGGL((dev::k_dnf_scan<dev::MODE_ENUM>), dim3(grid), dim3(block), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *block_sums, uint64_t *total,
                       hipStream_t s) {
  const uint64_t nb = (n + dev::SCAN_BLOCK - 1) / dev::SCAN_BLOCK;
  if (nb == 0) {
    hipLaunchKernelGGL(dev::k_set_u64, dim3(1), dim3(64), 0, s, total, (uint64_t)0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(dev::k_scan_reduce, dim3((unsigned)nb), dim3(dev::SCAN_THREADS), 0, s, in, n, block_sums);
  hipLaunchKernelGGL(dev::k_scan_sums, dim3(1), dim3(dev::SCAN_THREADS), 0, s, block_sums, nb, total);
  hipLaunchKernelGGL(dev::k_scan_apply, dim3((unsigned)nb), dim3(dev::SCAN_THREADS), 0, s, in, n, block_sums, out);
  return hipGetLastError();
}

uint64_t scan_block_count(uint64_t n) { return (n + dev::SCAN_BLOCK - 1) / dev::SCAN_BLOCK; }

hipError_t launch_zero(uint64_t *p, uint64_t n, uint32_t *head, uint32_t nhead, hipStream_t s) {
  if (!head) nhead = 0;
  const uint64_t threads = std::max<uint64_t>(std::max<uint64_t>(n, nhead), 1);
  const unsigned grid = (unsigned)((threads + 255) / 256);
  hipLaunchKernelGGL(dev::k_zero_u64, dim3(grid), dim3(256), 0, s, p, n, head, nhead);
  return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t *p, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(dev::k_set_u64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace fbg
