// batch.hip -- the batched kernels' launches and occupancy queries: the
// persistent work-queue evaluator k_batch (counts; counts and DNF vectors),
// the direct batched DNF write-out k_batch_direct with k_sum_tile_counts,
// and the batched enumeration's k_list_tiles / k_batch_compact.
#define FBG_DEVICE_BATCH_KERNELS
#include "fbg_device.h"

namespace fbg {

namespace {

template <int VAR, int MODE>
hipError_t launch_batch_w(int log2w, const BatchArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  switch (log2w) {
    case 0: hipLaunchKernelGGL((dev::k_batch<0, VAR, MODE>), dim3(grid), dim3(block), lds, s, a); break;
    case 1: hipLaunchKernelGGL((dev::k_batch<1, VAR, MODE>), dim3(grid), dim3(block), lds, s, a); break;
    case 2: hipLaunchKernelGGL((dev::k_batch<2, VAR, MODE>), dim3(grid), dim3(block), lds, s, a); break;
    case 3: hipLaunchKernelGGL((dev::k_batch<3, VAR, MODE>), dim3(grid), dim3(block), lds, s, a); break;
    case 4: hipLaunchKernelGGL((dev::k_batch<4, VAR, MODE>), dim3(grid), dim3(block), lds, s, a); break;
    case 5: hipLaunchKernelGGL((dev::k_batch<5, VAR, MODE>), dim3(grid), dim3(block), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_batch_mode(int log2w, int var, const BatchArgs &a, int grid, int block, size_t lds,
                             hipStream_t s) {
  switch (var) {
    case 0: return launch_batch_w<0, MODE>(log2w, a, grid, block, lds, s);
    case 1: return launch_batch_w<1, MODE>(log2w, a, grid, block, lds, s);
    case 2: return launch_batch_w<2, MODE>(log2w, a, grid, block, lds, s);
    case 3: return launch_batch_w<3, MODE>(log2w, a, grid, block, lds, s);
  }
  return hipErrorInvalidValue;
}

int blocks_per_cu(const void *kernel, int block, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, lds) != hipSuccess || nb <= 0) nb = 1;
  return nb;
}

template <int VAR, int MODE>
int batch_occ_w(int log2w, int block, size_t lds) {
  switch (log2w) {
    case 0: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_batch<0, VAR, MODE>), block, lds);
    case 1: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_batch<1, VAR, MODE>), block, lds);
    case 2: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_batch<2, VAR, MODE>), block, lds);
    case 3: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_batch<3, VAR, MODE>), block, lds);
    case 4: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_batch<4, VAR, MODE>), block, lds);
    default: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_batch<5, VAR, MODE>), block, lds);
  }
}

template <int MODE>
int batch_occ_mode(int log2w, int var, int block, size_t lds) {
  switch (var) {
    case 0: return batch_occ_w<0, MODE>(log2w, block, lds);
    case 1: return batch_occ_w<1, MODE>(log2w, block, lds);
    case 2: return batch_occ_w<2, MODE>(log2w, block, lds);
    default: return batch_occ_w<3, MODE>(log2w, block, lds);
  }
}

}  // namespace

hipError_t launch_batch(int mode, int log2w, int var, const BatchArgs &a, int grid, int block, size_t lds,
                        hipStream_t s) {
  if (mode == dev::MODE_COUNT) return launch_batch_mode<dev::MODE_COUNT>(log2w, var, a, grid, block, lds, s);
  if (mode == dev::MODE_DNF) return launch_batch_mode<dev::MODE_DNF>(log2w, var, a, grid, block, lds, s);
  return hipErrorInvalidValue;
}

int batch_blocks_per_cu(int mode, int log2w, int var, int block, size_t lds) {
  if (mode == dev::MODE_DNF) return batch_occ_mode<dev::MODE_DNF>(log2w, var, block, lds);
  return batch_occ_mode<dev::MODE_COUNT>(log2w, var, block, lds);
}

hipError_t launch_batch_direct(int log2w, const BatchArgs &a, int grid, int block, int sum_blocks, hipStream_t s) {
  switch (log2w) {
    case 0: hipLaunchKernelGGL((dev::k_batch_direct<0>), dim3(grid), dim3(block), 0, s, a); break;
    case 1: hipLaunchKernelGGL((dev::k_batch_direct<1>), dim3(grid), dim3(block), 0, s, a); break;
    case 2: hipLaunchKernelGGL((dev::k_batch_direct<2>), dim3(grid), dim3(block), 0, s, a); break;
    case 3: hipLaunchKernelGGL((dev::k_batch_direct<3>), dim3(grid), dim3(block), 0, s, a); break;
    case 4: hipLaunchKernelGGL((dev::k_batch_direct<4>), dim3(grid), dim3(block), 0, s, a); break;
    case 5: hipLaunchKernelGGL((dev::k_batch_direct<5>), dim3(grid), dim3(block), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dev::k_sum_tile_counts, dim3(a.nitems, (unsigned)sum_blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_list_tiles(const BatchEnumArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(dev::k_list_tiles, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_compact(int log2w, const BatchEnumArgs &a, int grid, int block, hipStream_t s) {
  switch (log2w) {
    case 0: hipLaunchKernelGGL((dev::k_batch_compact<0>), dim3(grid), dim3(block), 0, s, a); break;
    case 1: hipLaunchKernelGGL((dev::k_batch_compact<1>), dim3(grid), dim3(block), 0, s, a); break;
    case 2: hipLaunchKernelGGL((dev::k_batch_compact<2>), dim3(grid), dim3(block), 0, s, a); break;
    case 3: hipLaunchKernelGGL((dev::k_batch_compact<3>), dim3(grid), dim3(block), 0, s, a); break;
    case 4: hipLaunchKernelGGL((dev::k_batch_compact<4>), dim3(grid), dim3(block), 0, s, a); break;
    case 5: hipLaunchKernelGGL((dev::k_batch_compact<5>), dim3(grid), dim3(block), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fbg
