// eval_dnf.hip -- the single-program evaluator kernels of the DNF write-out:
// k_eval<W, MODE_DNF, VAR> for every tiling and variant, their launches and
// occupancy queries.
#include "fbg_device.h"

namespace fbg {

namespace {

template <int MODE, int VAR>
hipError_t launch_w(int log2w, const EvalArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  switch (log2w) {
    case 0: hipLaunchKernelGGL((dev::k_eval<0, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 1: hipLaunchKernelGGL((dev::k_eval<1, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 2: hipLaunchKernelGGL((dev::k_eval<2, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 3: hipLaunchKernelGGL((dev::k_eval<3, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 4: hipLaunchKernelGGL((dev::k_eval<4, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    case 5: hipLaunchKernelGGL((dev::k_eval<5, MODE, VAR>), dim3(grid), dim3(block), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  switch (var) {
    case 0: return launch_w<MODE, 0>(log2w, a, grid, block, lds, s);
    case 1: return launch_w<MODE, 1>(log2w, a, grid, block, lds, s);
    case 2: return launch_w<MODE, 2>(log2w, a, grid, block, lds, s);
    case 3: return launch_w<MODE, 3>(log2w, a, grid, block, lds, s);
  }
  return hipErrorInvalidValue;
}

int blocks_per_cu(const void *kernel, int block, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, lds) != hipSuccess || nb <= 0) nb = 1;
  return nb;
}

template <int MODE, int VAR>
int occ_w(int log2w, int block, size_t lds) {
  switch (log2w) {
    case 0: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_eval<0, MODE, VAR>), block, lds);
    case 1: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_eval<1, MODE, VAR>), block, lds);
    case 2: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_eval<2, MODE, VAR>), block, lds);
    case 3: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_eval<3, MODE, VAR>), block, lds);
    case 4: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_eval<4, MODE, VAR>), block, lds);
    default: return blocks_per_cu(reinterpret_cast<const void *>(&dev::k_eval<5, MODE, VAR>), block, lds);
  }
}

template <int MODE>
int occ_mode(int log2w, int var, int block, size_t lds) {
  switch (var) {
    case 0: return occ_w<MODE, 0>(log2w, block, lds);
    case 1: return occ_w<MODE, 1>(log2w, block, lds);
    case 2: return occ_w<MODE, 2>(log2w, block, lds);
    default: return occ_w<MODE, 3>(log2w, block, lds);
  }
}

}  // namespace

hipError_t launch_eval_dnf(int log2w, int var, const EvalArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  return launch_mode<dev::MODE_DNF>(log2w, var, a, grid, block, lds, s);
}

int eval_occ_dnf(int log2w, int var, int block, size_t lds) { return occ_mode<dev::MODE_DNF>(log2w, var, block, lds); }

}  // namespace fbg
