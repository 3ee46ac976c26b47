// XCD-aware tile order for the stencil kernels on gfx950.
#pragma once
#include <hip/hip_runtime.h>

namespace shk {

// Tile coordinates of this workgroup under an XCD-aware permutation of the
// launch grid.  Workgroups are handed to the eight XCDs round-robin by linear
// id, so XCD x receives ids x, x + 8, ...; mapping the k-th of them to tile
// start_x + k gives every XCD one contiguous run of tiles (rows of tiles),
// and the halo rows a tile shares with its neighbours are then mostly read
// through the same L2.  The map is a bijection for any grid size, so
// correctness does not depend on how the hardware actually dispatches.
__device__ __forceinline__ void xcd_tile(int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int n = gx * gy * gridDim.z;
  const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int q = n >> 3, r = n & 7;
  const int x = lin & 7, k = lin >> 3;
  const int t = x * q + (x < r ? x : r) + k;
  bx = t % gx;
  const int rest = t / gx;
  by = rest % gy;
  bz = rest / gy;
}

}  // namespace shk
