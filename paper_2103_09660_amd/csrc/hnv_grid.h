// Launch geometry for grids of more blocks than one grid dimension holds.
// A dispatch counts each grid dimension in work-items with 32 bits, so a
// one-dimensional launch of 256-thread blocks must stay below 2^24 blocks.
// Larger launches fold their blocks into rows of kGridX blocks (gridDim.y
// rows); their kernels take linear_block() as the block index and return
// from the padding blocks at the end of the last row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hnv {

constexpr int64_t kGridX = int64_t(1) << 23;

inline dim3 fold_grid(int64_t blocks)
{
    if (blocks <= kGridX)
        return dim3((unsigned)blocks, 1, 1);
    return dim3((unsigned)kGridX, (unsigned)((blocks + kGridX - 1) / kGridX), 1);
}

__device__ __forceinline__ int64_t linear_block() { return (int64_t)blockIdx.y * gridDim.x + blockIdx.x; }

}  // namespace hnv
