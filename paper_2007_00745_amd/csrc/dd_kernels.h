// Host/device declarations of the double-double render.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mandel {

struct DDArgs {
    double cx0h, cx0l, cy0h, cy0l; // double-double window centre
    double dx, dy;                 // pixel pitch
    double R2;                     // R*R, rounded once
    int32_t m, n, max_iter;
    int32_t tile_w, tile_h, tiles_x;
    int64_t ntiles;
    int32_t *out;                  // device int32[m*n], row-major
    unsigned long long *head;      // tile queue head (cleared before the launch)
    uint64_t *stats;               // optional: uint64[4] accumulated
};

hipError_t launch_render_dd(const DDArgs &a, dim3 grid, dim3 block, hipStream_t s);
int dd_blocks_per_cu(int threads);

} // namespace mandel
