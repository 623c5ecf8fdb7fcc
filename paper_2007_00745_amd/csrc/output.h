// Output path: Boolean colouring kernel and the PPM writer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mandel {

hipError_t launch_colour(const int32_t *counts, int64_t npix, int32_t max_iter, uint8_t *rgb,
                         hipStream_t s);
// 0 on success, -1 on an I/O error.
int write_ppm(const char *path, const uint8_t *rgb, int32_t m, int32_t n);

} // namespace mandel
