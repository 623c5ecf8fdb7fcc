// The paper's output path: counts -> colours -> an image file written by one
// process (Sec. III: the master writes the set to a PPM file; Sec. I with
// Eq. (2): a pixel's colour is determined by its iteration count).
//
// Colouring is the Boolean escape-time rule: a pixel whose count reached
// max_iter (never escaped: taken to belong to the set) is black, every other
// pixel white.  The kernel is bound by HBM traffic: 4 bytes read and 3 written
// per pixel, moved 4 pixels per thread as one 16-byte load and three 4-byte
// stores when the buffers allow it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>

#include "output.h"

namespace mandel {

namespace {

__device__ __forceinline__ uint32_t colour_of(int32_t count, int32_t max_iter)
{
    return count >= max_iter ? 0u : 255u;
}

// Four pixels per thread: counts[4q .. 4q+3] -> rgb bytes [12q, 12q + 12).
__global__ void colour4_kernel(const int4 *__restrict__ counts, int64_t nquads, int32_t max_iter,
                               uint32_t *__restrict__ rgb_words)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nquads; q += stride) {
        const int4 c = counts[q];
        const uint32_t a = colour_of(c.x, max_iter), b = colour_of(c.y, max_iter);
        const uint32_t d = colour_of(c.z, max_iter), e = colour_of(c.w, max_iter);
        // bytes: a a a b | b b d d | d e e e   (little-endian words)
        rgb_words[3 * q + 0] = a | (a << 8) | (a << 16) | (b << 24);
        rgb_words[3 * q + 1] = b | (b << 8) | (d << 16) | (d << 24);
        rgb_words[3 * q + 2] = d | (e << 8) | (e << 16) | (e << 24);
    }
}

// One pixel per thread (any alignment, and the tail after the quads).
__global__ void colour1_kernel(const int32_t *__restrict__ counts, int64_t first, int64_t npix,
                               int32_t max_iter, uint8_t *__restrict__ rgb)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix;
         p += stride) {
        const uint8_t v = (uint8_t)colour_of(counts[p], max_iter);
        rgb[3 * p + 0] = v;
        rgb[3 * p + 1] = v;
        rgb[3 * p + 2] = v;
    }
}

unsigned grid_for(int64_t items)
{
    int64_t blocks = (items + 255) / 256;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 65536)
        blocks = 65536;
    return (unsigned)blocks;
}

} // namespace

hipError_t launch_colour(const int32_t *counts, int64_t npix, int32_t max_iter, uint8_t *rgb,
                         hipStream_t s)
{
    int64_t done = 0;
    const bool vec = ((uintptr_t)counts % 16 == 0) && ((uintptr_t)rgb % 4 == 0);
    if (vec && npix >= 4) {
        const int64_t nquads = npix / 4;
        hipLaunchKernelGGL(colour4_kernel, dim3(grid_for(nquads)), dim3(256), 0, s,
                           (const int4 *)counts, nquads, max_iter, (uint32_t *)rgb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        done = nquads * 4;
    }
    if (done < npix) {
        hipLaunchKernelGGL(colour1_kernel, dim3(grid_for(npix - done)), dim3(256), 0, s, counts,
                           done, npix, max_iter, rgb);
        return hipGetLastError();
    }
    return hipSuccess;
}

int write_ppm(const char *path, const uint8_t *rgb, int32_t m, int32_t n)
{
    FILE *f = std::fopen(path, "wb");
    if (!f)
        return -1;
    int ok = std::fprintf(f, "P6\n%d %d\n255\n", n, m) > 0;
    const size_t bytes = (size_t)m * (size_t)n * 3;
    if (ok && bytes)
        ok = std::fwrite(rgb, 1, bytes, f) == bytes;
    if (std::fclose(f) != 0)
        ok = 0;
    return ok ? 0 : -1;
}

} // namespace mandel
