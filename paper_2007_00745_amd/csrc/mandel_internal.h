// Host-side helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mandel.h"
#include "render_kernels.h"

namespace mandel {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void clear_error();
int workspace_head(hipStream_t s, unsigned long long **head);
int workspace_order(void *stream, uint32_t **hist);
int device_cus(int *cus);
int64_t tile_count(int32_t m, int32_t n, int32_t tw, int32_t th);
int make_view(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter, double R,
              int32_t tile_w, int32_t tile_h, ViewDesc *d);
int check_sched(const mandel_sched *s, mandel_sched *o);
int tile_grid(const mandel_sched &s, bool batch, int64_t ntiles, dim3 *grid, dim3 *block);
int test_mode(const mandel_sched &s);
int32_t auto_tile_parts(int64_t ntiles, int64_t waves, int32_t tile_w, int32_t tile_h,
                        int32_t max_iter);

} // namespace mandel
