// Host launchers of the tile-ordering kernels: probe features, the FP32 cost
// model (inference and training), and the descending bucket order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "render_kernels.h"

namespace mandel {

hipError_t launch_features(const ViewDesc *views, int32_t nviews, const RowRef *rows,
                           int64_t ntiles, int32_t tile_w, int32_t tile_h, int32_t probe_cap,
                           float *feat, hipStream_t s);
hipError_t launch_probe_key(const float *feat, int64_t ntiles, int32_t probe_cap, float *keys,
                            hipStream_t s);
hipError_t launch_mlp_forward(const float *params, const float *x, int64_t n, float *y,
                              hipStream_t s);
// hist: device uint32[2 * MANDEL_ORDER_BUCKETS] scratch
hipError_t launch_order_desc(const float *keys, int64_t n, int32_t *perm, uint32_t *hist,
                             hipStream_t s);
hipError_t launch_mlp_train_step(float *params, float *m, float *v, int32_t t, const float *x,
                                 const float *target, const int32_t *idx, int32_t batch,
                                 float lr, float *loss, float *work, hipStream_t s);

} // namespace mandel
