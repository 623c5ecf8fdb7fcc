// Tile ordering kernels for gfx950: probe features, the FP32 tile cost model
// (inference, and training by minibatch Adam), and the descending bucket
// order.  The order only decides when each tile is rendered; counts are
// unaffected (pixels are independent, paper Sec. II-A).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "costmodel.h"
#include "mandel.h"
#include "mandel_internal.h"

#pragma clang fp contract(off)

namespace mandel {

namespace {

constexpr int NF = MANDEL_FEATURES;   // 68
constexpr int NH = MANDEL_HIDDEN;     // 64
constexpr int OFF_MU = 0;
constexpr int OFF_ISD = NF;
constexpr int OFF_W1 = MANDEL_MLP_NORM;           // [NH][NF]
constexpr int OFF_B1 = OFF_W1 + NH * NF;
constexpr int OFF_W2 = OFF_B1 + NH;               // [NH][NH]
constexpr int OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH;
constexpr int OFF_B3 = OFF_W3 + NH;
static_assert(OFF_B3 + 1 == MANDEL_MLP_PARAMS, "parameter layout");
constexpr int NTRAIN = MANDEL_MLP_PARAMS - MANDEL_MLP_NORM; // 8641

// The view table is never written by these kernels: read as constant memory, a
// wave-uniform descriptor comes through the scalar cache into SGPRs.
typedef const __attribute__((address_space(4))) ViewDesc ConstViewDesc;

__device__ __forceinline__ int32_t find_view_b(ConstViewDesc *views, int32_t nviews, int64_t t)
{
    int32_t lo = 0, hi = nviews - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Probe cap of a view: min(max_iter, probe_cap) for probe_cap > 0; for probe_cap = -k
// (k >= 1) a share of the view's own limit, max(1, floor(max_iter / k)).
__device__ __forceinline__ int32_t probe_cap_of(int32_t max_iter, int32_t probe_cap)
{
    if (probe_cap > 0)
        return max_iter < probe_cap ? max_iter : probe_cap;
    const int32_t c = max_iter / -probe_cap;
    return c > 1 ? c : 1;
}

// ---- probe features: one wavefront per tile, one probe pixel per lane ------
constexpr int32_t PROBE_BLOCK = 16;  // updates per untested block
constexpr int32_t PROBE_REPLAYS = 2; // replays before a wave tests every update

__global__ void __launch_bounds__(256) features_kernel(const ViewDesc *views, int32_t nviews,
                                                       const RowRef *rows, int64_t ntiles,
                                                       int32_t tile_w, int32_t tile_h,
                                                       int32_t probe_cap, float *feat)
{
    // one tile per wavefront: t is the same in all 64 lanes
    const int64_t t = (int64_t)blockIdx.x * (blockDim.x / 64) +
                      (int64_t)__builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    if (t >= ntiles)
        return;
    const int lane = threadIdx.x & 63;
    ConstViewDesc *table = (ConstViewDesc *)views;
    const int32_t v = find_view_b(table, nviews, t);
    ConstViewDesc &vd = table[v];
    const int32_t lt = (int32_t)(t - vd.tile_off); // a plan has fewer than 2^31 tiles
    const int32_t ty = lt / vd.tiles_x;
    const int32_t tx = lt - ty * vd.tiles_x;
    const int32_t x0 = tx * tile_w, y0 = ty * tile_h;
    const int32_t w = vd.n - x0 < tile_w ? vd.n - x0 : tile_w;
    const int32_t h = vd.m - y0 < tile_h ? vd.m - y0 : tile_h;
    const int32_t r = lane >> 3, k = lane & 7;
    // probe pixel: column x0 + floor((k + 0.5) w / 8), row y0 + floor((r + 0.5) h / 8)
    const int32_t j = x0 + (int32_t)(((int64_t)(2 * k + 1) * w) / 16);
    const int32_t i = y0 + (int32_t)(((int64_t)(2 * r + 1) * h) / 16);
    const double offx = ((double)j + 0.5) - 0.5 * (double)vd.n;
    const double px = offx * vd.dx;
    const double cx = vd.cx0 + px;
    double cy;
    if (vd.rows_off >= 0) { // collapsed rows: the row's coordinate from the plan's table
        cy = rows[vd.rows_off + i].cy;
    } else {
        const double offy = ((double)i + 0.5) - 0.5 * (double)vd.m;
        const double py = offy * vd.dy;
        cy = vd.cy0 + py;
    }
    const int32_t cap = probe_cap_of(vd.max_iter, probe_cap);
    // min(count, cap) needs the tests of z_1 .. z_{cap-1} only: count >= cap gives cap.
    // The wave advances in blocks of up to PROBE_BLOCK updates.  While no lane has
    // escaped and every lane's |c| lies in the disk where an escaped orbit keeps
    // growing (the render's deferred-test condition), a block runs untested and one
    // test of its last state tells whether any of its states escaped.  If one did, the
    // whole wave returns to the block's first state and replays it with a test after
    // every update, which finds the first escape exactly.  After PROBE_REPLAYS replays
    // the wave tests every update until it is done.
    const double R2 = vd.R2;
    const bool safe = cx * cx + cy * cy <= vd.safe2;
    double x = 0.0, y = 0.0;
    int32_t cnt = cap;
    bool live = true;
    int32_t replays = __builtin_amdgcn_ballot_w64(!safe) != 0 ? PROBE_REPLAYS : 0;
    auto update = [&]() {
        const double xx = x * x;
        const double yy = y * y;
        const double tt = x * y;
        x = (xx - yy) + cx;
        y = __builtin_fma(2.0, tt, cy);
    };
    for (int32_t it = 0; it < cap - 1;) { // z_it formed and tested in every live lane
        const int32_t L = cap - 1 - it < PROBE_BLOCK ? cap - 1 - it : PROBE_BLOCK;
        if (replays < PROBE_REPLAYS) {
            const double xs = x, ys = y;
            if (L == PROBE_BLOCK) {
#pragma unroll
                for (int32_t u = 0; u < PROBE_BLOCK; ++u)
                    update();
            } else {
                for (int32_t u = 0; u < L; ++u)
                    update();
            }
            const bool esc = live && !(x * x + y * y <= R2);
            if (__builtin_amdgcn_ballot_w64(esc) == 0) {
                it += L;
                continue;
            }
            x = xs;
            y = ys;
            ++replays;
        }
        for (int32_t u = 1; u <= L; ++u) { // form z_{it+u}, then test it
            update();
            const bool esc = live && x * x + y * y > R2;
            cnt = esc ? it + u : cnt;
            live = live && !esc;
        }
        it += L;
        if (__builtin_amdgcn_ballot_w64(live) == 0)
            break;
    }
    float *f = feat + t * NF;
    f[4 + lane] = logf(1.0f + (float)cnt) / logf(1.0f + (float)cap);
    if (lane < 4) {
        float val;
        if (lane == 0)
            val = (float)(vd.cx0 +
                          (((double)x0 + 0.5 * (double)w) - 0.5 * (double)vd.n) * vd.dx);
        else if (lane == 1)
            val = (float)(vd.rows_off >= 0
                              ? rows[vd.rows_off + y0 + h / 2].cy
                              : vd.cy0 + (((double)y0 + 0.5 * (double)h) - 0.5 * (double)vd.m) *
                                             vd.dy);
        else if (lane == 2)
            val = log10f((float)((double)w * vd.dx));
        else
            val = logf((float)vd.max_iter);
        f[lane] = val;
    }
}

// ---- probe-sum heuristic key: ln(1 + sum of the (capped) probe counts) ------
__global__ void probe_key_kernel(const float *feat, int64_t n, int32_t probe_cap, float *keys)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n)
        return;
    const float *f = feat + t * NF;
    const float cap = (float)probe_cap_of((int32_t)rintf(expf(f[3])), probe_cap);
    const float L = logf(1.0f + cap);
    float s = 0.0f;
    for (int k = 0; k < 64; ++k)
        s += expf(f[4 + k] * L) - 1.0f;
    keys[t] = logf(1.0f + s);
}

// ---- MLP inference on the matrix cores ---------------------------------------
// The two hidden layers are dense contractions over 16-row blocks of tiles:
//   H1[16 x 64] = relu(Xs[16 x 68] W1^T + b1),  H2[16 x 64] = relu(H1 W2^T + b2),
// each computed as 4 column blocks of 16 with v_mfma_f32_16x16x4_f32 (FP32 inputs,
// FP32 accumulation).  Operand layouts of that instruction (wave64): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16] of one K = 4 step, and the result
// D[4 (l / 16) + r][l % 16] in accumulator register r.  H1 passes through LDS to
// change from the result layout to the operand layout.  The output layer is a dot
// product per row, summed over the 16 lanes that hold the row's columns.
typedef float mf4 __attribute__((ext_vector_type(4)));

constexpr int MLP_ROWS = 16;          // rows per wave and block step
constexpr int MLP_WAVES = 4;          // wavefronts per workgroup
constexpr int H_STRIDE = NH + 4;      // LDS row stride of H1 (bank spread)

__global__ void __launch_bounds__(256) mlp_forward_kernel(const float *params, const float *x,
                                                          int64_t n, float *y)
{
    __shared__ float P[MANDEL_MLP_PARAMS];
    __shared__ float H[MLP_WAVES][MLP_ROWS * H_STRIDE];
    for (int q = threadIdx.x; q < MANDEL_MLP_PARAMS; q += blockDim.x)
        P[q] = params[q];
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int lr = l & 15;  // operand row (A) / column (B, D) of this lane
    const int lk = l >> 4;  // operand K index within a step (A, B); row group (D)
    float *Hw = H[w];
    const int64_t groups = (n + MLP_ROWS - 1) / MLP_ROWS;
    for (int64_t g = (int64_t)blockIdx.x * MLP_WAVES + w; g < groups;
         g += (int64_t)gridDim.x * MLP_WAVES) {
        const int64_t row0 = g * MLP_ROWS;
        const int64_t arow = row0 + lr;
        const bool aok = arow < n;
        const float *xr = x + (aok ? arow : 0) * NF;
        // layer 1
        mf4 acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const float b = P[OFF_B1 + 16 * nb + lr];
            acc[nb] = mf4{b, b, b, b};
        }
#pragma unroll
        for (int st = 0; st < NF / 4; ++st) {
            const int k = 4 * st + lk;
            const float a = aok ? (xr[k] - P[OFF_MU + k]) * P[OFF_ISD + k] : 0.0f;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                    a, P[OFF_W1 + (16 * nb + lr) * NF + k], acc[nb], 0, 0, 0);
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Hw[(4 * lk + r) * H_STRIDE + 16 * nb + lr] = fmaxf(acc[nb][r], 0.0f);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // layer 2
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const float b = P[OFF_B2 + 16 * nb + lr];
            acc[nb] = mf4{b, b, b, b};
        }
#pragma unroll
        for (int st = 0; st < NH / 4; ++st) {
            const int k = 4 * st + lk;
            const float a = Hw[lr * H_STRIDE + k];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                    a, P[OFF_W2 + (16 * nb + lr) * NH + k], acc[nb], 0, 0, 0);
        }
        // output layer: row 4 lk + r gets sum over columns j of w3[j] relu(H2[row][j])
        float part[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s = 0.0f;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                s = fmaf(P[OFF_W3 + 16 * nb + lr], fmaxf(acc[nb][r], 0.0f), s);
            part[r] = s;
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                part[r] += __shfl_xor(part[r], off, 16);
        if (lr == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + 4 * lk + r;
                if (row < n)
                    y[row] = P[OFF_B3] + part[r];
            }
        }
        // H1 of this block is read; the next block may overwrite it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---- MLP training ------------------------------------------------------------
// work layout (floats): A1[B][64] | A2[B][64] | gy[B] | err[B] | gA1[B][64] | gA2[B][64]
//                       | partial[GSLICES][NTRAIN]
constexpr int GSLICES = 16; // the minibatch is split into this many slices for gradient sums

__device__ __forceinline__ float lane_value(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ float wave_sum_f(float v)
{
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// One wavefront per sample, lane o = hidden unit o: forward pass with saved
// pre-activations, output error, and backpropagation to both hidden layers.
__global__ void __launch_bounds__(256) train_fwd_bwd_kernel(const float *params, const float *x,
                                                            const float *target,
                                                            const int32_t *idx, int32_t B,
                                                            float *work)
{
    const int b = blockIdx.x * (blockDim.x / 64) + (threadIdx.x / 64);
    if (b >= B)
        return; // whole wavefronts leave together
    const int o = threadIdx.x & 63;
    float *A1 = work, *A2 = work + (size_t)B * NH, *gy = work + (size_t)2 * B * NH;
    float *err = gy + B;
    float *gA1 = work + (size_t)2 * B * NH + 2 * (size_t)B;
    float *gA2 = gA1 + (size_t)B * NH;
    const int64_t row = idx[b];
    const float *xr = x + row * NF;
    float a1 = params[OFF_B1 + o];
    for (int i = 0; i < NF; ++i) {
        const float xi = (xr[i] - params[OFF_MU + i]) * params[OFF_ISD + i];
        a1 = fmaf(params[OFF_W1 + o * NF + i], xi, a1);
    }
    const float h1 = fmaxf(a1, 0.0f);
    float a2 = params[OFF_B2 + o];
    for (int i = 0; i < NH; ++i)
        a2 = fmaf(params[OFF_W2 + o * NH + i], lane_value(h1, i), a2);
    const float w3o = params[OFF_W3 + o];
    const float y = params[OFF_B3] + wave_sum_f(w3o * fmaxf(a2, 0.0f));
    const float e = y - target[row];
    const float g = 2.0f * e / (float)B;
    const float ga2 = a2 > 0.0f ? g * w3o : 0.0f;
    float gh1 = 0.0f;
    for (int k = 0; k < NH; ++k)
        gh1 = fmaf(lane_value(ga2, k), params[OFF_W2 + k * NH + o], gh1);
    A1[(size_t)b * NH + o] = a1;
    A2[(size_t)b * NH + o] = a2;
    gA2[(size_t)b * NH + o] = ga2;
    gA1[(size_t)b * NH + o] = a1 > 0.0f ? gh1 : 0.0f;
    if (o == 0) {
        gy[b] = g;
        err[b] = e * e;
    }
}

// Partial gradient of trainable parameter j over slice blockIdx.y of the minibatch.
__global__ void __launch_bounds__(256) train_grad_partial_kernel(const float *params,
                                                                 const float *x,
                                                                 const int32_t *idx, int32_t B,
                                                                 float *work)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NTRAIN)
        return;
    const int sl = blockIdx.y;
    const int per = (B + GSLICES - 1) / GSLICES;
    const int b0 = sl * per, b1 = b0 + per < B ? b0 + per : B;
    const float *A1 = work, *A2 = work + (size_t)B * NH, *gy = work + (size_t)2 * B * NH;
    const float *gA1 = work + (size_t)2 * B * NH + 2 * (size_t)B;
    const float *gA2 = gA1 + (size_t)B * NH;
    float *partial = work + (size_t)4 * B * NH + 2 * (size_t)B;
    const int p = MANDEL_MLP_NORM + j;
    float g = 0.0f;
    if (p < OFF_B1) { // W1[o][i]
        const int o = (p - OFF_W1) / NF, i = (p - OFF_W1) % NF;
        const float mu = params[OFF_MU + i], isd = params[OFF_ISD + i];
        for (int b = b0; b < b1; ++b) {
            const float xi = (x[(int64_t)idx[b] * NF + i] - mu) * isd;
            g = fmaf(gA1[(size_t)b * NH + o], xi, g);
        }
    } else if (p < OFF_W2) { // b1[o]
        const int o = p - OFF_B1;
        for (int b = b0; b < b1; ++b)
            g += gA1[(size_t)b * NH + o];
    } else if (p < OFF_B2) { // W2[o][i]
        const int o = (p - OFF_W2) / NH, i = (p - OFF_W2) % NH;
        for (int b = b0; b < b1; ++b)
            g = fmaf(gA2[(size_t)b * NH + o], fmaxf(A1[(size_t)b * NH + i], 0.0f), g);
    } else if (p < OFF_W3) { // b2[o]
        const int o = p - OFF_B2;
        for (int b = b0; b < b1; ++b)
            g += gA2[(size_t)b * NH + o];
    } else if (p < OFF_B3) { // w3[o]
        const int o = p - OFF_W3;
        for (int b = b0; b < b1; ++b)
            g = fmaf(gy[b], fmaxf(A2[(size_t)b * NH + o], 0.0f), g);
    } else { // b3
        for (int b = b0; b < b1; ++b)
            g += gy[b];
    }
    partial[(size_t)sl * NTRAIN + j] = g;
}

// Sum of the slice partials, then Adam (Kingma & Ba): moments, bias correction,
// step.  Gradients were formed from saved activations before any update.
__global__ void __launch_bounds__(256) train_adam_kernel(float *params, float *m, float *v,
                                                         int32_t B, const float *work, float lr,
                                                         float bc1, float bc2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NTRAIN)
        return;
    const float *partial = work + (size_t)4 * B * NH + 2 * (size_t)B;
    float g = 0.0f;
    for (int sl = 0; sl < GSLICES; ++sl)
        g += partial[(size_t)sl * NTRAIN + j];
    const int p = MANDEL_MLP_NORM + j;
    const float mj = 0.9f * m[p] + 0.1f * g;
    const float vj = 0.999f * v[p] + 0.001f * g * g;
    m[p] = mj;
    v[p] = vj;
    const float mh = mj / bc1;
    const float vh = vj / bc2;
    params[p] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

__global__ void __launch_bounds__(256) train_loss_kernel(int32_t B, const float *work, float *loss)
{
    __shared__ float red[256];
    const float *err = work + (size_t)2 * B * NH + B;
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += blockDim.x)
        s += err[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *loss = red[0] / (float)B;
}

// ---- standardisation and targets ---------------------------------------------------
// One block per feature column: mean and (population) standard deviation.
__global__ void __launch_bounds__(256) norm_kernel(float *params, const float *feat, int64_t n)
{
    __shared__ double red[2][256];
    const int c = blockIdx.x;
    double s = 0.0, s2 = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double v = (double)feat[r * NF + c];
        s += v;
        s2 += v * v;
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = red[0][0] / (double)n;
        double var = red[1][0] / (double)n - mu * mu;
        if (var < 0.0)
            var = 0.0;
        double sd = sqrt(var);
        if (sd < 1e-6)
            sd = 1e-6;
        params[OFF_MU + c] = (float)mu;
        params[OFF_ISD + c] = (float)(1.0 / sd);
    }
}

__global__ void targets_kernel(const int64_t *cost, int64_t n, float *target)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const int64_t c = cost[t] > 1 ? cost[t] : 1;
        target[t] = (float)log((double)c);
    }
}

// ---- descending bucket order ---------------------------------------------------
constexpr int NB = MANDEL_ORDER_BUCKETS;

__device__ __forceinline__ int bucket_of(float key)
{
    if (!(key == key))
        return NB - 1; // NaN: last
    // NB - 1 buckets for numbers (out-of-range keys clamp to the end ones), the
    // last bucket only for NaN
    const float u = (MANDEL_ORDER_KEY_HI - key) * ((float)(NB - 1) / (MANDEL_ORDER_KEY_HI - MANDEL_ORDER_KEY_LO));
    int b = (int)floorf(fminf(fmaxf(u, 0.0f), (float)(NB - 2)));
    return b;
}

__global__ void zero_u32_kernel(uint32_t *p, int n)
{
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x)
        p[q] = 0u;
}

// Runs f(bucket, lanes, leader) once per distinct bucket among the valid lanes of
// the wavefront (exec must be full): neighbouring tiles often share a bucket, and
// one atomic per distinct bucket avoids serialising on a single address.
template <typename F>
__device__ __forceinline__ void per_distinct_bucket(bool valid, int b, F &&f)
{
    uint64_t pending = __builtin_amdgcn_ballot_w64(valid);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int lb = __shfl(b, leader, 64);
        const uint64_t same = __builtin_amdgcn_ballot_w64(valid && b == lb) & pending;
        f(lb, same, leader);
        pending &= ~same;
    }
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ void __launch_bounds__(1024) hist_kernel(const float *keys, int64_t n, uint32_t *hist)
{
    __shared__ uint32_t h[NB];
    for (int q = threadIdx.x; q < NB; q += blockDim.x)
        h[q] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t start = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t t0 = start; t0 < n; t0 += stride) { // wave-uniform trip count
        const int64_t t = t0 + lane;
        const bool valid = t < n;
        const int b = valid ? bucket_of(keys[t]) : 0;
        per_distinct_bucket(valid, b, [&](int lb, uint64_t same, int leader) {
            if (lane == leader)
                atomicAdd(&h[lb], (uint32_t)__popcll(same));
        });
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NB; q += blockDim.x)
        if (h[q])
            atomicAdd(&hist[q], h[q]);
}

// exclusive scan of hist[0..NB) into cursor[0..NB) (one block of 1024 threads)
__global__ void __launch_bounds__(1024) scan_kernel(const uint32_t *hist, uint32_t *cursor)
{
    __shared__ uint32_t part[1024];
    constexpr int PER = NB / 1024;
    const int t = threadIdx.x;
    uint32_t loc[PER];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        loc[k] = s;
        s += hist[t * PER + k];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    const uint32_t base = part[t] - s; // exclusive prefix of this thread's chunk
#pragma unroll
    for (int k = 0; k < PER; ++k)
        cursor[t * PER + k] = base + loc[k];
}

// Positions: each wavefront reserves, per distinct bucket, a range of the
// workgroup's count for that bucket (LDS atomics); after a barrier the first
// reserver of each bucket takes the workgroup's whole range from the global
// cursor (one global atomic per bucket per workgroup).
__global__ void __launch_bounds__(1024) scatter_kernel(const float *keys, int64_t n,
                                                       uint32_t *cursor, int32_t *perm)
{
    __shared__ uint32_t cnt[NB];
    __shared__ uint32_t base[NB];
    for (int q = threadIdx.x; q < NB; q += blockDim.x)
        cnt[q] = 0u;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = t < n;
    const int b = valid ? bucket_of(keys[t]) : 0;
    uint32_t my_off = 0;
    bool first = false;
    per_distinct_bucket(valid, b, [&](int lb, uint64_t same, int leader) {
        uint32_t off = 0;
        if (lane == leader)
            off = atomicAdd(&cnt[lb], (uint32_t)__popcll(same));
        off = (uint32_t)__shfl((int)off, leader, 64);
        if ((same >> lane) & 1u)
            my_off = off + lanes_below(same);
        if (lane == leader && off == 0u)
            first = true;
    });
    __syncthreads();
    if (first)
        base[b] = atomicAdd(&cursor[b], cnt[b]);
    __syncthreads();
    if (valid)
        perm[base[b] + my_off] = (int32_t)t;
}

unsigned blocks_for(int64_t n, int threads, int64_t cap = 1 << 30)
{
    int64_t b = (n + threads - 1) / threads;
    if (b < 1)
        b = 1;
    if (b > cap)
        b = cap;
    return (unsigned)b;
}

} // namespace

hipError_t launch_features(const ViewDesc *views, int32_t nviews, const RowRef *rows,
                           int64_t ntiles, int32_t tile_w, int32_t tile_h, int32_t probe_cap,
                           float *feat, hipStream_t s)
{
    // one wavefront per workgroup: a wave whose probes finish early frees its slot at
    // once (with four per group the group held it until its slowest wave ended): the
    // 8192^2 view's 131 072 tiles 0.229 -> 0.177 ms, the uneven batch's 169 k tiles of
    // 128 x 16 unchanged (0.345 ms)
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(ntiles, 1)), dim3(64), 0, s, views,
                       nviews, rows, ntiles, tile_w, tile_h, probe_cap, feat);
    return hipGetLastError();
}

hipError_t launch_probe_key(const float *feat, int64_t n, int32_t probe_cap, float *keys,
                            hipStream_t s)
{
    hipLaunchKernelGGL(probe_key_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, feat, n,
                       probe_cap, keys);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, const float *x, int64_t n, float *y,
                              hipStream_t s)
{
    // each workgroup stages the parameters once and loops over 16-row blocks
    const int64_t groups = (n + MLP_ROWS - 1) / MLP_ROWS;
    int64_t blocks = (groups + MLP_WAVES - 1) / MLP_WAVES;
    if (blocks > 2048)
        blocks = 2048;
    if (blocks < 1)
        return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(64 * MLP_WAVES), 0, s,
                       params, x, n, y);
    return hipGetLastError();
}

hipError_t launch_order_desc(const float *keys, int64_t n, int32_t *perm, uint32_t *hist,
                             hipStream_t s)
{
    hipLaunchKernelGGL(zero_u32_kernel, dim3(8), dim3(1024), 0, s, hist, 2 * NB);
    hipLaunchKernelGGL(hist_kernel, dim3(blocks_for(n, 1024, 256)), dim3(1024), 0, s, keys, n,
                       hist);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, hist, hist + NB);
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(n, 1024)), dim3(1024), 0, s, keys, n,
                       hist + NB, perm);
    return hipGetLastError();
}

hipError_t launch_mlp_train_step(float *params, float *m, float *v, int32_t t, const float *x,
                                 const float *target, const int32_t *idx, int32_t B, float lr,
                                 float *loss, float *work, hipStream_t s)
{
    const double bc1 = 1.0 - std::pow(0.9, (double)t);
    const double bc2 = 1.0 - std::pow(0.999, (double)t);
    hipLaunchKernelGGL(train_fwd_bwd_kernel, dim3(blocks_for(B, 4)), dim3(256), 0, s, params, x,
                       target, idx, B, work);
    if (loss)
        hipLaunchKernelGGL(train_loss_kernel, dim3(1), dim3(256), 0, s, B, work, loss);
    hipLaunchKernelGGL(train_grad_partial_kernel, dim3(blocks_for(NTRAIN, 256), GSLICES),
                       dim3(256), 0, s, params, x, idx, B, work);
    hipLaunchKernelGGL(train_adam_kernel, dim3(blocks_for(NTRAIN, 256)), dim3(256), 0, s, params,
                       m, v, B, work, lr, (float)bc1, (float)bc2);
    return hipGetLastError();
}

} // namespace mandel

using namespace mandel;

extern "C" {

int mandel_mlp_forward(const float *params, const float *x, int64_t n, float *y, void *stream)
{
    clear_error();
    if (n < 0)
        return fail(MANDEL_EINVAL, "negative n");
    if (n == 0)
        return MANDEL_OK;
    if (!params || !x || !y)
        return fail(MANDEL_EINVAL, "null pointer");
    hipError_t e = launch_mlp_forward(params, x, n, y, (hipStream_t)stream);
    return e == hipSuccess ? MANDEL_OK : hip_fail(e, "mlp forward launch");
}

int64_t mandel_mlp_work_floats(int32_t batch)
{
    if (batch < 1)
        return 0;
    return (int64_t)batch * (4 * NH + 2) + (int64_t)GSLICES * NTRAIN;
}

int mandel_mlp_train_step(float *params, float *adam_m, float *adam_v, int32_t t, const float *x,
                          const float *target, const int32_t *idx, int32_t batch, float lr,
                          float *loss, float *work, void *stream)
{
    clear_error();
    if (!params || !adam_m || !adam_v || !x || !target || !idx || !work)
        return fail(MANDEL_EINVAL, "null pointer");
    if (batch < 1 || batch > 4096)
        return fail(MANDEL_EINVAL, "batch=%d outside [1, 4096]", batch);
    if (t < 1)
        return fail(MANDEL_EINVAL, "Adam step t=%d must be >= 1", t);
    if (!(lr > 0.0f) || !std::isfinite(lr))
        return fail(MANDEL_EINVAL, "lr must be finite and > 0");
    hipError_t e = launch_mlp_train_step(params, adam_m, adam_v, t, x, target, idx, batch, lr,
                                         loss, work, (hipStream_t)stream);
    return e == hipSuccess ? MANDEL_OK : hip_fail(e, "mlp train launch");
}

int mandel_mlp_set_norm(float *params, const float *feat, int64_t n, void *stream)
{
    clear_error();
    if (!params || !feat || n < 1)
        return fail(MANDEL_EINVAL, "need params, feat and n >= 1");
    hipLaunchKernelGGL(norm_kernel, dim3(NF), dim3(256), 0, (hipStream_t)stream, params, feat,
                       n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MANDEL_OK : hip_fail(e, "norm launch");
}

int mandel_cost_targets(const int64_t *cost, int64_t n, float *target, void *stream)
{
    clear_error();
    if (n < 0)
        return fail(MANDEL_EINVAL, "negative n");
    if (n == 0)
        return MANDEL_OK;
    if (!cost || !target)
        return fail(MANDEL_EINVAL, "null pointer");
    hipLaunchKernelGGL(targets_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       (hipStream_t)stream, cost, n, target);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MANDEL_OK : hip_fail(e, "targets launch");
}

int mandel_order_desc(const float *keys, int64_t n, int32_t *perm, void *stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31))
        return fail(MANDEL_EINVAL, "n=%lld outside [0, 2^31)", (long long)n);
    if (n == 0)
        return MANDEL_OK;
    if (!keys || !perm)
        return fail(MANDEL_EINVAL, "null pointer");
    uint32_t *hist = nullptr;
    int rc = workspace_order(stream, &hist);
    if (rc)
        return rc;
    hipError_t e = launch_order_desc(keys, n, perm, hist, (hipStream_t)stream);
    return e == hipSuccess ? MANDEL_OK : hip_fail(e, "order launch");
}

} // extern "C"
