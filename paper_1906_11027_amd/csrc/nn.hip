// nn.hip -- kernels of the learned warm start: a small convolutional net that
// maps droplet parameters plus a radial coordinate grid to the steady density
// field, trained and evaluated entirely on the GPU.
//
// Conventions: activations NCHW float32; weights [Cout][Cin][3][3] stored as
// bfloat16 for compute (FP32 master copy for the optimiser); every product
// accumulates in FP32.  Padding is circular (the droplet domain is periodic).
//
// conv3x3 forward: a block computes a 16 x 16 pixel tile of one image for all
// (<= 32) output channels; input channels stream through LDS in chunks of 8
// (an 18 x 18 halo tile per channel) together with the matching weights; each
// thread keeps its pixel's Cout accumulators in registers.  Backward-data is
// the same kernel applied to the channel-transposed, spatially flipped
// weights.  Backward-weight accumulates per-block partial sums over a fixed
// share of (tile, image) pairs (a 32 x 288 x 256 contraction per pair), then a
// column reduction sums the partials in a fixed order (deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sc_lbm.h"

namespace sclbm {
namespace nn {

constexpr int TS = 16;      // pixel tile side
constexpr int CCH = 8;      // input channels per LDS chunk
constexpr int MAXC = 32;    // largest channel count

__device__ __forceinline__ float bf16_to_f(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

__device__ __forceinline__ uint16_t f_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}

// v mod n for the halo coordinates of a tile: one add or subtract when v is
// within one period of [0, n), a full modulo otherwise (images narrower than
// the tile plus its halo)
__device__ __forceinline__ int wrapc(int v, int n)
{
    const int r = v < 0 ? v + n : (v >= n ? v - n : v);
    if (r >= 0 && r < n) return r;
    const int m = v % n;
    return m < 0 ? m + n : m;
}

template <int COUT>
__global__ void __launch_bounds__(TS* TS)
k_conv_fwd(const float* __restrict__ in, const uint16_t* __restrict__ w, const float* __restrict__ bias,
           float* __restrict__ out, int cin, int cout, int h, int wd)
{
    __shared__ float tile[CCH][TS + 2][TS + 3];
    __shared__ float ws[CCH][9][COUT];   // output channels contiguous: vector LDS reads
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TS + tx;
    const int tiles_x = (wd + TS - 1) / TS;
    const int x0 = (blockIdx.x % tiles_x) * TS, y0 = (blockIdx.x / tiles_x) * TS;
    const int b = blockIdx.y;
    const int64_t plane = (int64_t)h * wd;
    const float* inb = in + (int64_t)b * cin * plane;
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = (co < cout && bias) ? bias[co] : 0.f;
    for (int c0 = 0; c0 < cin; c0 += CCH) {
        const int nc = cin - c0 < CCH ? cin - c0 : CCH;
        for (int i = tid; i < CCH * (TS + 2) * (TS + 2); i += TS * TS) {
            const int c = i / ((TS + 2) * (TS + 2));
            const int r = i % ((TS + 2) * (TS + 2));
            const int ly = r / (TS + 2), lx = r % (TS + 2);
            float v = 0.f;
            if (c < nc) {
                const int gy = wrapc(y0 + ly - 1, h), gx = wrapc(x0 + lx - 1, wd);
                v = inb[(int64_t)(c0 + c) * plane + (int64_t)gy * wd + gx];
            }
            tile[c][ly][lx] = v;
        }
        for (int i = tid; i < COUT * CCH * 9; i += TS * TS) {
            const int co = i / (CCH * 9), r = i % (CCH * 9), c = r / 9, k = r % 9;
            ws[c][k][co] = (co < cout && c < nc) ? bf16_to_f(w[((int64_t)co * cin + c0 + c) * 9 + k]) : 0.f;
        }
        __syncthreads();
        for (int c = 0; c < nc; ++c) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float v = tile[c][ty + k / 3][tx + k % 3];
#pragma unroll
                for (int co = 0; co < COUT; ++co) acc[co] += ws[c][k][co] * v;
            }
        }
        __syncthreads();
    }
    const int x = x0 + tx, y = y0 + ty;
    if (x < wd && y < h) {
        float* ob = out + (int64_t)b * cout * plane + (int64_t)y * wd + x;
#pragma unroll
        for (int co = 0; co < COUT; ++co)
            if (co < cout) ob[(int64_t)co * plane] = acc[co];
    }
}

// wt[ci][co][8 - k] = w[co][ci][k]
__global__ void k_transpose_flip(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt, int cin, int cout)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cin * cout * 9) return;
    const int co = i / (cin * 9), r = i % (cin * 9), ci = r / 9, k = r % 9;
    wt[((int64_t)ci * cout + co) * 9 + (8 - k)] = w[i];
}

// partial[blk][(ci*cout + co)*9 + k] and partial[blk][E + co] (bias): the
// block's share of (tile, image) pairs.  Per pair the gradient is a small
// contraction over the tile's pixels p, gw[co][ci][k] += g[co][p] in[ci][p+k];
// thread (cog, ci) = (tid / 32, tid % 32) owns 4 output channels x 9 taps of
// one input channel, so each pixel costs 4 + 9 LDS reads for 36 FMAs.  The
// input tile holds every channel, one plane of 18 x 19 + 1 floats each (an
// odd stride: the 32 channels a half-wave reads sit in 32 different banks).
constexpr int TPL = (TS + 2) * (TS + 3) + 1;   // floats per input-channel plane in LDS

__global__ void __launch_bounds__(TS* TS)
k_conv_bwd_w(const float* __restrict__ in, const float* __restrict__ gout, float* __restrict__ partial, int batch,
             int cin, int cout, int h, int wd)
{
    __shared__ float tile[MAXC * TPL];
    __shared__ float gs[MAXC][TS * TS];
    const int tid = threadIdx.y * TS + threadIdx.x;
    const int ci = tid % MAXC, cog = tid / MAXC;   // 8 groups of 4 output channels
    const int tiles_x = (wd + TS - 1) / TS, tiles_y = (h + TS - 1) / TS;
    const int nwork = tiles_x * tiles_y * batch;
    const int64_t plane = (int64_t)h * wd;
    const int E = cout * cin * 9;
    float acc[4][9];
    float bacc = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[j][k] = 0.f;
    for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
        const int b = wi / (tiles_x * tiles_y), t = wi % (tiles_x * tiles_y);
        const int x0 = (t % tiles_x) * TS, y0 = (t / tiles_x) * TS;
        // output-gradient tile, every channel (zero outside the image and
        // for channels beyond cout)
        for (int i = tid; i < MAXC * TS * TS; i += TS * TS) {
            const int co = i / (TS * TS), p = i % (TS * TS);
            const int x = x0 + p % TS, y = y0 + p / TS;
            gs[co][p] = (co < cout && x < wd && y < h) ? gout[((int64_t)b * cout + co) * plane + (int64_t)y * wd + x]
                                                       : 0.f;
        }
        // input tile with a wrapped halo of one, every channel
        for (int i = tid; i < cin * (TS + 2) * (TS + 2); i += TS * TS) {
            const int c = i / ((TS + 2) * (TS + 2));
            const int r = i % ((TS + 2) * (TS + 2));
            const int ly = r / (TS + 2), lx = r % (TS + 2);
            const int gy = wrapc(y0 + ly - 1, h), gx = wrapc(x0 + lx - 1, wd);
            tile[c * TPL + ly * (TS + 3) + lx] = in[((int64_t)b * cin + c) * plane + (int64_t)gy * wd + gx];
        }
        __syncthreads();
        if (tid < cout) {
            float sb = 0.f;
            for (int p = 0; p < TS * TS; ++p) sb += gs[tid][p];
            bacc += sb;
        }
        if (ci < cin && cog * 4 < cout) {
            const float* tc = tile + ci * TPL;
            for (int py = 0; py < TS; ++py) {
#pragma unroll 4
                for (int px = 0; px < TS; ++px) {
                    const int p = py * TS + px;
                    float g[4], v[9];
#pragma unroll
                    for (int j = 0; j < 4; ++j) g[j] = gs[cog * 4 + j][p];
#pragma unroll
                    for (int k = 0; k < 9; ++k) v[k] = tc[(py + k / 3) * (TS + 3) + px + k % 3];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int k = 0; k < 9; ++k) acc[j][k] += g[j] * v[k];
                }
            }
        }
        __syncthreads();
    }
    float* pb = partial + (int64_t)blockIdx.x * (E + cout);
    if (ci < cin) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = cog * 4 + j;
            if (co < cout)
#pragma unroll
                for (int k = 0; k < 9; ++k) pb[(ci * cout + co) * 9 + k] = acc[j][k];
        }
    }
    if (tid < cout) pb[E + tid] = bacc;
}

// Sum the per-block partials in a fixed order: gw[co][ci][k] from the
// ci-major partial entries, gbias[co] from the trailing bias columns.  A block
// covers 64 columns with 4 row groups (rows r = g mod 4), combined in group
// order through LDS.
constexpr int kSumCols = 64, kSumGroups = 4;
__global__ void __launch_bounds__(kSumCols* kSumGroups)
k_sum_partials(const float* __restrict__ m, int nrow, int cin, int cout, float* __restrict__ gw,
               float* __restrict__ gbias)
{
    __shared__ float part[kSumGroups][kSumCols];
    const int E = cin * cout * 9;
    const int ncol = E + cout;
    const int lc = threadIdx.x % kSumCols, g = threadIdx.x / kSumCols;
    const int j = blockIdx.x * kSumCols + lc;
    float s = 0.f;
    if (j < ncol)
        for (int r = g; r < nrow; r += kSumGroups) s += m[(int64_t)r * ncol + j];
    part[g][lc] = s;
    __syncthreads();
    if (g != 0 || j >= ncol) return;
    s = ((part[0][lc] + part[1][lc]) + part[2][lc]) + part[3][lc];
    if (j < E) {
        const int ci = j / (cout * 9), rr = j % (cout * 9), co = rr / 9, k = rr % 9;
        gw[((int64_t)co * cin + ci) * 9 + k] = s;
    } else {
        gbias[j - E] = s;
    }
}

__global__ void k_tanh_fwd(float* __restrict__ x, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = tanhf(x[i]);
}

__global__ void k_tanh_bwd(const float* __restrict__ y, float* __restrict__ g, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        g[i] *= 1.f - y[i] * y[i];
}

// grad = 2 (out - tgt) / n; partial[blk] = sum (out - tgt)^2 over the block's share
__global__ void __launch_bounds__(256)
k_mse(const float* __restrict__ out, const float* __restrict__ tgt, float* __restrict__ grad, int64_t n,
      double* __restrict__ partial)
{
    __shared__ double red[4];
    double s = 0.0;
    const float scale = 2.f / (float)n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = out[i] - tgt[i];
        if (grad) grad[i] = scale * d;
        s += (double)d * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pb, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        if (pb) pb[i] = f_to_bf16(pi);
    }
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f_to_bf16(x[i]);
}

// Input features of image b: channel 0 the distance to the domain centre
// scaled by 1/scale_r, channels 1..4 the image's four (already normalised)
// parameters broadcast over the grid.
__global__ void k_features(const float* __restrict__ prm, float* __restrict__ out, int batch, int h, int wd,
                           float scale_r)
{
    const int64_t plane = (int64_t)h * wd;
    const int64_t total = plane * batch;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / plane);
        const int64_t p = i % plane;
        const int y = (int)(p / wd), x = (int)(p % wd);
        const float dx = (float)(x - wd / 2), dy = (float)(y - h / 2);
        float* ob = out + (int64_t)b * 5 * plane + p;
        // distance to the centre relative to the radius carried in params[b][0]
        ob[0] = sqrtf(dx * dx + dy * dy) / scale_r - prm[b * 4];
        for (int c = 0; c < 4; ++c) ob[(int64_t)(c + 1) * plane] = prm[b * 4 + c];
    }
}

// Initial field of a learned start, one workgroup per image (n x n):
// v = mean over the 8 symmetries of the square about node (c, c), c = n/2,
// of base + inv_scale * resid; clamp to [lo, hi]; then shift uniformly to
// the target mass.  Sums in double.
constexpr int kStartThreads = 1024;

__global__ void __launch_bounds__(kStartThreads)
k_start_field(const float* __restrict__ resid, const double* __restrict__ base, const double* __restrict__ mass,
              double* __restrict__ out, int n, float inv_scale, double lo, double hi)
{
    __shared__ double red[kStartThreads / 64];
    __shared__ double shift;
    const int64_t plane = (int64_t)n * n;
    const float* r = resid + blockIdx.x * plane;
    const double* bs = base + blockIdx.x * plane;
    double* o = out + blockIdx.x * plane;
    const int c2 = 2 * (n / 2);
    double acc = 0.0;
    for (int64_t p = threadIdx.x; p < plane; p += blockDim.x) {
        const int i = (int)(p / n), j = (int)(p % n);
        const int ii[2] = {i, (c2 - i + n) % n};
        const int jj[2] = {j, (c2 - j + n) % n};
        double v = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const int64_t q0 = (int64_t)ii[a] * n + jj[b];
                const int64_t q1 = (int64_t)jj[b] * n + ii[a];
                v += (bs[q0] + (double)(inv_scale * r[q0])) + (bs[q1] + (double)(inv_scale * r[q1]));
            }
        v *= 0.125;
        v = v < lo ? lo : (v > hi ? hi : v);
        o[p] = v;
        acc += v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kStartThreads / 64; ++k) t += red[k];
        shift = (mass[blockIdx.x] - t) / (double)plane;
    }
    __syncthreads();
    const double d = shift;
    for (int64_t p = threadIdx.x; p < plane; p += blockDim.x) o[p] += d;
}

static int grid_for(int64_t n)
{
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace nn
}  // namespace sclbm

using namespace sclbm::nn;

static int nn_status(hipError_t e) { return e == hipSuccess ? SC_OK : SC_E_DEVICE; }

static bool conv_shape_ok(int batch, int cin, int cout, int h, int w)
{
    return batch >= 1 && cin >= 1 && cin <= MAXC && (cout == 1 || cout == MAXC) && h >= 1 && w >= 1 &&
           batch <= 65535;
}

extern "C" int sc_nn_conv3x3_fwd(const float* in, const uint16_t* w, const float* bias, float* out, int32_t batch,
                                 int32_t cin, int32_t cout, int32_t h, int32_t wd, void* stream)
{
    if (!in || !w || !out || !conv_shape_ok(batch, cin, cout, h, wd)) return SC_E_INVAL;
    const int tiles = ((wd + TS - 1) / TS) * ((h + TS - 1) / TS);
    dim3 grid(tiles, batch), block(TS, TS);
    if (cout == MAXC)
        hipLaunchKernelGGL(k_conv_fwd<MAXC>, grid, block, 0, (hipStream_t)stream, in, w, bias, out, cin, cout, h, wd);
    else
        hipLaunchKernelGGL(k_conv_fwd<1>, grid, block, 0, (hipStream_t)stream, in, w, bias, out, cin, cout, h, wd);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_conv3x3_bwd_data(const float* gout, const uint16_t* w, uint16_t* wt_scratch, float* gin,
                                      int32_t batch, int32_t cin, int32_t cout, int32_t h, int32_t wd, void* stream)
{
    if (!gout || !w || !wt_scratch || !gin || !conv_shape_ok(batch, cin, cout, h, wd) || cin != MAXC)
        return SC_E_INVAL;
    const int nw = cin * cout * 9;
    hipLaunchKernelGGL(k_transpose_flip, (nw + 255) / 256, 256, 0, (hipStream_t)stream, w, wt_scratch, cin, cout);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nn_status(e);
    // gradient w.r.t. the input: convolution of gout (cout channels) with the
    // flipped, transposed weights (cin output channels), no bias
    return sc_nn_conv3x3_fwd(gout, wt_scratch, nullptr, gin, batch, cout, cin, h, wd, stream);
}

extern "C" int32_t sc_nn_bwd_weight_scratch_floats(int32_t cin, int32_t cout, int32_t nblk)
{
    return nblk * (cin * cout * 9 + cout);
}

extern "C" int sc_nn_conv3x3_bwd_weight(const float* in, const float* gout, float* partial_scratch, int32_t nblk,
                                        float* gw, float* gbias, int32_t batch, int32_t cin, int32_t cout, int32_t h,
                                        int32_t wd, void* stream)
{
    if (!in || !gout || !partial_scratch || !gw || !gbias || nblk < 1 || !conv_shape_ok(batch, cin, cout, h, wd))
        return SC_E_INVAL;
    const int E = cin * cout * 9;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_conv_bwd_w, nblk, dim3(TS, TS), 0, s, in, gout, partial_scratch, batch, cin, cout, h, wd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nn_status(e);
    hipLaunchKernelGGL(k_sum_partials, (E + cout + kSumCols - 1) / kSumCols, kSumCols * kSumGroups, 0, s,
                       partial_scratch, nblk, cin, cout, gw, gbias);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_tanh_fwd(float* x, int64_t n, void* stream)
{
    if (!x || n < 0) return SC_E_INVAL;
    hipLaunchKernelGGL(k_tanh_fwd, grid_for(n), 256, 0, (hipStream_t)stream, x, n);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_tanh_bwd(const float* y, float* g, int64_t n, void* stream)
{
    if (!y || !g || n < 0) return SC_E_INVAL;
    hipLaunchKernelGGL(k_tanh_bwd, grid_for(n), 256, 0, (hipStream_t)stream, y, g, n);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_mse(const float* out, const float* tgt, float* grad, double* partial_scratch, int32_t nblk,
                         int64_t n, void* stream)
{
    if (!out || !tgt || !partial_scratch || nblk < 1 || n < 1) return SC_E_INVAL;
    hipLaunchKernelGGL(k_mse, nblk, 256, 0, (hipStream_t)stream, out, tgt, grad, n, partial_scratch);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_adam(float* p, const float* g, float* m, float* v, uint16_t* p_bf16, int64_t n, float lr,
                          float beta1, float beta2, float eps, int32_t t, void* stream)
{
    if (!p || !g || !m || !v || n < 0 || t < 1) return SC_E_INVAL;
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, grid_for(n), 256, 0, (hipStream_t)stream, p, g, m, v, p_bf16, n, lr, beta1, beta2,
                       eps, c1, c2);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_to_bf16(const float* x, uint16_t* y, int64_t n, void* stream)
{
    if (!x || !y || n < 0) return SC_E_INVAL;
    hipLaunchKernelGGL(k_to_bf16, grid_for(n), 256, 0, (hipStream_t)stream, x, y, n);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_features(const float* params, float* out, int32_t batch, int32_t h, int32_t wd, float scale_r,
                              void* stream)
{
    if (!params || !out || batch < 1 || h < 1 || wd < 1 || !(scale_r > 0.f)) return SC_E_INVAL;
    hipLaunchKernelGGL(k_features, grid_for((int64_t)batch * h * wd), 256, 0, (hipStream_t)stream, params, out, batch,
                       h, wd, scale_r);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_start_field(const float* resid, const double* base, const double* mass, double* out,
                                 int32_t batch, int32_t h, int32_t wd, float inv_scale, double lo, double hi,
                                 void* stream)
{
    if (!resid || !base || !mass || !out || batch < 1 || batch > 65535 || h < 1 || h != wd || !(lo <= hi) ||
        (int64_t)h * wd > ((int64_t)1 << 31))
        return SC_E_INVAL;
    hipLaunchKernelGGL(k_start_field, batch, kStartThreads, 0, (hipStream_t)stream, resid, base, mass, out, h,
                       inv_scale, lo, hi);
    return nn_status(hipGetLastError());
}
