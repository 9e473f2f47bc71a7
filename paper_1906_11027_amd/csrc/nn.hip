// nn.hip -- kernels of the learned warm start: a small convolutional net that
// maps droplet parameters plus a radial coordinate grid to the steady density
// field, trained and evaluated entirely on the GPU.
//
// Conventions: activations NCHW float32; weights [Cout][Cin][3][3] stored as
// bfloat16 for compute (FP32 master copy for the optimiser); every product
// accumulates in FP32.  Padding is circular (the droplet domain is periodic).
//
// The 3 x 3 convolutions are dense contractions and run on the matrix cores:
//   forward (32 output channels): per 16 x 16 pixel tile, out[p][co] =
//     sum over 9 taps of x_t[p][ci] W_t[ci][co], one 16 x 16 x 32 bf16 MFMA
//     per (16 pixels, 16 channels, tap).  The FP32 activations enter as the
//     exact sum of three bf16 parts (hi + mid + lo, 8 significant bits each),
//     so each product is the FP32 activation times the bf16 weight, exact,
//     accumulated in FP32 -- three MFMAs per product, the price of keeping the
//     activations in full FP32.
//   backward-data: the forward kernel on the channel-transposed, spatially
//     flipped weights.
//   backward-weight: gW_t[co][ci] = sum_p g[co][p] x[ci][p + d_t], a
//     contraction over pixels, on FP32 16 x 16 x 4 MFMAs (both operands FP32:
//     no splitting of the output gradient).  Per-block partial sums over a
//     fixed share of (tile, image) pairs, then a column reduction in a fixed
//     order (deterministic).
// The one-output-channel forward (the net's last layer) stays on the vector
// ALU: a 288-term dot product per pixel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sc_lbm.h"
#include "kernels.h"   // xcd_swizzle

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
    // XCD-aware order: the tiles one XCD runs together are neighbours, so
    // the cache lines two tiles share are fetched into one L2
    const int ntl = gridDim.x, L = xcd_swizzle(blockIdx.y * ntl + blockIdx.x, ntl * gridDim.y);
    const int tl = L % ntl, b = L / ntl;
    const int x0 = (tl % tiles_x) * TS, y0 = (tl / tiles_x) * TS;
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

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// exact split of an FP32 value into three bf16 parts, v = hi + mid + lo:
// each part truncates the remainder to its top 8 significant bits, and the
// remainders are exact differences, so 24 bits are carried in all
__device__ __forceinline__ void split3(float v, uint32_t& hi, uint32_t& mid, uint32_t& lo)
{
    const uint32_t u = __float_as_uint(v);
    const float r1 = v - __uint_as_float(u & 0xffff0000u);
    const uint32_t u1 = __float_as_uint(r1);
    const float r2 = r1 - __uint_as_float(u1 & 0xffff0000u);
    hi = u >> 16;
    mid = u1 >> 16;
    lo = __float_as_uint(r2) >> 16;
}

constexpr int kHaloPx = (TS + 2) * (TS + 2);   // pixels of a tile with its halo
constexpr int kPxSlot = 32;                     // bf16 per pixel (or weight row) in LDS: 64 B
constexpr int kPartBf = kHaloPx * kPxSlot;      // one bf16 part of the input tile

// LDS slot s holds 32 bf16 channels as four 16-byte chunks; chunk k is
// stored at position k ^ ((s >> 2) & 3).  A quarter-wave reads one chunk of
// 16 consecutive slots, which then fall on 16 distinct bank quads.
__device__ __forceinline__ int slot_chunk(int s, int k) { return (k ^ (s >> 2)) & 3; }

// Forward 3 x 3 convolution to 32 output channels on bf16 MFMAs.  A block
// (4 waves) takes (image, 16 x 16 tile) work items in turn; wave v computes
// tile rows 4v .. 4v+3.  LDS holds the input tile (halo 1, channels padded
// to 32 with zeros) as three bf16 parts, pixel-major with the channels
// contiguous, and the weights as [tap][co][ci] bf16, staged once per block
// (80,640 B in all: two blocks share a CU, so one stages while the other
// multiplies).  The tile's global loads are all issued before any is used:
// one round trip per tile.  MFMA operands (16 x 16 x 32):
// lane l supplies row or column l % 16 and the 8 consecutive k = 8 (l / 16)
// ...; its accumulator holds rows 4 (l / 16) + i, column l % 16.  Here rows
// are the pixels of a 16-pixel row segment, columns output channels and k
// input channels.
constexpr int kFwdStage = ((MAXC / 2) * kHaloPx + TS * TS - 1) / (TS * TS);   // staging loads per thread

// Epilogue applied to each output before it is stored (fusing the
// elementwise pass that would otherwise re-read the whole activation)
enum ConvEpi { kEpiNone = 0, kEpiTanh = 1, kEpiTanhGrad = 2 };

template <int EPI>
__device__ __forceinline__ float conv_epi(float v, const float* __restrict__ y, int64_t i)
{
    if (EPI == kEpiTanh) return tanhf(v);
    if (EPI == kEpiTanhGrad) {
        const float yv = y[i];
        return v * (1.f - yv * yv);
    }
    return v;
}

template <int EPI>
__global__ void __launch_bounds__(TS* TS, 2)
k_conv_fwd_mfma(const float* __restrict__ in, const uint16_t* __restrict__ w, const float* __restrict__ bias,
                float* __restrict__ out, const float* __restrict__ y, int batch, int cin, int h, int wd)
{
    __shared__ __align__(16) uint16_t xs[3 * kPartBf];
    __shared__ __align__(16) uint16_t wsl[9 * MAXC * kPxSlot];
    const int tid = threadIdx.y * TS + threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int tiles_x = (wd + TS - 1) / TS, tiles = tiles_x * ((h + TS - 1) / TS);
    const int nwork = tiles * batch;
    const int64_t plane = (int64_t)h * wd;

    for (int j = tid; j < 9 * MAXC * MAXC; j += TS * TS) {
        const int t = j >> 10, co = (j >> 5) & 31, ci = j & 31;
        const int sl = t * MAXC + co;
        wsl[sl * kPxSlot + slot_chunk(sl, ci >> 3) * 8 + (ci & 7)] =
            ci < cin ? w[((int64_t)co * cin + ci) * 9 + t] : (uint16_t)0;
    }
    float bv[2];
#pragma unroll
    for (int n = 0; n < 2; ++n) bv[n] = bias ? bias[n * 16 + r16] : 0.f;

    // XCD-aware order: at any time the blocks of one XCD hold neighbouring
    // tiles, so the cache lines two tiles share are fetched into one L2
    for (int wi = xcd_swizzle(blockIdx.x, gridDim.x); wi < nwork; wi += gridDim.x) {
        const int b = wi / tiles, tt = wi - b * tiles;
        const int x0 = (tt % tiles_x) * TS, y0 = (tt / tiles_x) * TS;
        const float* inb = in + (int64_t)b * cin * plane;
        float v0[kFwdStage], v1[kFwdStage];
#pragma unroll
        for (int q = 0; q < kFwdStage; ++q) {
            const int j = tid + q * TS * TS;
            v0[q] = v1[q] = 0.f;
            if (j < (MAXC / 2) * kHaloPx) {
                const int pr = j / kHaloPx, px = j - pr * kHaloPx;
                const int ly = px / (TS + 2), lx = px - ly * (TS + 2);
                // 32-bit element offsets within the image (checked on the host)
                const uint32_t g = (uint32_t)(wrapc(y0 + ly - 1, h) * wd + wrapc(x0 + lx - 1, wd));
                const uint32_t c = 2 * pr;
                if ((int)c < cin) v0[q] = inb[c * (uint32_t)plane + g];
                if ((int)c + 1 < cin) v1[q] = inb[(c + 1) * (uint32_t)plane + g];
            }
        }
        __syncthreads();   // the previous item's reads of xs are done
#pragma unroll
        for (int q = 0; q < kFwdStage; ++q) {
            const int j = tid + q * TS * TS;
            if (j < (MAXC / 2) * kHaloPx) {
                const int pr = j / kHaloPx, px = j - pr * kHaloPx;
                uint32_t h0, m0, l0, h1, m1, l1;
                split3(v0[q], h0, m0, l0);
                split3(v1[q], h1, m1, l1);
                uint32_t* d = (uint32_t*)(xs + px * kPxSlot + slot_chunk(px, pr >> 2) * 8 + 2 * (pr & 3));
                d[0] = h0 | (h1 << 16);
                d[kPartBf / 2] = m0 | (m1 << 16);
                d[kPartBf] = l0 | (l1 << 16);
            }
        }
        __syncthreads();

        f32x4 acc[4][2];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[r][n] = f32x4{bv[n], bv[n], bv[n], bv[n]};
#pragma unroll 1
        for (int t = 0; t < 9; ++t) {   // rolled: unrolled, the scheduler hoists too many LDS reads
            const int dy = t / 3, dx = t % 3;
            const int s0 = t * MAXC + r16, s1 = s0 + 16;
            const bf16x8 b0 = *(const bf16x8*)(wsl + s0 * kPxSlot + slot_chunk(s0, kq) * 8);
            const bf16x8 b1 = *(const bf16x8*)(wsl + s1 * kPxSlot + slot_chunk(s1, kq) * 8);
#pragma unroll
            for (int part = 0; part < 3; ++part)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int px = (4 * wv + r + dy) * (TS + 2) + r16 + dx;
                    const bf16x8 a = *(const bf16x8*)(xs + part * kPartBf + px * kPxSlot + slot_chunk(px, kq) * 8);
                    acc[r][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc[r][0], 0, 0, 0);
                    acc[r][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc[r][1], 0, 0, 0);
                }
        }
        const int xq = x0 + 4 * kq;
        const bool vec = (wd & 3) == 0 && xq + 3 < wd;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int yy = y0 + 4 * wv + r;
            if (yy >= h) continue;
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                const int64_t o0 = ((int64_t)b * MAXC + n * 16 + r16) * plane + (int64_t)yy * wd + xq;
                float* o = out + o0;
                if (vec) {
                    *(float4*)o = make_float4(conv_epi<EPI>(acc[r][n][0], y, o0), conv_epi<EPI>(acc[r][n][1], y, o0 + 1),
                                              conv_epi<EPI>(acc[r][n][2], y, o0 + 2),
                                              conv_epi<EPI>(acc[r][n][3], y, o0 + 3));
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (xq + i < wd) o[i] = conv_epi<EPI>(acc[r][n][i], y, o0 + i);
                }
            }
        }
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
// block's share of (tile, image) pairs.  Per pair and tap t the gradient is a
// contraction over the tile's 256 pixels, gW_t[co][ci] += g[co][p] x[ci][p +
// d_t], on FP32 16 x 16 x 4 MFMAs: wave v owns the 16 x 16 block (co tile
// v / 2, ci tile v % 2) of all nine taps (36 accumulator registers); k runs
// over 4 consecutive pixels of a tile row.  LDS holds the output-gradient
// tile [co][260] and the input tile with its halo [ci][18 x 18], both FP32;
// the row strides (4 and 4 mod 64 banks) keep the 16 channel rows a
// quarter-wave reads in distinct banks.
constexpr int kGStride = TS * TS + 4;      // floats per output-gradient channel in LDS
constexpr int kXStride = kHaloPx;          // floats per input channel in LDS (324 = 4 mod 64)

__global__ void __launch_bounds__(TS* TS, 2)
k_conv_bwd_w(const float* __restrict__ in, const float* __restrict__ gout, float* __restrict__ partial, int batch,
             int cin, int cout, int h, int wd)
{
    __shared__ float gs[MAXC * kGStride];
    __shared__ float xs[MAXC * kXStride];
    const int tid = threadIdx.y * TS + threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int mt = wv >> 1, nt = wv & 1;   // co tile, ci tile of this wave
    const int r16 = lane & 15, kq = lane >> 4;
    const int tiles_x = (wd + TS - 1) / TS, tiles_y = (h + TS - 1) / TS;
    const int nwork = tiles_x * tiles_y * batch;
    const int64_t plane = (int64_t)h * wd;
    const int E = cout * cin * 9;
    const bool active = mt * 16 < cout && nt * 16 < cin;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    for (int wi = xcd_swizzle(blockIdx.x, gridDim.x); wi < nwork; wi += gridDim.x) {   // XCD-aware, as above
        const int b = wi / (tiles_x * tiles_y), tt = wi % (tiles_x * tiles_y);
        const int x0 = (tt % tiles_x) * TS, y0 = (tt / tiles_x) * TS;
        // output-gradient tile, every channel (zero outside the image and
        // for channels beyond cout), and the input tile with a wrapped halo
        // of one (zero for channels beyond cin): every load issued first.
        // Thread tid stages pixel tid of the tile and halo pixels tid and
        // tid + 256 (the latter for tid < 68), all channels.
        float gv[MAXC], xv[MAXC], xw[MAXC];
        // 32-bit element offsets within the image (checked on the host)
        const float* gb = gout + (int64_t)b * cout * plane;
        const float* xb0 = in + (int64_t)b * cin * plane;
        const bool two = tid + TS * TS < kHaloPx;
        {
            const int x = x0 + tid % TS, y = y0 + tid / TS;
            const bool in_img = x < wd && y < h;
            const uint32_t po = (uint32_t)(y * wd + x);
            const int r1 = two ? tid + TS * TS : 0;
            const uint32_t h0 = (uint32_t)(wrapc(y0 + tid / (TS + 2) - 1, h) * wd + wrapc(x0 + tid % (TS + 2) - 1, wd));
            const uint32_t h1 = (uint32_t)(wrapc(y0 + r1 / (TS + 2) - 1, h) * wd + wrapc(x0 + r1 % (TS + 2) - 1, wd));
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                const uint32_t co = (uint32_t)c * (uint32_t)plane;
                gv[c] = (c < cout && in_img) ? gb[co + po] : 0.f;
                xv[c] = c < cin ? xb0[co + h0] : 0.f;
                xw[c] = (two && c < cin) ? xb0[co + h1] : 0.f;
            }
        }
        __syncthreads();   // the previous item's reads of gs and xs are done
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            gs[c * kGStride + tid] = gv[c];
            xs[c * kXStride + tid] = xv[c];
            if (two) xs[c * kXStride + tid + TS * TS] = xw[c];
        }
        __syncthreads();
        {   // bias: thread (co = tid / 8, slice tid % 8) sums 32 pixels
            const float* gr = gs + (tid >> 3) * kGStride + (tid & 7) * 32;
            float sb = 0.f;
#pragma unroll 8
            for (int p = 0; p < 32; ++p) sb += gr[p];
            bacc += sb;
        }
        if (!active) continue;   // this wave's co or ci tile lies wholly beyond cout or cin
        const float* ga = gs + (mt * 16 + r16) * kGStride;
        const float* xb = xs + (nt * 16 + r16) * kXStride;
#pragma unroll 2
        for (int ks = 0; ks < TS * TS / 4; ++ks) {
            const int p = 4 * ks + kq;             // pixel of this lane's k
            const int hp = (p / TS) * (TS + 2) + p % TS;   // its halo index at tap (0, 0)
            const float av = ga[p];
#pragma unroll
            for (int t = 0; t < 9; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, xb[hp + (t / 3) * (TS + 2) + t % 3], acc[t], 0, 0,
                                                              0);
        }
    }
    float* pb = partial + (int64_t)blockIdx.x * (E + cout);
    const int ci = nt * 16 + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int co = mt * 16 + 4 * kq + i;
        if (ci < cin && co < cout)
#pragma unroll
            for (int t = 0; t < 9; ++t) pb[(ci * cout + co) * 9 + t] = acc[t][i];
    }
    // bias partial: the 8 slices of each channel, summed in a fixed order
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) bacc += __shfl_xor(bacc, off, 64);
    if ((tid & 7) == 0 && (tid >> 3) < cout) pb[E + (tid >> 3)] = bacc;
}

// The 32 -> 32 weight gradient on bf16 MFMAs.  The same contraction over
// pixels, gW_t[co][ci] += g[co][p] x[ci][p + d_t], with both operands split
// exactly into three bf16 parts and the six part products whose weights
// reach 2^-24 summed (hi.hi, hi.mid, mid.hi, hi.lo, mid.mid, lo.hi): FP32
// operands to within about 2^-24 of each product.  k runs over 32 pixels
// (two tile rows) per MFMA, 8 consecutive pixels of one row per lane.  A tap
// shifts the input by dx = 0, 1, 2 columns, so its 8-pixel run is 16-byte
// aligned (one vector read), 4-byte aligned (four dword reads) or 2-byte
// aligned (five dword reads realigned by v_alignbyte).  LDS: the input tile
// with its halo as [part][ci][18 rows][24 columns] and the output gradient as
// [part][co][256 + 8]; channel strides of 220 and 132 dwords put the 16
// channels a quarter-wave reads on distinct bank quads.  One block per CU
// (135 KB of LDS); wave v owns the 16 x 16 block (co tile v / 2, ci tile
// v % 2) of all nine taps.  The bias gradient sums the FP32 output gradient
// per thread and channel, then over the block in a fixed order.
constexpr int kXRS = 24;                       // bf16 per input row in LDS (18 + pad, 16-byte rows)
constexpr int kXCS = 18 * kXRS + 8;            // bf16 per input channel (220 dwords = 28 mod 64)
constexpr int kXPart = MAXC * kXCS;
constexpr int kGCS = TS * TS + 8;              // bf16 per output-gradient channel (132 dwords = 4 mod 64)
constexpr int kGPart = MAXC * kGCS;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int DX>
__device__ __forceinline__ bf16x8 x_run(const uint16_t* __restrict__ xs, int e)
{
    if (DX == 0) return *(const bf16x8*)(xs + e);
    u32x4 v;
    if (DX == 2) {
        const uint32_t* d = (const uint32_t*)(xs + e);
        v = u32x4{d[0], d[1], d[2], d[3]};
    } else {
        const uint32_t* d = (const uint32_t*)(xs + e - 1);
        const uint32_t d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4];
        v = u32x4{__builtin_amdgcn_alignbyte(d1, d0, 2), __builtin_amdgcn_alignbyte(d2, d1, 2),
                  __builtin_amdgcn_alignbyte(d3, d2, 2), __builtin_amdgcn_alignbyte(d4, d3, 2)};
    }
    return __builtin_bit_cast(bf16x8, v);
}

__global__ void __launch_bounds__(TS* TS, 1)
k_conv_bwd_w_bf16(const float* __restrict__ in, const float* __restrict__ gout, float* __restrict__ partial,
                  int batch, int h, int wd)
{
    __shared__ __align__(16) uint16_t xs[3 * kXPart];
    __shared__ __align__(16) uint16_t gs[3 * kGPart];
    const int tid = threadIdx.y * TS + threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int mt = wv >> 1, nt = wv & 1;
    const int r16 = lane & 15, kq = lane >> 4;
    const int tiles_x = (wd + TS - 1) / TS, tiles_y = (h + TS - 1) / TS;
    const int nwork = tiles_x * tiles_y * batch;
    const int64_t plane = (int64_t)h * wd;
    constexpr int E = MAXC * MAXC * 9;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) bsum[c] = 0.f;
    const bool two = tid + TS * TS < kHaloPx;
    const int r1 = two ? tid + TS * TS : 0;
    // the tile's loads for the next work item are issued before this one's
    // products, so their latency hides behind the MFMAs (one block per CU)
    float gv[MAXC], xv[MAXC], xw[MAXC];
    auto load = [&](int wi) {
        const int b = wi / (tiles_x * tiles_y), tt = wi % (tiles_x * tiles_y);
        const int x0 = (tt % tiles_x) * TS, y0 = (tt / tiles_x) * TS;
        const float* gb = gout + (int64_t)b * MAXC * plane;
        const float* xb0 = in + (int64_t)b * MAXC * plane;
        const int x = x0 + tid % TS, y = y0 + tid / TS;
        const bool in_img = x < wd && y < h;
        const uint32_t po = (uint32_t)(y * wd + x);
        const uint32_t h0 = (uint32_t)(wrapc(y0 + tid / (TS + 2) - 1, h) * wd + wrapc(x0 + tid % (TS + 2) - 1, wd));
        const uint32_t h1 = (uint32_t)(wrapc(y0 + r1 / (TS + 2) - 1, h) * wd + wrapc(x0 + r1 % (TS + 2) - 1, wd));
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            const uint32_t co = (uint32_t)c * (uint32_t)plane;
            gv[c] = in_img ? gb[co + po] : 0.f;
            xv[c] = xb0[co + h0];
            xw[c] = two ? xb0[co + h1] : 0.f;
        }
    };
    int wi = xcd_swizzle(blockIdx.x, gridDim.x);
    if (wi < nwork) load(wi);
    for (; wi < nwork; wi += gridDim.x) {
        __syncthreads();   // the previous item's reads of gs and xs are done
        {
            const int ly0 = tid / (TS + 2), lx0 = tid % (TS + 2);
            const int ly1 = r1 / (TS + 2), lx1 = r1 % (TS + 2);
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                bsum[c] += gv[c];
                uint32_t p0, p1, p2;
                split3(gv[c], p0, p1, p2);
                uint16_t* gd = gs + c * kGCS + tid;
                gd[0] = (uint16_t)p0;
                gd[kGPart] = (uint16_t)p1;
                gd[2 * kGPart] = (uint16_t)p2;
                split3(xv[c], p0, p1, p2);
                uint16_t* xd = xs + c * kXCS + ly0 * kXRS + lx0;
                xd[0] = (uint16_t)p0;
                xd[kXPart] = (uint16_t)p1;
                xd[2 * kXPart] = (uint16_t)p2;
                if (two) {
                    split3(xw[c], p0, p1, p2);
                    uint16_t* xe = xs + c * kXCS + ly1 * kXRS + lx1;
                    xe[0] = (uint16_t)p0;
                    xe[kXPart] = (uint16_t)p1;
                    xe[2 * kXPart] = (uint16_t)p2;
                }
            }
        }
        __syncthreads();
        if (wi + (int)gridDim.x < nwork) load(wi + gridDim.x);
        const uint16_t* ga = gs + (mt * 16 + r16) * kGCS;
        const int xb = (nt * 16 + r16) * kXCS;
#pragma unroll 1
        for (int ch = 0; ch < TS * TS / 32; ++ch) {
            const int p0 = 32 * ch + 8 * kq;           // this lane's 8 pixels
            const int ry = p0 / TS, cx0 = p0 % TS;     // tile row, first column
            bf16x8 a[3];
#pragma unroll
            for (int gp = 0; gp < 3; ++gp) a[gp] = *(const bf16x8*)(ga + gp * kGPart + p0);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3, dx = t % 3;
                const int e = xb + (ry + dy) * kXRS + cx0 + dx;
#pragma unroll
                for (int xp = 0; xp < 3; ++xp) {
                    const int ex = e + xp * kXPart;
                    const bf16x8 bv = dx == 0 ? x_run<0>(xs, ex) : (dx == 1 ? x_run<1>(xs, ex) : x_run<2>(xs, ex));
#pragma unroll
                    for (int gp = 0; gp + xp < 3; ++gp)
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[gp], bv, acc[t], 0, 0, 0);
                }
            }
        }
    }
    float* pb = partial + (int64_t)blockIdx.x * (E + MAXC);
    const int ci = nt * 16 + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int co = mt * 16 + 4 * kq + i;
#pragma unroll
        for (int t = 0; t < 9; ++t) pb[(ci * MAXC + co) * 9 + t] = acc[t][i];
    }
    // bias: each thread's per-channel sums, then over the block in a fixed
    // order (thread 0, 1, ...) through LDS
    __syncthreads();
    float* red = (float*)xs;   // MAXC x 256 floats fit in the input tile's LDS
#pragma unroll
    for (int c = 0; c < MAXC; ++c) red[c * (TS * TS) + tid] = bsum[c];
    __syncthreads();
    if (tid < MAXC) {
        float sb = 0.f;
        for (int k = 0; k < TS * TS; ++k) sb += red[tid * (TS * TS) + k];
        pb[E + tid] = sb;
    }
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

// compute units of the current device (cached per device): the persistent
// forward kernel runs two blocks per CU
static int cu_count()
{
    static int cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// the MFMA kernels address an image's channels with 32-bit element offsets
static bool conv_shape_ok(int batch, int cin, int cout, int h, int w)
{
    return batch >= 1 && cin >= 1 && cin <= MAXC && (cout == 1 || cout == MAXC) && h >= 1 && w >= 1 &&
           batch <= 65535 && (int64_t)h * w * MAXC < ((int64_t)1 << 31);
}

// the 32-output-channel forward on the matrix cores, with its epilogue
static hipError_t launch_fwd_mfma(int epi, const float* in, const uint16_t* w, const float* bias, float* out,
                                  const float* y, int batch, int cin, int h, int wd, hipStream_t s)
{
    const int tiles = ((wd + TS - 1) / TS) * ((h + TS - 1) / TS);
    const int64_t nwork = (int64_t)tiles * batch;
    const int nb = (int)(nwork < 2 * cu_count() ? nwork : 2 * cu_count());
    const dim3 block(TS, TS);
    if (epi == kEpiTanh)
        hipLaunchKernelGGL(k_conv_fwd_mfma<kEpiTanh>, dim3(nb), block, 0, s, in, w, bias, out, y, batch, cin, h, wd);
    else if (epi == kEpiTanhGrad)
        hipLaunchKernelGGL(k_conv_fwd_mfma<kEpiTanhGrad>, dim3(nb), block, 0, s, in, w, bias, out, y, batch, cin, h,
                           wd);
    else
        hipLaunchKernelGGL(k_conv_fwd_mfma<kEpiNone>, dim3(nb), block, 0, s, in, w, bias, out, y, batch, cin, h, wd);
    return hipGetLastError();
}

extern "C" int sc_nn_conv3x3_fwd(const float* in, const uint16_t* w, const float* bias, float* out, int32_t batch,
                                 int32_t cin, int32_t cout, int32_t h, int32_t wd, void* stream)
{
    if (!in || !w || !out || !conv_shape_ok(batch, cin, cout, h, wd)) return SC_E_INVAL;
    if (cout == MAXC)
        return nn_status(launch_fwd_mfma(kEpiNone, in, w, bias, out, nullptr, batch, cin, h, wd, (hipStream_t)stream));
    const int tiles = ((wd + TS - 1) / TS) * ((h + TS - 1) / TS);
    dim3 grid(tiles, batch), block(TS, TS);
    hipLaunchKernelGGL(k_conv_fwd<1>, grid, block, 0, (hipStream_t)stream, in, w, bias, out, cin, cout, h, wd);
    return nn_status(hipGetLastError());
}

extern "C" int sc_nn_conv3x3_fwd_tanh(const float* in, const uint16_t* w, const float* bias, float* out,
                                      int32_t batch, int32_t cin, int32_t cout, int32_t h, int32_t wd, void* stream)
{
    if (!in || !w || !out || !conv_shape_ok(batch, cin, cout, h, wd) || cout != MAXC) return SC_E_INVAL;
    return nn_status(launch_fwd_mfma(kEpiTanh, in, w, bias, out, nullptr, batch, cin, h, wd, (hipStream_t)stream));
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

extern "C" int sc_nn_conv3x3_bwd_data_tanh(const float* gout, const uint16_t* w, uint16_t* wt_scratch, const float* y,
                                           float* gin, int32_t batch, int32_t cin, int32_t cout, int32_t h, int32_t wd,
                                           void* stream)
{
    if (!gout || !w || !wt_scratch || !y || !gin || !conv_shape_ok(batch, cin, cout, h, wd) || cin != MAXC)
        return SC_E_INVAL;
    const int nw = cin * cout * 9;
    hipLaunchKernelGGL(k_transpose_flip, (nw + 255) / 256, 256, 0, (hipStream_t)stream, w, wt_scratch, cin, cout);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nn_status(e);
    return nn_status(
        launch_fwd_mfma(kEpiTanhGrad, gout, wt_scratch, nullptr, gin, y, batch, cout, h, wd, (hipStream_t)stream));
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
    if (cin == MAXC && cout == MAXC)
        hipLaunchKernelGGL(k_conv_bwd_w_bf16, nblk, dim3(TS, TS), 0, s, in, gout, partial_scratch, batch, h, wd);
    else
        hipLaunchKernelGGL(k_conv_bwd_w, nblk, dim3(TS, TS), 0, s, in, gout, partial_scratch, batch, cin, cout, h,
                           wd);
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
