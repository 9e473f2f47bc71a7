// kernels_batch.hip -- one launch advances many independent D2Q9 droplets
// of different sizes and parameters by one step (batched parameter sweeps).
//
// Work list: one entry per (item, tile) of every active item; block b takes
// entry b.  Each item has a descriptor (its two state buffers, grid, G c0,
// tau and stencil order).  The block body is the tile kernel of
// kernels_2d.hip with the stencil order chosen per block (a uniform switch
// over the four compiled orders) and an LDS tile sized for the largest
// radius (3), so items of every order share one launch.  Items drop out of
// the work list when they converge; the host rebuilds the list.
#include "reduce.h"
#include "tile2.h"

namespace sclbm {

template <typename T>
struct BatchItem {
    const T* a;          // state buffer 0
    T* b;                // state buffer 1
    int nx, ny;
    int order;           // 4, 6, 8, 10
    T gc0, omega, guo;
};

constexpr int kBTX = 32, kBTY = 8, kBRMAX = 3;

template <typename T, int ORDER>
__device__ __forceinline__ void batch_force(const T* c, int LW, T& sx, T& sy)
{
    using ST = Stencil<2, ORDER>;
    sx = T(0);
    sy = T(0);
    T ax = T(0), ay = T(0);
#pragma unroll
    for (int p = 0; p < ST::NP; ++p) {
        constexpr PairList P = ST::P;
        const int ex = P.e[p][0], ey = P.e[p][1];
        const T d = c[ey * LW + ex] - c[-ey * LW - ex];
        if (ex) ax += T(ex) * d;
        if (ey) ay += T(ey) * d;
        if (P.shell_end(p)) {   // one weight per shell
            sx += T(P.w[p]) * ax;
            sy += T(P.w[p]) * ay;
            ax = ay = T(0);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBTX* kBTY)
k_d2q9_batch(const BatchItem<T>* __restrict__ items, const int2* __restrict__ work, int parity,
             StepArgs<T> common)
{
    constexpr int TX = kBTX, TY = kBTY, RM = kBRMAX;
    constexpr int LW = TX + 2 * RM, LH = TY + 2 * RM;
    constexpr int NT = TX * TY;
    __shared__ T psi_s[LH * LW];

    const int2 wk = work[blockIdx.x];
    const BatchItem<T> it = items[wk.x];
    StepArgs<T> a = common;
    a.fin = parity ? it.b : it.a;
    a.fout = parity ? (T*)it.a : it.b;
    a.nx = it.nx;
    a.ny = it.ny;
    a.nz = 1;
    a.n = (int64_t)it.nx * it.ny;
    a.gc0 = it.gc0;
    a.omega = it.omega;
    a.guo = it.guo;
    const int nx = a.nx, ny = a.ny;
    const int64_t n = a.n;
    const int R = it.order == 4 ? 1 : (it.order == 10 ? 3 : 2);
    const uint32_t TS = sizeof(T), rowb = (uint32_t)nx * TS;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    const int tiles_x = (it.nx + TX - 1) / TX;
    const int x0 = (wk.y % tiles_x) * TX, y0 = (wk.y / tiles_x) * TY;

    const int xr = x0 + tx, yr = y0 + ty;
    const bool valid = xr < nx && yr < ny;
    uint32_t xo[3], yo[3];
    nbr_offsets<T>(xr < nx ? xr : xr % nx, nx, TS, xo);
    nbr_offsets<T>(yr < ny ? yr : yr % ny, ny, rowb, yo);
    T g[9];
    pull_d2q9(a.fin, n, xo, yo, g);
    const T dr = sum9(g);
    psi_s[(ty + RM) * LW + tx + RM] = psi_of(a.rho_ref + dr, a);

    // halo ring of width R around the tile, stored at LDS origin RM - R
    const int rw = TX + 2 * R, rh = TY + 2 * R;
    const int ring = rw * rh - TX * TY;
    for (int i = tid; i < ring; i += NT) {
        int lx, ly;
        if (i < R * rw) {
            ly = i / rw;
            lx = i - ly * rw;
        } else if (i < 2 * R * rw) {
            const int j = i - R * rw;
            ly = TY + R + j / rw;
            lx = j % rw;
        } else {
            const int j = i - 2 * R * rw;
            ly = R + j / (2 * R);
            const int c = j % (2 * R);
            lx = c < R ? c : TX + c;
        }
        uint32_t hxo[3], hyo[3];
        nbr_offsets<T>(wrap_near(x0 - R + lx, nx), nx, TS, hxo);
        nbr_offsets<T>(wrap_near(y0 - R + ly, ny), ny, rowb, hyo);
        T h[9];
        pull_d2q9(a.fin, n, hxo, hyo, h);
        psi_s[(ly + RM - R) * LW + lx + RM - R] = psi_of(a.rho_ref + sum9(h), a);
    }
    __syncthreads();

    const T* c = psi_s + (ty + RM) * LW + tx + RM;
    T sx, sy;
    switch (it.order) {   // uniform across the block
    case 4: batch_force<T, 4>(c, LW, sx, sy); break;
    case 6: batch_force<T, 6>(c, LW, sx, sy); break;
    case 8: batch_force<T, 8>(c, LW, sx, sy); break;
    default: batch_force<T, 10>(c, LW, sx, sy); break;
    }
    const T pref = -a.gc0 * c[0];
    collide_d2q9_srt(g, dr, pref * sx, pref * sy, a);
    if (valid) {
        const uint32_t off = yo[1] + xo[1];
#pragma unroll
        for (int b = 0; b < 9; ++b) st_off(a.fout + b * n, off, g[b]);
    }
}

// Two steps per launch: the two-step tile of the single-grid kernel
// (tile2.h) per work entry, with the item's stencil order (a uniform switch)
// and LDS sized for the largest radius.  Work entries of one item are listed
// in strip order; the XCD swizzle gives each XCD a contiguous range of them,
// so tiles that share halo lines run on the same XCD (same L2).
template <typename T, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_d2q9_batch2(const BatchItem<T>* __restrict__ items, const int2* __restrict__ work, int parity,
              StepArgs<T> common)
{
    using LD = Tile2Lds<kBRMAX, TX, TY>;
    __shared__ T psi1[LD::P1N];
    __shared__ T psi2[LD::P2N];
    __shared__ T s1[9 * LD::C1N];
    const int2 wk = work[xcd_swizzle(blockIdx.x, gridDim.x)];
    const BatchItem<T> it = items[wk.x];
    StepArgs<T> a = common;
    a.fin = parity ? it.b : it.a;
    a.fout = parity ? (T*)it.a : it.b;
    a.nx = it.nx;
    a.ny = it.ny;
    a.nz = 1;
    a.n = (int64_t)it.nx * it.ny;
    a.gc0 = it.gc0;
    a.omega = it.omega;
    a.guo = it.guo;
    const int tiles_x = (it.nx + TX - 1) / TX;
    const int x0 = (wk.y % tiles_x) * TX, y0 = (wk.y / tiles_x) * TY;
    switch (it.order) {   // uniform across the block
    case 4: d2q9_tile2_body<T, 4, TX, TY, NT>(a, x0, y0, psi1, psi2, s1); break;
    case 6: d2q9_tile2_body<T, 6, TX, TY, NT>(a, x0, y0, psi1, psi2, s1); break;
    case 8: d2q9_tile2_body<T, 8, TX, TY, NT>(a, x0, y0, psi1, psi2, s1); break;
    default: d2q9_tile2_body<T, 10, TX, TY, NT>(a, x0, y0, psi1, psi2, s1); break;
    }
}

// ------------------------------------------------------------ shapes ----
struct BatchShape {
    int tw, th, steps;
    const char* name;
};
static const BatchShape kBatchShapes[] = {
    {kBTX, kBTY, 1, "batch32x8"},
    {32, 8, 2, "batch2x32x8t256"},
    {64, 16, 2, "batch2x64x16t1024"},
    {32, 16, 2, "batch2x32x16t512"},
};
constexpr int kNumBatchShapes = sizeof(kBatchShapes) / sizeof(kBatchShapes[0]);

int batch_num_shapes() { return kNumBatchShapes; }
int batch_shape_steps(int v) { return (v >= 0 && v < kNumBatchShapes) ? kBatchShapes[v].steps : 0; }
void batch_shape_tile(int v, int* tw, int* th)
{
    const BatchShape& b = kBatchShapes[(v >= 0 && v < kNumBatchShapes) ? v : 0];
    *tw = b.tw;
    *th = b.th;
}
const char* batch_shape_name(int v) { return (v >= 0 && v < kNumBatchShapes) ? kBatchShapes[v].name : "?"; }

template <typename T>
static hipError_t batch_launch_t(int shape, const BatchItem<T>* items, const int2* work, int nwork, int parity,
                                 const StepArgs<T>& common, hipStream_t s)
{
    switch (shape) {
    case 0:
        hipLaunchKernelGGL(k_d2q9_batch<T>, dim3(nwork), dim3(kBTX, kBTY), 0, s, items, work, parity, common);
        break;
    case 1:
        hipLaunchKernelGGL((k_d2q9_batch2<T, 32, 8, 256>), dim3(nwork), dim3(256), 0, s, items, work, parity,
                           common);
        break;
    case 2:
        hipLaunchKernelGGL((k_d2q9_batch2<T, 64, 16, 1024>), dim3(nwork), dim3(1024), 0, s, items, work, parity,
                           common);
        break;
    case 3:
        hipLaunchKernelGGL((k_d2q9_batch2<T, 32, 16, 512>), dim3(nwork), dim3(512), 0, s, items, work, parity,
                           common);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_d2q9(int shape, const void* items, const int2* work, int nwork, int parity, int precision,
                             const void* common, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    if (precision == 0)
        return batch_launch_t<float>(shape, (const BatchItem<float>*)items, work, nwork, parity,
                                     *(const StepArgs<float>*)common, s);
    return batch_launch_t<double>(shape, (const BatchItem<double>*)items, work, nwork, parity,
                                  *(const StepArgs<double>*)common, s);
}

size_t batch_item_bytes(int precision)
{
    return precision == 0 ? sizeof(BatchItem<float>) : sizeof(BatchItem<double>);
}

void batch_fill_item(void* dst, int precision, const void* a, void* b, int nx, int ny, int order, double gc0,
                     double tau)
{
    if (precision == 0) {
        BatchItem<float> it{(const float*)a, (float*)b, nx, ny, order, (float)gc0, (float)(1.0 / tau),
                            (float)(1.0 - 0.5 / tau)};
        *(BatchItem<float>*)dst = it;
    } else {
        BatchItem<double> it{(const double*)a, (double*)b, nx, ny, order, gc0, 1.0 / tau, 1.0 - 0.5 / tau};
        *(BatchItem<double>*)dst = it;
    }
}

// ------------------------------------------------------------- check ----
// Steady-state check of the active items: block k takes check entry k, a
// (item, 16 x 16 tile) pair, and runs the fused check of that tile on the
// item's current buffer with the item's stencil order; its partial row is
// row k.  Then one block per active item sums the rows of its entries in
// order into the item's result row.
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_batch_check(const BatchItem<T>* __restrict__ items, const int2* __restrict__ cwork, int parity,
              StepArgs<T> common, double* __restrict__ partials, double* __restrict__ results)
{
    using CT = CheckTile<2>;
    __shared__ T psi_s[check_lds_max<2>()];
    const int2 wk = cwork[blockIdx.x];
    const BatchItem<T> it = items[wk.x];
    StepArgs<T> a = common;
    a.fin = parity ? it.b : it.a;
    a.nx = it.nx;
    a.ny = it.ny;
    a.nz = 1;
    a.n = (int64_t)it.nx * it.ny;
    a.gc0 = it.gc0;
    const int tiles_x = (it.nx + CT::TX - 1) / CT::TX;
    const int x0 = (wk.y % tiles_x) * CT::TX, y0 = (wk.y / tiles_x) * CT::TY;
    const int64_t ic = (int64_t)(it.nx / 2) + (int64_t)it.nx * (it.ny / 2);
    double* extra = results + (int64_t)wk.x * kCheckSlots + kObsSlots;
    double acc[kNR];
#pragma unroll
    for (int k = 0; k < kNR; ++k) acc[k] = slot_start(k);
    switch (it.order) {   // uniform across the block
    case 4: check_tile<T, D2Q9, 1, 4>(a, x0, y0, 0, psi_s, acc, ic, extra); break;
    case 6: check_tile<T, D2Q9, 1, 6>(a, x0, y0, 0, psi_s, acc, ic, extra); break;
    case 8: check_tile<T, D2Q9, 1, 8>(a, x0, y0, 0, psi_s, acc, ic, extra); break;
    default: check_tile<T, D2Q9, 1, 10>(a, x0, y0, 0, psi_s, acc, ic, extra); break;
    }
    block_reduce_store(acc, partials + (int64_t)blockIdx.x * kNR);
}

__global__ void __launch_bounds__(kRedThreads)
k_batch_check_final(const int4* __restrict__ citems, const double* __restrict__ partials, double* __restrict__ results)
{
    const int4 ci = citems[blockIdx.x];   // item, first entry, entry count
    double acc[kNR];
#pragma unroll
    for (int k = 0; k < kNR; ++k) acc[k] = slot_start(k);
    for (int b = threadIdx.x; b < ci.z; b += blockDim.x) {
        const double* p = partials + (int64_t)(ci.y + b) * kNR;
#pragma unroll
        for (int k = 0; k < kNR; ++k) acc[k] = is_max_slot(k) ? fmax(acc[k], p[k]) : acc[k] + p[k];
    }
    block_reduce_store(acc, results + (int64_t)ci.x * kCheckSlots);
}

int batch_check_tile() { return CheckTile<2>::TX; }

hipError_t launch_batch_check(const void* items, const int2* cwork, int ncwork, const int4* citems, int nactive,
                              int parity, int precision, const void* common, double* partials, double* results,
                              hipStream_t s)
{
    if (ncwork <= 0 || nactive <= 0) return hipSuccess;
    if (precision == 0)
        hipLaunchKernelGGL(k_batch_check<float>, dim3(ncwork), dim3(kRedThreads), 0, s,
                           (const BatchItem<float>*)items, cwork, parity, *(const StepArgs<float>*)common, partials,
                           results);
    else
        hipLaunchKernelGGL(k_batch_check<double>, dim3(ncwork), dim3(kRedThreads), 0, s,
                           (const BatchItem<double>*)items, cwork, parity, *(const StepArgs<double>*)common,
                           partials, results);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_check_final, dim3(nactive), dim3(kRedThreads), 0, s, citems, partials, results);
    return hipGetLastError();
}

// ------------------------------------------- net momentum of a state ----
// Stored mass and momentum of one FP64 D2Q9 state (shifted storage):
// partial[blk] = (sum g_b, sum g_b c_bx, sum g_b c_by) over the block's
// grid-stride share of the n nodes; a fixed-order tree in LDS per block.
constexpr int kMomThreads = 256;

__global__ void __launch_bounds__(kMomThreads)
k_d2q9_mass_momentum(const double* __restrict__ g, int64_t n, double* __restrict__ partial)
{
    __shared__ double red[3][kMomThreads];
    double m = 0.0, jx = 0.0, jy = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kMomThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kMomThreads) {
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            const double v = g[b * n + i];
            m += v;
            jx += D2Q9::cx[b] * v;
            jy += D2Q9::cy[b] * v;
        }
    }
    red[0][threadIdx.x] = m;
    red[1][threadIdx.x] = jx;
    red[2][threadIdx.x] = jy;
    __syncthreads();
    for (int w = kMomThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) partial[blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// Every node's populations move by the equilibrium change of a uniform
// velocity shift du at the node's own (post-collision) density:
// g_b += 3 w_b rho_x (c_b . du).  The node's mass is unchanged (sum_b w_b c_b
// = 0) and its momentum grows by rho_x du, the state's by M du.
__global__ void k_d2q9_momentum_shift(double* __restrict__ g, int64_t n, double rho_ref, double ux, double uy)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double rho = rho_ref;
#pragma unroll
        for (int b = 0; b < 9; ++b) rho += g[b * n + i];
#pragma unroll
        for (int b = 1; b < 9; ++b)
            g[b * n + i] += 3.0 * D2Q9::w[b] * rho * (D2Q9::cx[b] * ux + D2Q9::cy[b] * uy);
    }
}

int momentum_blocks() { return 256; }

hipError_t launch_d2q9_mass_momentum(const double* g, int64_t n, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_d2q9_mass_momentum, dim3(momentum_blocks()), dim3(kMomThreads), 0, s, g, n, partial);
    return hipGetLastError();
}

hipError_t launch_d2q9_momentum_shift(double* g, int64_t n, double rho_ref, double ux, double uy, hipStream_t s)
{
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_d2q9_momentum_shift, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, s, g, n,
                       rho_ref, ux, uy);
    return hipGetLastError();
}

}  // namespace sclbm
