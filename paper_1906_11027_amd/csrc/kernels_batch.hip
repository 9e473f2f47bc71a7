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
#include "kernels.h"

namespace sclbm {

template <typename T>
struct BatchItem {
    const T* a;          // state buffer 0
    T* b;                // state buffer 1
    int nx, ny;
    int tiles_x;         // tiles per row of this item
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
    const int x0 = (wk.y % it.tiles_x) * TX, y0 = (wk.y / it.tiles_x) * TY;

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

int batch_tile_w() { return kBTX; }
int batch_tile_h() { return kBTY; }

hipError_t launch_batch_d2q9(const void* items, const int2* work, int nwork, int parity, int precision,
                             const void* common, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    dim3 block(kBTX, kBTY);
    if (precision == 0)
        hipLaunchKernelGGL(k_d2q9_batch<float>, dim3(nwork), block, 0, s, (const BatchItem<float>*)items, work,
                           parity, *(const StepArgs<float>*)common);
    else
        hipLaunchKernelGGL(k_d2q9_batch<double>, dim3(nwork), block, 0, s, (const BatchItem<double>*)items, work,
                           parity, *(const StepArgs<double>*)common);
    return hipGetLastError();
}

size_t batch_item_bytes(int precision)
{
    return precision == 0 ? sizeof(BatchItem<float>) : sizeof(BatchItem<double>);
}

void batch_fill_item(void* dst, int precision, const void* a, void* b, int nx, int ny, int order, double gc0,
                     double tau)
{
    const int tiles_x = (nx + kBTX - 1) / kBTX;
    if (precision == 0) {
        BatchItem<float> it{(const float*)a, (float*)b, nx, ny, tiles_x, order, (float)gc0, (float)(1.0 / tau),
                            (float)(1.0 - 0.5 / tau)};
        *(BatchItem<float>*)dst = it;
    } else {
        BatchItem<double> it{(const double*)a, (double*)b, nx, ny, tiles_x, order, gc0, 1.0 / tau, 1.0 - 0.5 / tau};
        *(BatchItem<double>*)dst = it;
    }
}

}  // namespace sclbm
