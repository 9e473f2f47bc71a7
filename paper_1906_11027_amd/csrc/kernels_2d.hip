// kernels_2d.hip -- fused D2Q9 step for gfx950: psi(rho) halo tile in LDS,
// interaction force (Sec. 2, Eq. (1)) on the E4/E6/E8/E10 stencil, Guo-forced
// BGK collision (Eq. (3)-(4)) and pull streaming, one pass over the state.
//
// Tile kernel: a block owns a TX x TY tile; every thread owns RPT consecutive
// rows of one column.
//   phase 1  pull the 9 values of the owned nodes (kept in registers), form
//            rho and psi and write psi to LDS; then fill the psi halo ring of
//            width R (stencil radius) by pulling those nodes too (their f
//            lines are the neighbouring tiles' and mostly hit L2);
//   phase 2  F from LDS (sum over +-e pairs), velocity, equilibrium, Guo
//            source, relaxation, coalesced store at the node's own address.
// Ragged tiles: out-of-grid threads still fill LDS with wrapped (valid)
// psi and only skip the store, so any nx, ny >= 1 works.
#include "kernels.h"

namespace sclbm {

template <typename T, int ORDER, int TX, int TY, int RPT>
__global__ void __launch_bounds__(TX*(TY / RPT))
k_d2q9_tile(StepArgs<T> a)
{
    using ST = Stencil<2, ORDER>;
    constexpr int R = ST::R;
    constexpr int LW = TX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int NT = TX * (TY / RPT);
    __shared__ T psi_s[LH * LW];

    const int nx = a.nx, ny = a.ny;
    const int64_t n = a.n;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;

    const int xr = x0 + tx;
    const bool xin = xr < nx;
    const int x = xin ? xr : xr % nx;
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int xp = x == nx - 1 ? 0 : x + 1;

    T g[RPT][9];
    T dr[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty * RPT + k;
        const int yr = y0 + ly;
        const int y = yr < ny ? yr : yr % ny;
        const int ym = y == 0 ? ny - 1 : y - 1;
        const int yp = y == ny - 1 ? 0 : y + 1;
        pull_d2q9(a.fin, n, nx, x, xm, xp, y, ym, yp, g[k]);
        dr[k] = sum9(g[k]);
        psi_s[(ly + R) * LW + tx + R] = psi_of(a.rho_ref + dr[k], a);
    }

    // halo ring: R rows on top and bottom (full width), R columns each side
    constexpr int RING = LH * LW - TX * TY;
    for (int i = tid; i < RING; i += NT) {
        int lx, ly;
        if (i < R * LW) {
            ly = i / LW;
            lx = i - ly * LW;
        } else if (i < 2 * R * LW) {
            const int j = i - R * LW;
            ly = TY + R + j / LW;
            lx = j % LW;
        } else {
            const int j = i - 2 * R * LW;
            ly = R + j / (2 * R);
            const int c = j % (2 * R);
            lx = c < R ? c : TX + c;
        }
        const int hx = wrap_any(x0 - R + lx, nx);
        const int hy = wrap_any(y0 - R + ly, ny);
        const int hxm = hx == 0 ? nx - 1 : hx - 1, hxp = hx == nx - 1 ? 0 : hx + 1;
        const int hym = hy == 0 ? ny - 1 : hy - 1, hyp = hy == ny - 1 ? 0 : hy + 1;
        T h[9];
        pull_d2q9(a.fin, n, nx, hx, hxm, hxp, hy, hym, hyp, h);
        psi_s[ly * LW + lx] = psi_of(a.rho_ref + sum9(h), a);
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty * RPT + k;
        const int yr = y0 + ly;
        const T* c = psi_s + (ly + R) * LW + tx + R;
        T sx = T(0), sy = T(0);
#pragma unroll
        for (int p = 0; p < ST::NP; ++p) {
            constexpr PairList P = ST::P;
            const int ex = P.e[p][0], ey = P.e[p][1];
            const T d = c[ey * LW + ex] - c[-ey * LW - ex];
            const T wd = T(P.w[p]) * d;
            if (ex) sx += T(ex) * wd;
            if (ey) sy += T(ey) * wd;
        }
        const T pref = -a.gc0 * c[0];
        collide_d2q9_srt(g[k], dr[k], pref * sx, pref * sy, a);
        if (xin && yr < ny) {
            T* o = a.fout + (int64_t)yr * nx + xr;
#pragma unroll
            for (int b = 0; b < 9; ++b) o[b * n] = g[k][b];
        }
    }
}

// ------------------------------------------------------------ dispatch ----
struct Shape2D {
    int tx, ty, rpt;
    const char* name;
};
static const Shape2D kShapes2D[] = {
    {64, 16, 4, "tile64x16r4"},
    {64, 8, 2, "tile64x8r2"},
    {32, 8, 1, "tile32x8r1"},
    {64, 4, 1, "tile64x4r1"},
};
constexpr int kNumShapes2D = sizeof(kShapes2D) / sizeof(kShapes2D[0]);

int num_variants_d2q9() { return kNumShapes2D; }
const char* variant_name_d2q9(int v) { return (v >= 0 && v < kNumShapes2D) ? kShapes2D[v].name : "?"; }

template <typename T, int ORDER, int TX, int TY, int RPT>
static hipError_t launch_tile(const StepArgs<T>& a, hipStream_t s)
{
    dim3 block(TX, TY / RPT);
    dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY);
    hipLaunchKernelGGL((k_d2q9_tile<T, ORDER, TX, TY, RPT>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename T, int ORDER>
static hipError_t launch_order(const StepArgs<T>& a, int variant, hipStream_t s)
{
    switch (variant) {
    case 0: return launch_tile<T, ORDER, 64, 16, 4>(a, s);
    case 1: return launch_tile<T, ORDER, 64, 8, 2>(a, s);
    case 2: return launch_tile<T, ORDER, 32, 8, 1>(a, s);
    case 3: return launch_tile<T, ORDER, 64, 4, 1>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_any(const StepArgs<T>& a, int order, int variant, hipStream_t s)
{
    switch (order) {
    case 4: return launch_order<T, 4>(a, variant, s);
    case 6: return launch_order<T, 6>(a, variant, s);
    case 8: return launch_order<T, 8>(a, variant, s);
    case 10: return launch_order<T, 10>(a, variant, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_d2q9(const StepArgs<float>& a, int order, int variant, hipStream_t s)
{
    return launch_any<float>(a, order, variant, s);
}
hipError_t launch_step_d2q9(const StepArgs<double>& a, int order, int variant, hipStream_t s)
{
    return launch_any<double>(a, order, variant, s);
}

}  // namespace sclbm
