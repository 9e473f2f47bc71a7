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
#include "tile2.h"

namespace sclbm {

template <int ORDER, int TX, int TY>
struct TileLds {
    static constexpr int R = Stencil<2, ORDER>::R;
    static constexpr int LW = TX + 2 * R;
    static constexpr int LH = TY + 2 * R;
};

// One tile of the fused step (both phases); psi_s holds LH x LW values.
template <typename T, int ORDER, int TX, int TY, int RPT>
__device__ __forceinline__ void d2q9_tile_body(const StepArgs<T>& a, int x0, int y0, T* __restrict__ psi_s)
{
    using ST = Stencil<2, ORDER>;
    constexpr int R = ST::R;
    constexpr int LW = TX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int NT = TX * (TY / RPT);

    const int nx = a.nx, ny = a.ny;
    const int64_t n = a.n;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;

    const uint32_t TS = sizeof(T), rowb = (uint32_t)nx * TS;
    const int xr = x0 + tx;
    const bool xin = xr < nx;
    const int x = xin ? xr : xr % nx;
    uint32_t xo[3];
    nbr_offsets<T>(x, nx, TS, xo);

    // this thread's halo-ring nodes (R rows above and below at full width,
    // R columns each side): coordinates first, so the ring pulls are issued
    // together with the tile's own pulls
    constexpr int RING = LH * LW - TX * TY;
    constexpr int RPERT = (RING + NT - 1) / NT;
    int rl[RPERT];
    uint32_t rxo[RPERT][3], ryo[RPERT][3];
#pragma unroll
    for (int q = 0; q < RPERT; ++q) {
        const int i = tid + q * NT;
        int lx = 0, ly = 0;
        if (i < R * LW) {
            ly = i / LW;
            lx = i - ly * LW;
        } else if (i < 2 * R * LW) {
            const int j = i - R * LW;
            ly = TY + R + j / LW;
            lx = j % LW;
        } else if (i < RING) {
            const int j = i - 2 * R * LW;
            ly = R + j / (2 * R);
            const int c = j % (2 * R);
            lx = c < R ? c : TX + c;
        }
        rl[q] = i < RING ? ly * LW + lx : -1;
        nbr_offsets<T>(wrap_near(x0 - R + lx, nx), nx, TS, rxo[q]);
        nbr_offsets<T>(wrap_near(y0 - R + ly, ny), ny, rowb, ryo[q]);
    }

    T g[RPT][9];
    T dr[RPT];
    uint32_t own[RPT];
    T h[RPERT][9];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int yr = y0 + ty * RPT + k;
        uint32_t yo[3];
        nbr_offsets<T>(yr < ny ? yr : yr % ny, ny, rowb, yo);
        own[k] = yo[1] + xo[1];
        pull_d2q9(a.fin, n, xo, yo, g[k]);
    }
#pragma unroll
    for (int q = 0; q < RPERT; ++q)
        if (rl[q] >= 0) pull_d2q9(a.fin, n, rxo[q], ryo[q], h[q]);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        dr[k] = sum9(g[k]);
        psi_s[(ty * RPT + k + R) * LW + tx + R] = psi_of(a.rho_ref + dr[k], a);
    }
#pragma unroll
    for (int q = 0; q < RPERT; ++q)
        if (rl[q] >= 0) psi_s[rl[q]] = psi_of(a.rho_ref + sum9(h[q]), a);
    __syncthreads();

#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty * RPT + k;
        const int yr = y0 + ly;
        const T* c = psi_s + (ly + R) * LW + tx + R;
        T sx = T(0), sy = T(0), ax = T(0), ay = T(0);
#pragma unroll
        for (int p = 0; p < ST::NP; ++p) {
            constexpr PairList P = ST::P;
            const int ex = P.e[p][0], ey = P.e[p][1];
            const T d = c[ey * LW + ex] - c[-ey * LW - ex];
            if (ex) ax += T(ex) * d;
            if (ey) ay += T(ey) * d;
            if (P.shell_end(p)) {
                sx += T(P.w[p]) * ax;
                sy += T(P.w[p]) * ay;
                ax = ay = T(0);
            }
        }
        const T pref = -a.gc0 * c[0];
        collide_d2q9_srt(g[k], dr[k], pref * sx, pref * sy, a);
        if (xin && yr < ny) {
#pragma unroll
            for (int b = 0; b < 9; ++b) st_off(a.fout + b * n, own[k], g[k][b]);
        }
    }
}

// One tile per block, tiles in strip order.
template <typename T, int ORDER, int TX, int TY, int RPT>
__global__ void __launch_bounds__(TX*(TY / RPT))
k_d2q9_tile(StepArgs<T> a, int nbx, int nby, int sw)
{
    using LD = TileLds<ORDER, TX, TY>;
    __shared__ T psi_s[LD::LH * LD::LW];
    int bx, by;
    strip_tile(xcd_swizzle(blockIdx.x, gridDim.x), nbx, nby, sw, bx, by);
    d2q9_tile_body<T, ORDER, TX, TY, RPT>(a, bx * TX, by * TY, psi_s);
}

// y-marching kernel for large grids.  A block of NT threads owns the
// NT - 2R output columns [x0, x0 + NT - 2R) and H rows [y0, y0 + H); thread t
// handles column x0 - R + t, so the R outermost threads on each side only
// supply halo psi.  The block walks rows y0 - R ... y0 + H + R - 1: row j's
// psi goes into one of 2R + 2 LDS row slots, and once rows j - 2R ... j are
// resident row j - R is collided and stored.  The 9 values of the next row
// are loaded while the current row is processed (prefetch distance 1), and
// the values of the R pending rows stay in registers: the row loop is
// unrolled by R + 2 so the register window is statically indexed.  Each
// interior value is read from HBM once; the halo costs 2R columns per block
// (same XCD, L2 hits) and 2R + 2 rows per H (neighbouring segment).
template <typename T, int ORDER, int NT, int PF>
__global__ void __launch_bounds__(NT)
k_d2q9_march(StepArgs<T> a, int H, int nbx)
{
    using ST = Stencil<2, ORDER>;
    constexpr int R = ST::R;
    constexpr int TXO = NT - 2 * R;
    constexpr int NS = 2 * R + 2;
    constexpr int W = R + 1 + PF;   // R pending rows, the current row, PF rows in flight
    __shared__ T psi_s[NS * NT];

    const int nx = a.nx, ny = a.ny;
    const int64_t n = a.n;
    const int L = xcd_swizzle(blockIdx.x, gridDim.x);
    const int x0 = (L % nbx) * TXO, y0 = (L / nbx) * H;
    const int t = threadIdx.x;
    const uint32_t TS = sizeof(T), rowb = (uint32_t)nx * TS;
    const int xr = x0 - R + t;
    uint32_t xo[3];
    nbr_offsets<T>(wrap_any(xr, nx), nx, TS, xo);
    const bool interior = t >= R && t < NT - R && xr < nx;
    const int nrows = H + 2 * R;

    T g[W][9];
    int yl = wrap_any(y0 - R, ny);   // last row whose load was issued
#pragma unroll
    for (int q = 0; q < PF; ++q) {   // rows 0 .. PF-1
        if (q) yl = yl == ny - 1 ? 0 : yl + 1;
        uint32_t yo[3];
        nbr_offsets<T>(yl, ny, rowb, yo);
        pull_d2q9(a.fin, n, xo, yo, g[q]);
    }
    for (int j0 = 0; j0 < nrows; j0 += W) {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int j = j0 + s;
            if (j < nrows) {   // uniform across the block
                if (j + PF < nrows) {
                    yl = yl == ny - 1 ? 0 : yl + 1;
                    uint32_t yo[3];
                    nbr_offsets<T>(yl, ny, rowb, yo);
                    pull_d2q9(a.fin, n, xo, yo, g[(s + PF) % W]);
                }
                const T dr = sum9(g[s]);
                psi_s[(j % NS) * NT + t] = psi_of(a.rho_ref + dr, a);
                __syncthreads();
                if (j >= 2 * R && interior) {
                    const int sc = (s + W - R) % W;     // slot of row j - R
                    const int yrel = j - 2 * R;
                    const int yr = y0 + yrel;
                    int sl[2 * R + 1];
#pragma unroll
                    for (int d = -R; d <= R; ++d) sl[d + R] = ((j - R + d) % NS) * NT + t;
                    T sx = T(0), sy = T(0), ax = T(0), ay = T(0);
#pragma unroll
                    for (int p = 0; p < ST::NP; ++p) {
                        constexpr PairList P = ST::P;
                        const int ex = P.e[p][0], ey = P.e[p][1];
                        const T d = psi_s[sl[R + ey] + ex] - psi_s[sl[R - ey] - ex];
                        if (ex) ax += T(ex) * d;
                        if (ey) ay += T(ey) * d;
                        if (P.shell_end(p)) {
                            sx += T(P.w[p]) * ax;
                            sy += T(P.w[p]) * ay;
                            ax = ay = T(0);
                        }
                    }
                    const T pref = -a.gc0 * psi_s[sl[R]];
                    const T drc = sum9(g[sc]);
                    collide_d2q9_srt(g[sc], drc, pref * sx, pref * sy, a);
                    if (yrel < H && yr < ny) {
                        const uint32_t off = (uint32_t)yr * rowb + (uint32_t)xr * TS;
#pragma unroll
                        for (int b = 0; b < 9; ++b) st_off(a.fout + b * n, off, g[sc][b]);
                    }
                }
            }
        }
    }
}

template <typename T, int ORDER, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_d2q9_tile2(StepArgs<T> a, int nbx, int nby, int sw)
{
    using LD = Tile2Lds<Stencil<2, ORDER>::R, TX, TY>;
    __shared__ T psi1[LD::P1N];
    __shared__ T psi2[LD::P2N];
    __shared__ T s1[9 * LD::C1N];
    int bx, by;
    strip_tile(xcd_swizzle(blockIdx.x, gridDim.x), nbx, nby, sw, bx, by);
    d2q9_tile2_body<T, ORDER, TX, TY, NT, true>(a, bx * TX, by * TY, psi1, psi2, s1);
}

// ------------------------------------------------------------ dispatch ----
struct Shape2D {
    const char* name;
};
static const Shape2D kShapes2D[] = {
    {"tile64x16r4"}, {"tile64x8r2"}, {"tile32x8r1"}, {"tile64x4r1"},
    {"march256h128"}, {"march256h128pf2"}, {"march512h128"}, {"march256h128pf3"}, {"march512h128pf2"},
    {"tile2x16x16"}, {"tile2x32x8"}, {"tile2x32x16"}, {"tile2x64x8"}, {"tile2x64x16"}, {"tile2x32x32"},
    {"tile2x32x8t512"}, {"tile2x32x8t1024"},
};
constexpr int kNumShapes2D = sizeof(kShapes2D) / sizeof(kShapes2D[0]);

int num_variants_d2q9() { return kNumShapes2D; }
int variant_steps_d2q9(int v) { return (v >= 9 && v <= 16) ? 2 : 1; }
const char* variant_name_d2q9(int v) { return (v >= 0 && v < kNumShapes2D) ? kShapes2D[v].name : "?"; }

template <typename T, int ORDER, int TX, int TY, int RPT>
static hipError_t launch_tile(const StepArgs<T>& a, hipStream_t s)
{
    const int nbx = (a.nx + TX - 1) / TX, nby = (a.ny + TY - 1) / TY;
    dim3 block(TX, TY / RPT);
    hipLaunchKernelGGL((k_d2q9_tile<T, ORDER, TX, TY, RPT>), dim3(nbx * nby), block, 0, s, a, nbx, nby,
                       kStripTiles);
    return hipGetLastError();
}

template <typename T, int ORDER, int TX, int TY, int NT = TX * TY>
static hipError_t launch_tile2(const StepArgs<T>& a, hipStream_t s)
{
    const int nbx = (a.nx + TX - 1) / TX, nby = (a.ny + TY - 1) / TY;
    hipLaunchKernelGGL((k_d2q9_tile2<T, ORDER, TX, TY, NT>), dim3(nbx * nby), dim3(NT), 0, s, a, nbx, nby,
                       kStripTiles);
    return hipGetLastError();
}

template <typename T, int ORDER, int NT, int PF>
static hipError_t launch_march(const StepArgs<T>& a, int H, hipStream_t s)
{
    constexpr int R = Stencil<2, ORDER>::R;
    constexpr int TXO = NT - 2 * R;
    if (H > a.ny) H = a.ny;
    const int nbx = (a.nx + TXO - 1) / TXO, nby = (a.ny + H - 1) / H;
    hipLaunchKernelGGL((k_d2q9_march<T, ORDER, NT, PF>), dim3(nbx * nby), dim3(NT), 0, s, a, H, nbx);
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
    case 4: return launch_march<T, ORDER, 256, 1>(a, 128, s);
    case 5: return launch_march<T, ORDER, 256, 2>(a, 128, s);
    case 6: return launch_march<T, ORDER, 512, 1>(a, 128, s);
    case 7: return launch_march<T, ORDER, 256, 3>(a, 128, s);
    case 8: return launch_march<T, ORDER, 512, 2>(a, 128, s);
    case 9: return launch_tile2<T, ORDER, 16, 16>(a, s);
    case 10: return launch_tile2<T, ORDER, 32, 8>(a, s);
    case 11: return launch_tile2<T, ORDER, 32, 16>(a, s);
    case 12: return launch_tile2<T, ORDER, 64, 8>(a, s);
    case 13: return launch_tile2<T, ORDER, 64, 16>(a, s);
    case 14: return launch_tile2<T, ORDER, 32, 32>(a, s);
    // more threads than tile nodes: more waves per CU and fewer halo nodes per
    // thread (the 256^2 grid has one 32 x 8 tile per CU)
    case 15: return launch_tile2<T, ORDER, 32, 8, 512>(a, s);
    case 16: return launch_tile2<T, ORDER, 32, 8, 1024>(a, s);
    // measured and dropped: 64 x 32 and 128 x 16 tiles with 1024 threads
    // (fewer halo nodes per tile node, but one block per CU); at 8192^2 the
    // tuner kept 64 x 16 (FP32) and 32 x 16 (FP64).  A 16 x 16 tile with
    // 1024 threads (11% fewer halo nodes than 32 x 8 at E8) took 2.85 us
    // per step at 256^2 against 2.59 for 32 x 8: its rows span half a
    // cache line.
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
