// kernels_3d.hip -- fused D3Q19 step for gfx950 (SRT or MRT, E4/E6/E8
// force stencil, Guo forcing, pull streaming).
//
// z-marching kernel: a block owns an x-y tile of TX x TY nodes (TX x TYB
// threads, RPT rows per thread) and a z range [z0, z0 + H).  It walks the
// planes z0 - R ... z0 + H + R - 1; for each plane it pulls the 19 values of
// its tile nodes (kept in registers), writes psi for the tile plus a ring of
// width R into a slot of an LDS ring buffer of 2R + 2 planes, and -- once
// the psi planes z - R ... z + R are resident -- computes F, collides and
// stores plane z = (current - R).  The f registers of the last R + 1 planes
// rotate through a statically indexed window (the z loop is unrolled by
// R + 1), so each tile node is read from HBM once per step; only the halo
// ring and the 2R extra planes per block are pulled twice (L2 hits).
// One barrier per plane: the 2R + 2 slots keep the next write away from the
// 2R + 1 planes still being read.
#include <algorithm>

#include "kernels.h"

namespace sclbm {

template <typename T>
__device__ __forceinline__ void pull_d3q19(const T* __restrict__ f, int64_t n, uint32_t zb, const uint32_t (&zo)[3],
                                           const uint32_t (&yo)[3], const uint32_t (&xo)[3], T (&g)[19])
{
    (void)zb;
#pragma unroll
    for (int b = 0; b < 19; ++b)
        g[b] = ld_off(f + b * n, zo[1 - D3Q19::cz[b]] + yo[1 - D3Q19::cy[b]] + xo[1 - D3Q19::cx[b]]);
}

// LDS of one march block: the psi ring
template <typename T, int ORDER, int TX, int TYB, int RPT>
constexpr int march_lds_floats()
{
    using ST = Stencil<3, ORDER>;
    return (2 * ST::R + 2) * (TX + 2 * ST::R) * (TYB * RPT + 2 * ST::R);
}

// One block's march over logical column segment L (x tile fastest, then y
// tile, then z segment).
template <typename T, int ORDER, bool MRT, int TX, int TYB, int RPT, int PF>
__device__ __forceinline__ void march_item(const StepArgs<T>& a, int H, int nbx, int nby, int L, T* __restrict__ psi_s)
{
    using ST = Stencil<3, ORDER>;
    constexpr int R = ST::R;
    constexpr int TY = TYB * RPT;
    constexpr int LW = TX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int PL = LW * LH;          // one psi plane
    constexpr int NS = 2 * R + 2;        // psi ring slots
    constexpr int NT = TX * TYB;
    constexpr int W = R + 1 + PF;        // f register window (PF = 1: next plane in flight)
    constexpr int RING = PL - TX * TY;   // halo nodes per plane
    constexpr int RPERT = (RING + NT - 1) / NT;

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t n = a.n;
    const uint32_t TS = sizeof(T), rowb = (uint32_t)nx * TS, planeb = (uint32_t)ny * rowb;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    const int x0 = (L % nbx) * TX, y0 = ((L / nbx) % nby) * TY, z0 = (L / (nbx * nby)) * H;

    const int xr = x0 + tx;
    const bool xin = xr < nx;
    uint32_t xo[3];
    nbr_offsets<T>(xin ? xr : xr % nx, nx, TS, xo);
    uint32_t yo[RPT][3];
    bool yin[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int yr = y0 + ty * RPT + k;
        yin[k] = yr < ny;
        nbr_offsets<T>(yr < ny ? yr : yr % ny, ny, rowb, yo[k]);
    }
    // this thread's halo-ring nodes (same in every plane): LDS index and offsets
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
            const int jj = i - R * LW;
            ly = TY + R + jj / LW;
            lx = jj % LW;
        } else if (i < RING) {
            const int jj = i - 2 * R * LW;
            ly = R + jj / (2 * R);
            const int c = jj % (2 * R);
            lx = c < R ? c : TX + c;
        }
        rl[q] = i < RING ? ly * LW + lx : -1;
        nbr_offsets<T>(wrap_near(x0 - R + lx, nx), nx, TS, rxo[q]);
        nbr_offsets<T>(wrap_near(y0 - R + ly, ny), ny, rowb, ryo[q]);
    }

    T g[W][RPT][19];
    T dr[W][RPT];
    T h[RPERT][19];
    const int nplanes = H + 2 * R;
    int zc = wrap_any(z0 - R, nz);   // plane whose pulls are issued next

    // pulls of one plane (tile nodes into register slot `gs`, ring nodes into h)
    auto issue = [&](T (&gs)[RPT][19]) {
        uint32_t zo[3];
        nbr_offsets<T>(zc, nz, planeb, zo);
#pragma unroll
        for (int k = 0; k < RPT; ++k) pull_d3q19(a.fin, n, 0u, zo, yo[k], xo, gs[k]);
#pragma unroll
        for (int q = 0; q < RPERT; ++q)
            if (rl[q] >= 0) pull_d3q19(a.fin, n, 0u, zo, ryo[q], rxo[q], h[q]);
        zc = zc == nz - 1 ? 0 : zc + 1;
    };
    if (PF) issue(g[0]);

    for (int j0 = 0; j0 < nplanes; j0 += W) {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int j = j0 + s;
            if (j < nplanes) {   // uniform across the block
                if (!PF) issue(g[s]);
                T* slot = psi_s + (j % NS) * PL;
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    dr[s][k] = sum19(g[s][k]);
                    slot[(ty * RPT + k + R) * LW + tx + R] = psi_of(a.rho_ref + dr[s][k], a);
                }
#pragma unroll
                for (int q = 0; q < RPERT; ++q)
                    if (rl[q] >= 0) slot[rl[q]] = psi_of(a.rho_ref + sum19(h[q]), a);
                if (PF && j + 1 < nplanes) issue(g[(s + 1) % W]);
                __syncthreads();

                if (j >= 2 * R) {
                    const int sc = (s + W - R) % W;      // register slot of plane j - R (static after unrolling)
                    const int zrel = j - 2 * R;          // 0 .. H-1
                    const int zr = z0 + zrel;
                    int sl[2 * R + 1];
#pragma unroll
                    for (int d = -R; d <= R; ++d) sl[d + R] = ((j - R + d) % NS) * PL;
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const int cidx = (ty * RPT + k + R) * LW + tx + R;
                        T sx = T(0), sy = T(0), sz = T(0), ax = T(0), ay = T(0), az = T(0);
#pragma unroll
                        for (int p = 0; p < ST::NP; ++p) {
                            constexpr PairList P = ST::P;
                            // keep the LDS reads in groups of 8 pairs so the
                            // scheduler cannot hoist all of them (registers)
                            if (p % 8 == 0 && p) __builtin_amdgcn_sched_barrier(0);
                            const int ex = P.e[p][0], ey = P.e[p][1], ez = P.e[p][2];
                            const T vp = psi_s[sl[R + ez] + cidx + ey * LW + ex];
                            const T vm = psi_s[sl[R - ez] + cidx - ey * LW - ex];
                            const T d = vp - vm;
                            if (ex) ax += T(ex) * d;
                            if (ey) ay += T(ey) * d;
                            if (ez) az += T(ez) * d;
                            if (P.shell_end(p)) {   // one weight per shell
                                sx += T(P.w[p]) * ax;
                                sy += T(P.w[p]) * ay;
                                sz += T(P.w[p]) * az;
                                ax = ay = az = T(0);
                            }
                        }
                        const T pref = -a.gc0 * psi_s[sl[R] + cidx];
                        collide_d3q19<T, MRT>(g[sc][k], dr[sc][k], pref * sx, pref * sy, pref * sz, a);
                        if (xin && yin[k] && zr < nz) {
                            const uint32_t off = (uint32_t)zr * planeb + yo[k][1] + xo[1];
#pragma unroll
                            for (int b = 0; b < 19; ++b) {
                                if constexpr (sizeof(T) == 8) st_off_nt(a.fout + b * n, off, g[sc][k][b]);
                                else st_off(a.fout + b * n, off, g[sc][k][b]);
                            }
                        }
                    }
                }
            }
        }
    }
}

template <typename T, int ORDER, bool MRT, int TX, int TYB, int RPT, int PF>
__global__ void __launch_bounds__(TX* TYB)
k_d3q19_march(StepArgs<T> a, int H, int nbx, int nby)
{
    __shared__ T psi_s[march_lds_floats<T, ORDER, TX, TYB, RPT>()];
    march_item<T, ORDER, MRT, TX, TYB, RPT, PF>(a, H, nbx, nby, xcd_swizzle(blockIdx.x, gridDim.x), psi_s);
}

// Persistent form: as many blocks as fit on the device at once, each taking
// column segments in generations of gridDim.x.  All blocks start together
// and every segment is the same work, so a generation's segments march in
// step; the XCD swizzle within a generation gives each XCD a compact patch
// of neighbouring columns.  A tile's halo ring, the edge rows of its
// neighbours, is then read while the neighbours hold those planes in the
// XCD's L2, not planes later, after it has been evicted.
template <typename T, int ORDER, bool MRT, int TX, int TYB, int RPT, int PF>
__global__ void __launch_bounds__(TX* TYB)
k_d3q19_march_p(StepArgs<T> a, int H, int nbx, int nby, int nitems)
{
    __shared__ T psi_s[march_lds_floats<T, ORDER, TX, TYB, RPT>()];
    const int nb = gridDim.x, b = blockIdx.x;
    for (int base = 0; base < nitems; base += nb) {
        const int r = nitems - base < nb ? nitems - base : nb;
        if (b >= r) break;   // uniform across the block
        if (base) __syncthreads();   // the previous segment's reads of the ring are done
        march_item<T, ORDER, MRT, TX, TYB, RPT, PF>(a, H, nbx, nby, base + xcd_swizzle(b, r), psi_s);
    }
}

// The same z-march without the register window: a tile node's 19 values are
// pulled twice, once when its plane enters the psi ring and again when the
// plane collides R planes later (then L2 hits: the block read those lines
// R planes before).  The window of R + 1 planes of 19 values is what holds
// k_d3q19_march at two waves per SIMD; without it the kernel fits WPE waves
// per SIMD, so more loads are in flight to cover their latency.  The same
// sum of the same 19 loaded values gives rho in both places, so psi and
// the collision see one density, as in k_d3q19_march.  One thread per
// column (TX x TY threads).
template <typename T, int ORDER, bool MRT, int TX, int TY, int WPE>
__global__ void __launch_bounds__(TX* TY, sizeof(T) == 8 ? (WPE + 1) / 2 : WPE)
k_d3q19_march_rl(StepArgs<T> a, int H, int nbx, int nby)
{
    using ST = Stencil<3, ORDER>;
    constexpr int R = ST::R;
    constexpr int LW = TX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int PL = LW * LH;
    constexpr int NS = 2 * R + 2;
    constexpr int NT = TX * TY;
    constexpr int RING = PL - TX * TY;
    constexpr int RPERT = (RING + NT - 1) / NT;
    __shared__ T psi_s[NS * PL];

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t n = a.n;
    const uint32_t TS = sizeof(T), rowb = (uint32_t)nx * TS, planeb = (uint32_t)ny * rowb;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    const int L = xcd_swizzle(blockIdx.x, gridDim.x);
    const int x0 = (L % nbx) * TX, y0 = ((L / nbx) % nby) * TY, z0 = (L / (nbx * nby)) * H;

    const int xr = x0 + tx, yr = y0 + ty;
    const bool inxy = xr < nx && yr < ny;
    uint32_t xo[3], yo[3];
    nbr_offsets<T>(xr < nx ? xr : xr % nx, nx, TS, xo);
    nbr_offsets<T>(yr < ny ? yr : yr % ny, ny, rowb, yo);
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
            const int jj = i - R * LW;
            ly = TY + R + jj / LW;
            lx = jj % LW;
        } else if (i < RING) {
            const int jj = i - 2 * R * LW;
            ly = R + jj / (2 * R);
            const int c = jj % (2 * R);
            lx = c < R ? c : TX + c;
        }
        rl[q] = i < RING ? ly * LW + lx : -1;
        nbr_offsets<T>(wrap_near(x0 - R + lx, nx), nx, TS, rxo[q]);
        nbr_offsets<T>(wrap_near(y0 - R + ly, ny), ny, rowb, ryo[q]);
    }

    const int cidx = (ty + R) * LW + tx + R;
    const int nplanes = H + 2 * R;
    int zp = wrap_any(z0 - R, nz);   // plane entering the psi ring
    for (int j = 0; j < nplanes; ++j) {
        const bool col = j >= 2 * R;
        const int zr = z0 + j - 2 * R;   // plane that collides in this pass
        T gc[19];
        if (col) {   // uniform across the block
            uint32_t zo[3];
            nbr_offsets<T>(zr < nz ? zr : zr - nz, nz, planeb, zo);
            pull_d3q19(a.fin, n, 0u, zo, yo, xo, gc);
        }
        {
            T gt[19], h[RPERT][19];
            uint32_t zo[3];
            nbr_offsets<T>(zp, nz, planeb, zo);
            pull_d3q19(a.fin, n, 0u, zo, yo, xo, gt);
#pragma unroll
            for (int q = 0; q < RPERT; ++q)
                if (rl[q] >= 0) pull_d3q19(a.fin, n, 0u, zo, ryo[q], rxo[q], h[q]);
            T* slot = psi_s + (j % NS) * PL;
            slot[cidx] = psi_of(a.rho_ref + sum19(gt), a);
#pragma unroll
            for (int q = 0; q < RPERT; ++q)
                if (rl[q] >= 0) slot[rl[q]] = psi_of(a.rho_ref + sum19(h[q]), a);
        }
        zp = zp == nz - 1 ? 0 : zp + 1;
        __syncthreads();
        if (col) {
            int sl[2 * R + 1];
#pragma unroll
            for (int d = -R; d <= R; ++d) sl[d + R] = ((j - R + d) % NS) * PL;
            T sx = T(0), sy = T(0), sz = T(0), ax = T(0), ay = T(0), az = T(0);
#pragma unroll
            for (int p = 0; p < ST::NP; ++p) {
                constexpr PairList P = ST::P;
                if (p % 8 == 0 && p) __builtin_amdgcn_sched_barrier(0);
                const int ex = P.e[p][0], ey = P.e[p][1], ez = P.e[p][2];
                const T vp = psi_s[sl[R + ez] + cidx + ey * LW + ex];
                const T vm = psi_s[sl[R - ez] + cidx - ey * LW - ex];
                const T d = vp - vm;
                if (ex) ax += T(ex) * d;
                if (ey) ay += T(ey) * d;
                if (ez) az += T(ez) * d;
                if (P.shell_end(p)) {
                    sx += T(P.w[p]) * ax;
                    sy += T(P.w[p]) * ay;
                    sz += T(P.w[p]) * az;
                    ax = ay = az = T(0);
                }
            }
            const T pref = -a.gc0 * psi_s[sl[R] + cidx];
            collide_d3q19<T, MRT>(gc, sum19(gc), pref * sx, pref * sy, pref * sz, a);
            if (inxy && zr < nz) {
                const uint32_t off = (uint32_t)zr * planeb + yo[1] + xo[1];
#pragma unroll
                for (int b = 0; b < 19; ++b) {
                    if constexpr (sizeof(T) == 8) st_off_nt(a.fout + b * n, off, gc[b]);
                    else st_off(a.fout + b * n, off, gc[b]);
                }
            }
        }
    }
}

// ------------------------------------------------------------ dispatch ----
struct Shape3D {
    int tx, tyb, rpt, h;
    const char* name;
};
static const Shape3D kShapes3D[] = {
    {32, 8, 2, 16, "march32x16h16"},
    {64, 4, 2, 16, "march64x8h16"},
    {32, 8, 1, 16, "march32x8h16"},
    {32, 8, 2, 32, "march32x16h32"},
    {32, 16, 1, 16, "march32x16r1h16"},
    {64, 8, 1, 16, "march64x8r1h16"},
    {32, 16, 1, 32, "march32x16r1h32"},
    {64, 8, 1, 16, "march64x8r1h16pf1"},
    {64, 8, 1, 32, "march64x8r1h32pf1"},
    {64, 8, 2, 32, "march64x16h32"},
    {64, 8, 1, 64, "march64x8r1h64pf1"},
    {32, 8, 1, 32, "march32x8r1h32pf1"},
    {32, 8, 1, 64, "march32x8r1h64pf1"},
    // 768 threads: three waves per SIMD at up to 168 VGPRs (the MRT E8
    // window needs ~153), and a halo ring of 0.42 nodes per tile node
    {64, 12, 1, 64, "march64x12r1h64pf1"},
    {64, 12, 1, 32, "march64x12r1h32pf1"},
    {64, 12, 1, 16, "march64x12r1h16pf1"},
    // k_d3q19_march_rl (pulls twice, no register window); rpt holds the
    // waves per SIMD the FP32 kernel is built for (FP64: half, rounded up).
    // At 320^3 the FP64 state runs 3-5% faster than on any window shape;
    // the FP32 state 25% slower (the second pulls miss L2 in part)
    {64, 8, 4, 64, "rl64x8h64w4"},
    {64, 8, 4, 32, "rl64x8h32w4"},
    // persistent k_d3q19_march_p (segments in generations of resident blocks):
    // 7% faster than the one-segment-per-block launch at 320^3 (FP32 MRT E8,
    // fetch 1.32 vs 1.37 of the algorithmic reads) and 6% at 128^3; the
    // 64 x 12 and 32 x 8 tiles were slower in this form too, and so was a
    // strip order of the segments (1 or 2 tile columns per strip: 4% and 2%
    // slower at 320^3, the x halo then crossing XCDs)
    {64, 8, 1, 64, "pmarch64x8r1h64pf1"},
    {64, 8, 1, 32, "pmarch64x8r1h32pf1"},
    {64, 8, 1, 16, "pmarch64x8r1h16pf1"},
    // the persistent form of the 256-thread window march, whose FP64
    // window fits in registers (256 VGPRs, two waves per SIMD): the FP64
    // state at 320^3 runs within 1% of the re-pull march (3.35-3.39 ms per
    // step) and fetches 1.40 of the algorithmic reads against 2.54
    {32, 8, 1, 64, "pmarch32x8r1h64pf1"},
    {32, 8, 1, 32, "pmarch32x8r1h32pf1"},
};
constexpr int kNumShapes3D = sizeof(kShapes3D) / sizeof(kShapes3D[0]);

int num_variants_d3q19() { return kNumShapes3D; }
const char* variant_name_d3q19(int v) { return (v >= 0 && v < kNumShapes3D) ? kShapes3D[v].name : "?"; }

template <typename T, int ORDER, bool MRT, int TX, int TYB, int RPT, int PF = 0>
static hipError_t launch_march(const StepArgs<T>& a, int H, hipStream_t s)
{
    if (H > a.nz) H = a.nz;
    dim3 block(TX, TYB);
    const int nbx = (a.nx + TX - 1) / TX, nby = (a.ny + TYB * RPT - 1) / (TYB * RPT);
    const int nbz = (a.nz + H - 1) / H;
    hipLaunchKernelGGL((k_d3q19_march<T, ORDER, MRT, TX, TYB, RPT, PF>), dim3(nbx * nby * nbz), block, 0, s,
                       a, H, nbx, nby);
    return hipGetLastError();
}

// persistent march: one generation of blocks is what the device holds at once
template <typename T, int ORDER, bool MRT, int TX, int TYB, int RPT, int PF>
static hipError_t launch_march_p(const StepArgs<T>& a, int H, hipStream_t s)
{
    if (H > a.nz) H = a.nz;
    const int nbx = (a.nx + TX - 1) / TX, nby = (a.ny + TYB * RPT - 1) / (TYB * RPT);
    const int nitems = nbx * nby * ((a.nz + H - 1) / H);
    static int per_cu = 0, cus = 0;   // per process: one device type
    if (!per_cu) {
        int dev = 0, n = 0, c = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_d3q19_march_p<T, ORDER, MRT, TX, TYB, RPT, PF>,
                                                         TX * TYB, 0) == hipSuccess &&
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0 && c > 0) {
            cus = c;
            per_cu = n;
        } else {
            return hipErrorUnknown;
        }
    }
    const int nb = std::min(nitems, per_cu * cus);
    hipLaunchKernelGGL((k_d3q19_march_p<T, ORDER, MRT, TX, TYB, RPT, PF>), dim3(nb), dim3(TX, TYB), 0, s, a, H, nbx,
                       nby, nitems);
    return hipGetLastError();
}

template <typename T, int ORDER, bool MRT, int TX, int TY, int WPE>
static hipError_t launch_march_rl(const StepArgs<T>& a, int H, hipStream_t s)
{
    if (H > a.nz) H = a.nz;
    const int nbx = (a.nx + TX - 1) / TX, nby = (a.ny + TY - 1) / TY, nbz = (a.nz + H - 1) / H;
    hipLaunchKernelGGL((k_d3q19_march_rl<T, ORDER, MRT, TX, TY, WPE>), dim3(nbx * nby * nbz), dim3(TX, TY), 0, s, a,
                       H, nbx, nby);
    return hipGetLastError();
}

template <typename T, int ORDER, bool MRT>
static hipError_t launch_v(const StepArgs<T>& a, int variant, hipStream_t s)
{
    switch (variant) {
    case 0: return launch_march<T, ORDER, MRT, 32, 8, 2>(a, 16, s);
    case 1: return launch_march<T, ORDER, MRT, 64, 4, 2>(a, 16, s);
    case 2: return launch_march<T, ORDER, MRT, 32, 8, 1>(a, 16, s);
    case 3: return launch_march<T, ORDER, MRT, 32, 8, 2>(a, 32, s);
    case 4: return launch_march<T, ORDER, MRT, 32, 16, 1>(a, 16, s);
    case 5: return launch_march<T, ORDER, MRT, 64, 8, 1>(a, 16, s);
    case 6: return launch_march<T, ORDER, MRT, 32, 16, 1>(a, 32, s);
    case 7: return launch_march<T, ORDER, MRT, 64, 8, 1, 1>(a, 16, s);
    case 8: return launch_march<T, ORDER, MRT, 64, 8, 1, 1>(a, 32, s);
    case 9: return launch_march<T, ORDER, MRT, 64, 8, 2, 0>(a, 32, s);
    case 10: return launch_march<T, ORDER, MRT, 64, 8, 1, 1>(a, 64, s);
    // 256 threads with the prefetch window: room for the FP64 window without spills
    case 11: return launch_march<T, ORDER, MRT, 32, 8, 1, 1>(a, 32, s);
    case 12: return launch_march<T, ORDER, MRT, 32, 8, 1, 1>(a, 64, s);
    case 13: return launch_march<T, ORDER, MRT, 64, 12, 1, 1>(a, 64, s);
    case 14: return launch_march<T, ORDER, MRT, 64, 12, 1, 1>(a, 32, s);
    case 15: return launch_march<T, ORDER, MRT, 64, 12, 1, 1>(a, 16, s);
    case 16: return launch_march_rl<T, ORDER, MRT, 64, 8, 4>(a, 64, s);
    case 17: return launch_march_rl<T, ORDER, MRT, 64, 8, 4>(a, 32, s);
    case 18: return launch_march_p<T, ORDER, MRT, 64, 8, 1, 1>(a, 64, s);
    case 19: return launch_march_p<T, ORDER, MRT, 64, 8, 1, 1>(a, 32, s);
    case 20: return launch_march_p<T, ORDER, MRT, 64, 8, 1, 1>(a, 16, s);
    case 21: return launch_march_p<T, ORDER, MRT, 32, 8, 1, 1>(a, 64, s);
    case 22: return launch_march_p<T, ORDER, MRT, 32, 8, 1, 1>(a, 32, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_any(const StepArgs<T>& a, int order, bool mrt, int variant, hipStream_t s)
{
    switch (order) {
    case 4: return mrt ? launch_v<T, 4, true>(a, variant, s) : launch_v<T, 4, false>(a, variant, s);
    case 6: return mrt ? launch_v<T, 6, true>(a, variant, s) : launch_v<T, 6, false>(a, variant, s);
    case 8: return mrt ? launch_v<T, 8, true>(a, variant, s) : launch_v<T, 8, false>(a, variant, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_d3q19(const StepArgs<float>& a, int order, bool mrt, int variant, hipStream_t s)
{
    return launch_any<float>(a, order, mrt, variant, s);
}
hipError_t launch_step_d3q19(const StepArgs<double>& a, int order, bool mrt, int variant, hipStream_t s)
{
    return launch_any<double>(a, order, mrt, variant, s);
}

}  // namespace sclbm
