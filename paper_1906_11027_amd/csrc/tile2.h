// tile2.h -- two D2Q9 time steps per tile (temporal blocking), shared by
// the single-grid kernel (kernels_2d.hip) and the batched sweep kernel
// (kernels_batch.hip).
#pragma once
#include "kernels.h"

namespace sclbm {

// Two time steps per launch (temporal blocking) for small, latency-bound
// grids, where the launch itself costs as much as a step.  A block owns a
// TX x TY tile and computes, with R the force-stencil radius:
//   phase 1  psi at t+1 on the tile + (2R+1) halo: pull the 9 values of each
//            node from the state (kept in registers), sum, psi -> LDS psi1;
//   phase 2  step t -> t+1 on the tile + (R+1) halo, a sub-region of the
//            first: force from psi1, collide the registers -> LDS s1;
//   phase 3  psi at t+2 on the tile + R halo, pulling from s1 -> LDS psi2;
//   phase 4  step t+1 -> t+2 on the tile: pull from s1, force from psi2,
//            collide, store.
// The halo nodes are recomputed by the neighbouring tiles (about 1.9x the
// node updates at 16 x 16), so this shape pays off only where launches
// dominate.  Every region is walked by a bounded loop over its node count;
// nodes outside the grid are computed on wrapped coordinates and not stored.
// LDS regions of the two-step tile (values of T): psi at t+1 on the tile +
// (2R+1), the post-collision copy s1 of 9 planes on the tile + (R+1), psi at
// t+2 on the tile + R.
template <int R, int TX, int TY>
struct Tile2Lds {
    static constexpr int H1 = 2 * R + 1, P1W = TX + 2 * H1, P1H = TY + 2 * H1, P1N = P1W * P1H;
    static constexpr int HC = R + 1, C1W = TX + 2 * HC, C1H = TY + 2 * HC, C1N = C1W * C1H;
    static constexpr int P2W = TX + 2 * R, P2H = TY + 2 * R, P2N = P2W * P2H;
};

// The two steps of one tile at origin (x0, y0); psi1, psi2 and s1 point to
// LDS of at least the sizes of Tile2Lds<R, TX, TY>.  Every thread of the
// NT-thread block calls it (barriers inside).  NTSTORE marks the output
// stores non-temporal (the single-grid kernel; the batched sweep keeps
// plain stores).
template <typename T, int ORDER, int TX, int TY, int NT, bool NTSTORE = false>
__device__ __forceinline__ void d2q9_tile2_body(const StepArgs<T>& a, int x0, int y0, T* __restrict__ psi1,
                                                T* __restrict__ psi2, T* __restrict__ s1)
{
    using ST = Stencil<2, ORDER>;
    constexpr int R = ST::R;
    using LD = Tile2Lds<R, TX, TY>;
    constexpr int H1 = LD::H1, P1W = LD::P1W, P1N = LD::P1N;
    constexpr int HC = LD::HC, C1W = LD::C1W, C1H = LD::C1H, C1N = LD::C1N;
    constexpr int P2W = LD::P2W, P2N = LD::P2N;

    const int nx = a.nx, ny = a.ny;
    const int64_t n = a.n;
    const uint32_t TS = sizeof(T), rowb = (uint32_t)nx * TS;
    const int tid = threadIdx.x;

    auto pull_global = [&](int gx, int gy, T (&g)[9]) {
        uint32_t xo[3], yo[3];
        nbr_offsets<T>(wrap_near(gx, nx), nx, TS, xo);
        nbr_offsets<T>(wrap_near(gy, ny), ny, rowb, yo);
        pull_d2q9(a.fin, n, xo, yo, g);
    };
    auto force_at = [&](const T* c, int LW, T& Fx, T& Fy) {
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
        Fx = pref * sx;
        Fy = pref * sy;
    };

    // phase 1: psi at t+1 on the tile + (2R+1) halo.  The per-thread node
    // loop has a compile-time bound and is unrolled, so the pulls of all its
    // nodes are in flight together.  The pulled values stay in registers for
    // phase 2, whose (R+1)-halo region lies inside this one.
    // A tile whose pulled region lies inside the grid (one test per block)
    // takes its addresses without wrapping.
    constexpr int K1 = (P1N + NT - 1) / NT;
    T g[K1][9];
    {
        if (x0 > H1 && x0 + TX + H1 < nx && y0 > H1 && y0 + TY + H1 < ny) {
#pragma unroll
            for (int q = 0; q < K1; ++q) {
                const int i = tid + q * NT;
                if (i < P1N) {
                    const int ly = i / P1W, lx = i - ly * P1W;
                    const uint32_t own = (uint32_t)(y0 - H1 + ly) * rowb + (uint32_t)(x0 - H1 + lx) * TS;
#pragma unroll
                    for (int b = 0; b < 9; ++b)
                        g[q][b] = ld_off(a.fin + b * n, own - (uint32_t)D2Q9::cy[b] * rowb -
                                                            (uint32_t)(D2Q9::cx[b] * (int)TS));
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < K1; ++q) {
                const int i = tid + q * NT;
                if (i < P1N) {
                    const int ly = i / P1W, lx = i - ly * P1W;
                    pull_global(x0 - H1 + lx, y0 - H1 + ly, g[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < K1; ++q) {
            const int i = tid + q * NT;
            if (i < P1N) psi1[i] = psi_of(a.rho_ref + sum9(g[q]), a);
        }
    }
    __syncthreads();
    // phase 2: step t -> t+1 on the tile + (R+1) halo, from the phase-1
    // registers of the nodes in that region (offset R inside the psi1 region)
#pragma unroll
    for (int q = 0; q < K1; ++q) {
        const int i = tid + q * NT;
        if (i < P1N) {
            const int ly = i / P1W, lx = i - ly * P1W;
            const int cx = lx - R, cy = ly - R;
            if (cx >= 0 && cx < C1W && cy >= 0 && cy < C1H) {
                T Fx, Fy;
                force_at(psi1 + ly * P1W + lx, P1W, Fx, Fy);
                collide_d2q9_srt(g[q], sum9(g[q]), Fx, Fy, a);
                const int ci = cy * C1W + cx;
#pragma unroll
                for (int b = 0; b < 9; ++b) s1[b * C1N + ci] = g[q][b];
            }
        }
    }
    __syncthreads();
    // pull at t+2 of the node at s1 coordinates (cx, cy): value b from (cx - c_b, cy - c_b)
    auto pull_s1 = [&](int cx, int cy, T (&g)[9]) {
#pragma unroll
        for (int b = 0; b < 9; ++b) g[b] = s1[b * C1N + (cy - D2Q9::cy[b]) * C1W + cx - D2Q9::cx[b]];
    };
    // phase 3: psi at t+2 on the tile + R halo
    constexpr int K3 = (P2N + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < K3; ++q) {
        const int i = tid + q * NT;
        if (i < P2N) {
            const int ly = i / P2W, lx = i - ly * P2W;
            T g[9];
            pull_s1(lx + 1, ly + 1, g);
            psi2[i] = psi_of(a.rho_ref + sum9(g), a);
        }
    }
    __syncthreads();
    // phase 4: step t+1 -> t+2 on the tile, store
    constexpr int K4 = (TX * TY + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < K4; ++q) {
        const int i = tid + q * NT;
        if (i >= TX * TY) break;
        const int lx = i % TX, ly = i / TX;
        T g[9];
        pull_s1(lx + HC, ly + HC, g);
        T Fx, Fy;
        force_at(psi2 + (ly + R) * P2W + lx + R, P2W, Fx, Fy);
        collide_d2q9_srt(g, sum9(g), Fx, Fy, a);
        const int xr = x0 + lx, yr = y0 + ly;
        if (xr < nx && yr < ny) {
            const uint32_t off = (uint32_t)yr * rowb + (uint32_t)xr * TS;
#pragma unroll
            for (int b = 0; b < 9; ++b) {
                if constexpr (NTSTORE) st_off_nt(a.fout + b * n, off, g[b]);
                else st_off(a.fout + b * n, off, g[b]);
            }
        }
    }
}

}  // namespace sclbm
