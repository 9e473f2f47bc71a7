// wide2d.h -- fused step for any 2D lattice of lattice.h (D2Q9, D2Q13,
// D2Q25), Guo forcing or the exact difference method, for gfx950.
//
// The larger velocity sets of Sec. 3 (Table 1) keep the equilibrium and
// forcing of the nearest-neighbour model with their own weights and cs^2,
// and stream over distance 2.  The kernel is the tile scheme of the D2Q9
// path written for a lattice template: a block owns a TX x TY tile, each
// thread RPT rows of one column;
//   phase 1  pull the Q values of the owned nodes into registers (reach M =
//            max |c_i| = 1 or 2, so 2M + 1 wrapped row and column offsets),
//            form rho and psi, write psi to LDS; then fill the psi halo ring
//            of the force stencil (radius R) by pulling and summing the ring
//            nodes' values one node at a time (L2 hits: the neighbouring
//            tiles' lines);
//   phase 2  interaction force from LDS (Sec. 2, Eq. (1), summed over +-e
//            pairs), collision with Guo forcing (Eq. (3)-(4)) or the exact
//            difference method (Sec. 3), coalesced store at the own address.
// Ragged tiles: out-of-grid threads still supply wrapped psi and skip the
// store, so any nx, ny >= 1 works.
// Walls (WALLS = true): solid nodes put psi(rho_w) into the force (the
// virtual wall density of Sec. 3) and, instead of colliding, send back what
// arrived: g*_b = g_{-b} (standard bounce-back; the rest-weight shift is
// symmetric, so it commutes with the reversal).
#pragma once
#include "kernels.h"

namespace sclbm {

template <typename L>
constexpr int lattice_reach()
{
    int m = 0;
    for (int b = 0; b < L::Q; ++b) {
        const int ax = L::cx[b] < 0 ? -L::cx[b] : L::cx[b];
        const int ay = L::cy[b] < 0 ? -L::cy[b] : L::cy[b];
        if (ax > m) m = ax;
        if (ay > m) m = ay;
    }
    return m;
}

// byte offsets of the wrapped coordinates v - M ... v + M of an axis of n nodes
template <int M>
__device__ __forceinline__ void offsets_m(int v, int n, uint32_t stride, uint32_t (&o)[2 * M + 1])
{
#pragma unroll
    for (int k = 0; k <= 2 * M; ++k) {
        int c = v - M + k;
        c = wrap_near(c, n);
        o[k] = (uint32_t)c * stride;
    }
}

// value b of node (x, y) comes from (x - cx_b, y - cy_b)
template <typename T, typename L, int M>
__device__ __forceinline__ void pull_lat(const T* __restrict__ f, int64_t n, const uint32_t (&xo)[2 * M + 1],
                                         const uint32_t (&yo)[2 * M + 1], T (&g)[L::Q])
{
#pragma unroll
    for (int b = 0; b < L::Q; ++b) g[b] = ld_off(f + b * n, yo[M - L::cy[b]] + xo[M - L::cx[b]]);
}

// the same pull for a node whose neighbours need no wrapping: own is the
// node's byte offset, rowb the byte stride of a row
template <typename T, typename L>
__device__ __forceinline__ void pull_lat_inner(const T* __restrict__ f, int64_t n, uint32_t own, uint32_t rowb,
                                               T (&g)[L::Q])
{
#pragma unroll
    for (int b = 0; b < L::Q; ++b)
        g[b] = ld_off(f + b * n, own - (uint32_t)L::cy[b] * rowb - (uint32_t)(L::cx[b] * (int)sizeof(T)));
}

// index of -c_b in the lattice's velocity list
template <typename L>
constexpr int opposite(int b)
{
    for (int k = 0; k < L::Q; ++k)
        if (L::cx[k] == -L::cx[b] && L::cy[k] == -L::cy[b]) return k;
    return b;
}

// pairwise sum of g[LO .. LO + N) in a fixed tree order
template <int LO, int N>
struct TreeSum {
    template <typename T, int Q>
    __device__ __forceinline__ static T of(const T (&g)[Q])
    {
        return TreeSum<LO, N / 2>::of(g) + TreeSum<LO + N / 2, N - N / 2>::of(g);
    }
};
template <int LO>
struct TreeSum<LO, 1> {
    template <typename T, int Q>
    __device__ __forceinline__ static T of(const T (&g)[Q])
    {
        return g[LO];
    }
};

// every moving velocity has an opposite of the same weight: b and
// opposite(b) differ, and the rest velocity is its own opposite
template <typename L>
constexpr bool has_opposite_pairs()
{
    for (int b = 1; b < L::Q; ++b) {
        const int m = opposite<L>(b);
        if (m < 1 || m == b || L::w[m] != L::w[b]) return false;
    }
    return true;
}

// Collision on shifted values g = f - w rho_ref, drho = rho - rho_ref.
//   Guo:  u = (j + F/2)/rho,  g* = g - (g - geq(u))/tau + (1 - 1/(2 tau)) phihat(u, F)
//   EDM:  v = j/rho, dv = F/rho,  g* = g - (g - geq(v))/tau + feq(v + dv) - feq(v)
// with feq = w rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u^2/(2 cs2)] and
// phihat = w [(c - u)/cs2 + (c.u) c / cs2^2] . F.  Over a pair of opposite
// velocities (b, -b) the relaxed equilibrium plus the source splits into a
// part even in c and a part odd in c, each a short polynomial in c.u and c.F
// (Guo) or c.v and c.s with s = v + dv (EDM), and
//   g*_{+-} = g_{+-} + (even +- odd - om g_{+-}).
// The EDM increment enters through (c.s)^2 - (c.v)^2 and s^2 - v^2, never as
// the difference of two computed equilibria.  Both conserve mass exactly.
// The rest population closes the balance in difference form,
//   g0* = g0 + sum_{b>=1} (g_b - g_b*),
// whose terms are the small collision increments: the only rounding left in
// the node's mass is that of the stored g0*, where summing the populations
// before and after would add the rounding of two Q-term sums of O(rho)
// values, repeated identically every step near a steady state.
template <typename T, typename L, bool EDM>
__device__ __forceinline__ void collide_lat(T (&g)[L::Q], T drho, T Fx, T Fy, const StepArgs<T>& a)
{
    constexpr int Q = L::Q;
    const T rho = a.rho_ref + drho;
    T jx = T(0), jy = T(0);
#pragma unroll
    for (int b = 1; b < Q; ++b) {
        const int m = opposite<L>(b);
        if (m < b) continue;
        const T d = g[b] - g[m];
        if (L::cx[b]) jx += T(L::cx[b]) * d;
        if (L::cy[b]) jy += T(L::cy[b]) * d;
    }
    const T inv = fast_rcp(rho);
    T dm = T(0);   // sum of g_b - g_b* over b >= 1
    constexpr double ics = 1.0 / L::cs2;
    constexpr double ics2h = 0.5 / (L::cs2 * L::cs2);
    const T om = a.omega;
    if (!EDM) {
        const T ux = (jx + T(0.5) * Fx) * inv;
        const T uy = (jy + T(0.5) * Fy) * inv;
        const T usq = T(0.5 * ics) * (ux * ux + uy * uy);
        const T uF = ux * Fx + uy * Fy;
        const T gu = a.guo;
        // om feq + gu phihat:  even  w [K0 + cu (a1 cu + a2 cF)],  odd  w (b1 cu + b2 cF)
        const T K0 = om * (drho - rho * usq) - gu * T(ics) * uF;
        const T a1 = om * rho * T(ics2h), a2 = gu * T(2.0 * ics2h);
        const T b1 = om * rho * T(ics), b2 = gu * T(ics);
#pragma unroll
        for (int b = 1; b < Q; ++b) {
            const int m = opposite<L>(b);
            if (m < b) continue;   // the pair was done from its first member
            const T cu = T(L::cx[b]) * ux + T(L::cy[b]) * uy;
            const T cF = T(L::cx[b]) * Fx + T(L::cy[b]) * Fy;
            const T w = T(L::w[b]);
            const T S = w * (K0 + cu * (a1 * cu + a2 * cF));
            const T A = w * (b1 * cu + b2 * cF);
            const T gp = g[b], gm = g[m];
            const T np = gp + ((S + A) - om * gp);
            const T nm = gm + ((S - A) - om * gm);
            dm += (gp - np) + (gm - nm);
            g[b] = np;
            g[m] = nm;
        }
    } else {
        const T vx = jx * inv, vy = jy * inv;
        const T sx = vx + Fx * inv, sy = vy + Fy * inv;   // s = v + F/rho
        const T vsq = T(0.5 * ics) * (vx * vx + vy * vy);
        const T ssq = T(0.5 * ics) * (sx * sx + sy * sy);
        // om feq(v) + feq(s) - feq(v):
        //   even  w [om drho + rho (ics2h t - K1)],  t = (c.s)^2 + (om - 1)(c.v)^2,
        //         K1 = (om - 1) vsq + ssq;
        //   odd   w rho ics (c.s + (om - 1) c.v)
        const T omm1 = om - T(1);
        const T K0 = om * drho;
        const T K1 = omm1 * vsq + ssq;
        const T ri = rho * T(ics);
#pragma unroll
        for (int b = 1; b < Q; ++b) {
            const int m = opposite<L>(b);
            if (m < b) continue;
            const T cv = T(L::cx[b]) * vx + T(L::cy[b]) * vy;
            const T cs = T(L::cx[b]) * sx + T(L::cy[b]) * sy;
            const T w = T(L::w[b]);
            const T q = omm1 * cv;
            const T S = w * (K0 + rho * (T(ics2h) * (cs * cs + q * cv) - K1));
            const T A = (w * ri) * (cs + q);
            const T gp = g[b], gm = g[m];
            const T np = gp + ((S + A) - om * gp);
            const T nm = gm + ((S - A) - om * gm);
            dm += (gp - np) + (gm - nm);
            g[b] = np;
            g[m] = nm;
        }
    }
    g[0] += dm;
}
static_assert(has_opposite_pairs<D2Q9>() && has_opposite_pairs<D2Q13>() && has_opposite_pairs<D2Q25>(),
              "every moving velocity needs an opposite of equal weight");

template <typename T, typename L, int ORDER, bool EDM, bool WALLS, int TX, int TY, int RPT>
__global__ void __launch_bounds__(TX*(TY / RPT))
k_wide_tile(StepArgs<T> a, int nbx, int nby, int sw)
{
    using ST = Stencil<2, ORDER>;
    constexpr int Q = L::Q;
    constexpr int M = lattice_reach<L>();
    constexpr int R = ST::R;
    constexpr int LW = TX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int NT = TX * (TY / RPT);
    constexpr int RING = LH * LW - TX * TY;
    __shared__ T psi_s[LH * LW];

    const int nx = a.nx, ny = a.ny;
    const int64_t n = a.n;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    int bx, by;
    strip_tile(xcd_swizzle(blockIdx.x, gridDim.x), nbx, nby, sw, bx, by);
    const int x0 = bx * TX, y0 = by * TY;

    const uint32_t TS = sizeof(T), rowb = (uint32_t)nx * TS;
    const int xr = x0 + tx;
    const bool xin = xr < nx;
    const int xw = xin ? xr : xr % nx;
    uint32_t xo[2 * M + 1];
    offsets_m<M>(xw, nx, TS, xo);

    T g[RPT][Q];
    uint32_t own[RPT];
    bool wall[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int yr = y0 + ty * RPT + k;
        const int yw = yr < ny ? yr : yr % ny;
        uint32_t yo[2 * M + 1];
        offsets_m<M>(yw, ny, rowb, yo);
        own[k] = yo[M] + xo[M];
        wall[k] = WALLS && a.solid[(int64_t)yw * nx + xw];
        pull_lat<T, L, M>(a.fin, n, xo, yo, g[k]);
    }
    T dr[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        dr[k] = TreeSum<0, Q>::of(g[k]);
        psi_s[(ty * RPT + k + R) * LW + tx + R] = wall[k] ? a.psi_w : psi_of(a.rho_ref + dr[k], a);
    }
    // halo ring: R rows above and below at full width, R columns each side
#pragma unroll 1
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
        const int hx = wrap_near(x0 - R + lx, nx), hy = wrap_near(y0 - R + ly, ny);
        if (WALLS && a.solid[(int64_t)hy * nx + hx]) {
            psi_s[ly * LW + lx] = a.psi_w;
            continue;
        }
        uint32_t hxo[2 * M + 1], hyo[2 * M + 1];
        offsets_m<M>(hx, nx, TS, hxo);
        offsets_m<M>(hy, ny, rowb, hyo);
        T h[Q];
        pull_lat<T, L, M>(a.fin, n, hxo, hyo, h);
        psi_s[ly * LW + lx] = psi_of(a.rho_ref + TreeSum<0, Q>::of(h), a);
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty * RPT + k;
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
        if (wall[k]) {
            T r[Q];
#pragma unroll
            for (int b = 0; b < Q; ++b) r[b] = g[k][opposite<L>(b)];
#pragma unroll
            for (int b = 0; b < Q; ++b) g[k][b] = r[b];
        } else {
            collide_lat<T, L, EDM>(g[k], dr[k], pref * sx, pref * sy, a);
        }
        if (xin && y0 + ly < ny) {
#pragma unroll
            for (int b = 0; b < Q; ++b) st_off(a.fout + b * n, own[k], g[k][b]);
        }
    }
}

// Two time steps per launch (temporal blocking), any lattice without walls.
// A block owns a TX x TY tile; with R the force-stencil radius and M the
// lattice's reach:
//   phase 1  psi at t+1 on the tile + (2R + M): pull each node's Q values
//            from the state (kept in registers), sum, psi -> LDS psi1;
//   phase 2  step t -> t+1 on the tile + (R + M), a sub-region of the first:
//            force from psi1, collide the registers -> LDS copy s1 of the
//            post-collision values;
//   phase 3  psi at t+2 on the tile + R, pulled from s1 -> LDS psi2;
//   phase 4  step t+1 -> t+2 on the tile: pull from s1, force from psi2,
//            collide, store.
// The state is read and written once per two updates; the (R + M) halo of
// phase 2 is collided again by the neighbouring tiles.
// The LDS copy s1 keeps each population only where phases 3 and 4 pull it:
// population b of the node at phase-2 coordinates (cx, cy) is pulled by the
// phase-3 node (cx + c_bx - M, cy + c_by - M), so plane b is the psi2 region
// (P2W x P2H) shifted by (M - c_b).  A pull then reads every plane at the
// pulling node's own psi2 index, and s1 holds Q P2N values instead of Q C1N.
template <int Q, int R, int M, int TX, int TY>
struct WideTile2 {
    static constexpr int H1 = 2 * R + M, P1W = TX + 2 * H1, P1H = TY + 2 * H1, P1N = P1W * P1H;
    static constexpr int HC = R + M, C1W = TX + 2 * HC, C1H = TY + 2 * HC, C1N = C1W * C1H;
    static constexpr int P2W = TX + 2 * R, P2H = TY + 2 * R, P2N = P2W * P2H;
    template <typename T>
    static constexpr size_t lds_bytes()
    {
        return sizeof(T) * ((size_t)P1N + P2N + (size_t)Q * P2N);
    }
};

template <typename T, int ORDER>
__device__ __forceinline__ void wide_force_at(const T* c, int LW, T gc0, T& Fx, T& Fy)
{
    using ST = Stencil<2, ORDER>;
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
    const T pref = -gc0 * c[0];
    Fx = pref * sx;
    Fy = pref * sy;
}

template <typename T, typename L, int ORDER, bool EDM, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_wide_tile2(StepArgs<T> a, int nbx, int nby, int sw)
{
    constexpr int Q = L::Q;
    constexpr int M = lattice_reach<L>();
    constexpr int R = Stencil<2, ORDER>::R;
    using W = WideTile2<Q, R, M, TX, TY>;
    constexpr int H1 = W::H1, P1W = W::P1W, P1N = W::P1N;
    constexpr int C1W = W::C1W, C1H = W::C1H;
    constexpr int P2W = W::P2W, P2H = W::P2H, P2N = W::P2N;
    __shared__ T psi1[P1N];
    __shared__ T psi2[P2N];
    __shared__ T s1[Q * P2N];

    const int nx = a.nx, ny = a.ny;
    const int64_t n = a.n;
    const uint32_t TS = sizeof(T), rowb = (uint32_t)nx * TS;
    const int tid = threadIdx.x;
    int bx, by;
    strip_tile(xcd_swizzle(blockIdx.x, gridDim.x), nbx, nby, sw, bx, by);
    const int x0 = bx * TX, y0 = by * TY;

    // phase 1 (the per-thread node loop has a compile-time bound and is
    // unrolled, so all of a thread's pulls are in flight together).  A tile
    // whose pulled region lies inside the grid (one test per block) takes
    // its addresses without wrapping.
    constexpr int K1 = (P1N + NT - 1) / NT;
    T g[K1][Q];
    if (x0 >= H1 + M && x0 + TX + H1 + M <= nx && y0 >= H1 + M && y0 + TY + H1 + M <= ny) {
#pragma unroll
        for (int q = 0; q < K1; ++q) {
            const int i = tid + q * NT;
            if (i < P1N) {
                const int ly = i / P1W, lx = i - ly * P1W;
                pull_lat_inner<T, L>(a.fin, n, (uint32_t)(y0 - H1 + ly) * rowb + (uint32_t)(x0 - H1 + lx) * TS,
                                     rowb, g[q]);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < K1; ++q) {
            const int i = tid + q * NT;
            if (i < P1N) {
                const int ly = i / P1W, lx = i - ly * P1W;
                uint32_t xo[2 * M + 1], yo[2 * M + 1];
                offsets_m<M>(wrap_near(x0 - H1 + lx, nx), nx, TS, xo);
                offsets_m<M>(wrap_near(y0 - H1 + ly, ny), ny, rowb, yo);
                pull_lat<T, L, M>(a.fin, n, xo, yo, g[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < K1; ++q) {
        const int i = tid + q * NT;
        if (i < P1N) psi1[i] = psi_of(a.rho_ref + TreeSum<0, Q>::of(g[q]), a);
    }
    __syncthreads();
    // phase 2: the (R + M)-halo region sits R inside the psi1 region
#pragma unroll
    for (int q = 0; q < K1; ++q) {
        const int i = tid + q * NT;
        if (i < P1N) {
            const int ly = i / P1W, lx = i - ly * P1W;
            const int cx = lx - R, cy = ly - R;
            if (cx >= 0 && cx < C1W && cy >= 0 && cy < C1H) {
                T Fx, Fy;
                wide_force_at<T, ORDER>(psi1 + ly * P1W + lx, P1W, a.gc0, Fx, Fy);
                collide_lat<T, L, EDM>(g[q], TreeSum<0, Q>::of(g[q]), Fx, Fy, a);
#pragma unroll
                for (int b = 0; b < Q; ++b) {
                    const int wx = cx - (M - L::cx[b]), wy = cy - (M - L::cy[b]);
                    if (wx >= 0 && wx < P2W && wy >= 0 && wy < P2H) s1[b * P2N + wy * P2W + wx] = g[q][b];
                }
            }
        }
    }
    __syncthreads();
    // pull at t+2 of the node at psi2 index i
    auto pull_s1 = [&](int i, T (&h)[Q]) {
#pragma unroll
        for (int b = 0; b < Q; ++b) h[b] = s1[b * P2N + i];
    };
    // phase 3: psi at t+2 on the tile + R
    constexpr int K3 = (P2N + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < K3; ++q) {
        const int i = tid + q * NT;
        if (i < P2N) {
            T h[Q];
            pull_s1(i, h);
            psi2[i] = psi_of(a.rho_ref + TreeSum<0, Q>::of(h), a);
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
        T h[Q];
        pull_s1((ly + R) * P2W + lx + R, h);
        T Fx, Fy;
        wide_force_at<T, ORDER>(psi2 + (ly + R) * P2W + lx + R, P2W, a.gc0, Fx, Fy);
        collide_lat<T, L, EDM>(h, TreeSum<0, Q>::of(h), Fx, Fy, a);
        const int xr = x0 + lx, yr = y0 + ly;
        if (xr < nx && yr < ny) {
            const uint32_t off = (uint32_t)yr * rowb + (uint32_t)xr * TS;
#pragma unroll
            for (int b = 0; b < Q; ++b) st_off_nt(a.fout + b * n, off, h[b]);
        }
    }
}

// LDS of a block on gfx950
constexpr size_t kLdsBytes = 160 * 1024;

template <typename T, typename L, int ORDER, bool EDM, int TX, int TY, int NT>
static hipError_t launch_wide_tile2(const StepArgs<T>& a, hipStream_t s)
{
    using W = WideTile2<L::Q, Stencil<2, ORDER>::R, lattice_reach<L>(), TX, TY>;
    if constexpr (W::template lds_bytes<T>() > kLdsBytes) {
        // the tile does not fit: a smaller two-step tile takes its place,
        // 32 x 8, else 32 x 4 (which fits every lattice and order in FP64)
        static_assert(TX * TY > 128, "the 32 x 4 two-step tile must fit");
        if constexpr (TX * TY > 256)
            return launch_wide_tile2<T, L, ORDER, EDM, 32, 8, 256>(a, s);
        else
            return launch_wide_tile2<T, L, ORDER, EDM, 32, 4, 256>(a, s);
    } else {
        const int nbx = (a.nx + TX - 1) / TX, nby = (a.ny + TY - 1) / TY;
        hipLaunchKernelGGL((k_wide_tile2<T, L, ORDER, EDM, TX, TY, NT>), dim3(nbx * nby), dim3(NT), 0, s, a, nbx,
                           nby, kStripTiles);
        return hipGetLastError();
    }
}

// Launch shapes of the any-lattice family (names as variant_name_wide()).
template <typename T, typename L, int ORDER, bool EDM, bool WALLS, int TX, int TY, int RPT>
static hipError_t launch_wide_tile(const StepArgs<T>& a, hipStream_t s)
{
    const int nbx = (a.nx + TX - 1) / TX, nby = (a.ny + TY - 1) / TY;
    hipLaunchKernelGGL((k_wide_tile<T, L, ORDER, EDM, WALLS, TX, TY, RPT>), dim3(nbx * nby), dim3(TX, TY / RPT), 0,
                       s, a, nbx, nby, kStripTiles);
    return hipGetLastError();
}

template <typename T, typename L, int ORDER, bool EDM, bool WALLS>
static hipError_t launch_wide_shape(const StepArgs<T>& a, int variant, hipStream_t s)
{
    switch (variant) {
    case 0: return launch_wide_tile<T, L, ORDER, EDM, WALLS, 64, 8, 2>(a, s);
    case 1: return launch_wide_tile<T, L, ORDER, EDM, WALLS, 32, 8, 1>(a, s);
    case 2: return launch_wide_tile<T, L, ORDER, EDM, WALLS, 64, 16, 4>(a, s);
    case 3: return launch_wide_tile<T, L, ORDER, EDM, WALLS, 64, 16, 2>(a, s);
    // wide rows use more of each cache line the pulls touch (reach M in x)
    case 4: return launch_wide_tile<T, L, ORDER, EDM, WALLS, 128, 16, 2>(a, s);
    case 5: return launch_wide_tile<T, L, ORDER, EDM, WALLS, 256, 8, 2>(a, s);
    // two steps per launch (no walls: the wall kernels step one at a time);
    // at 8192^2 the tuner picks 64 x 12 with 768 threads for D2Q13 E6 and
    // 64 x 16 with 1024 for D2Q25 E8 (150 KB of LDS in FP32).  A 32 x 16
    // tile with 512 threads (80 KB for D2Q25, two blocks per CU) tied on
    // D2Q25 (2.28 ms per step) and was 4% slower on D2Q13.
    case 6:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 32, 8, 256>(a, s);
        return hipErrorInvalidValue;
    case 7:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 64, 8, 512>(a, s);
        return hipErrorInvalidValue;
    case 8:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 64, 16, 1024>(a, s);
        return hipErrorInvalidValue;
    case 9:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 128, 8, 1024>(a, s);
        return hipErrorInvalidValue;
    case 10:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 64, 8, 1024>(a, s);
        return hipErrorInvalidValue;
    case 11:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 64, 12, 768>(a, s);
        return hipErrorInvalidValue;
    case 12:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 64, 12, 1024>(a, s);
        return hipErrorInvalidValue;
    // larger tiles, which the windowed post-collision copy fits in LDS:
    // 64 x 16 for D2Q25 E8 (150 KB in FP32), 128 x 12 for D2Q13
    case 13:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 64, 16, 768>(a, s);
        return hipErrorInvalidValue;
    case 14:
        if constexpr (!WALLS) return launch_wide_tile2<T, L, ORDER, EDM, 128, 12, 1024>(a, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T, typename L, bool EDM, bool WALLS>
static hipError_t launch_wide_order(const StepArgs<T>& a, int order, int variant, hipStream_t s)
{
    switch (order) {
    case 4: return launch_wide_shape<T, L, 4, EDM, WALLS>(a, variant, s);
    case 6: return launch_wide_shape<T, L, 6, EDM, WALLS>(a, variant, s);
    case 8: return launch_wide_shape<T, L, 8, EDM, WALLS>(a, variant, s);
    case 10: return launch_wide_shape<T, L, 10, EDM, WALLS>(a, variant, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, typename L, bool WALLS>
static hipError_t launch_wide_lattice(const StepArgs<T>& a, int order, bool edm, int variant, hipStream_t s)
{
    return edm ? launch_wide_order<T, L, true, WALLS>(a, order, variant, s)
               : launch_wide_order<T, L, false, WALLS>(a, order, variant, s);
}

}  // namespace sclbm
