// kernels.h -- device helpers and launcher declarations of the gfx950 path.
//
// State layout (both precisions): structure of arrays f[Q][N], node index
// i = x + nx (y + ny z), velocity order of lattice.h.  The stored value is
// the POST-collision distribution shifted by its rest weight,
//     g_b(x) = f*_b(x) - w_b rho_ref,
// so one step pulls f_b(x, t+1) = f*_b(x - c_b, t) (Sec. 2, Eq. (3)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"

namespace sclbm {

template <typename T>
struct StepArgs {
    const T* __restrict__ fin;   // state at t (post-collision, shifted)
    T* __restrict__ fout;        // state at t+1
    int nx, ny, nz;
    int64_t n;                   // nx * ny * nz
    T gc0;                       // G * c0 (force prefactor, Sec. 2 Eq. (1))
    T omega;                     // 1 / tau
    T guo;                       // 1 - 1 / (2 tau)   (Guo forcing, Eq. (4))
    T rho_ref;                   // storage shift
    T psi0, inv_rho_psi;         // psi = psi0 (1 - exp(-rho / rho_psi))
    int psi_kind;                // 0 exp form, 1 psi = rho, 2 Peng-Robinson
    T s_bulk, s_ghost;           // MRT rates (D3Q19)
    T cs2;                       // lattice sound speed squared
    T eos_RT, eos_b, eos_aa;     // Peng-Robinson R T, b and a alpha(T)
    T eos_k;                     // 2 / (G c0)
    const uint8_t* __restrict__ solid;   // wall mask [N] (1 = solid) or null
    T psi_w;                     // psi of the virtual wall density
};

// exp, 1/x and sqrt for the hot kernels.  The FP32 state uses the hardware
// instructions (v_exp_f32 computes 2^x, so exp(x) = 2^(x log2 e); v_rcp_f32,
// v_sqrt_f32; each within 1 ulp): a few operations instead of the
// correctly rounded sequences, well inside the FP32 state's own rounding.
// The FP64 state keeps the correctly rounded forms.
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ double fast_exp(double x) { return exp(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }

// Pseudo-potential.  The Peng-Robinson form inverts the bulk pressure of the
// model, p = cs2 rho + G c0 psi^2 / 2 (Sec. 3):
//   psi = sqrt(2 (p_PR(rho) - cs2 rho) / (G c0)),  0 where the root is not real.
template <typename T>
__device__ __forceinline__ T psi_of(T rho, const StepArgs<T>& a)
{
    if (a.psi_kind == 1) return rho;
    if (a.psi_kind == 2) {
        const T br = a.eos_b * rho;
        const T p = rho * a.eos_RT * fast_rcp(T(1) - br) -
                    a.eos_aa * rho * rho * fast_rcp(T(1) + T(2) * br - br * br);
        const T arg = (p - a.cs2 * rho) * a.eos_k;
        return arg > T(0) ? fast_sqrt(arg) : T(0);
    }
    return a.psi0 * (T(1) - fast_exp(-rho * a.inv_rho_psi));
}

__device__ __forceinline__ int wrap_any(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

// v mod n for v at most one period outside [0, n) without a division (halo
// coordinates of grids wider than the halo); any other v takes wrap_any.
__device__ __forceinline__ int wrap_near(int v, int n)
{
    const int r = v < 0 ? v + n : (v >= n ? v - n : v);
    return (r >= 0 && r < n) ? r : wrap_any(v, n);
}

// XCD-aware block order.  Work-groups are dealt round-robin to the 8 XCDs
// (block b runs on XCD b % 8), each with its own L2.  Remap the linear block
// id so that XCD k processes one contiguous range of logical tiles: tiles
// that share halo lines then run on the same XCD at about the same time.
// The map is a bijection on [0, nb) for any nb.
__device__ __forceinline__ int xcd_swizzle(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Logical tile order of the 2D tile kernels: vertical strips of `sw` tile
// columns, tiles advancing along x within a strip row, strip rows down y,
// strips one after another.  The tile below a tile then starts `sw` tiles
// later on the same XCD (xcd_swizzle keeps logical ranges together), so the
// halo rows the two share are still in that XCD's L2; in plain row-major
// order a full-width tile row of a large grid evicts them first.  A
// bijection from [0, nbx * nby) onto the tile grid for any sw >= 1.
constexpr int kStripTiles = 8;   // tile columns per strip

__device__ __forceinline__ void strip_tile(int L, int nbx, int nby, int sw, int& bx, int& by)
{
    const int full = nbx / sw;
    const int per = sw * nby;
    if (L < full * per) {
        const int s = L / per, r = L - s * per;
        by = r / sw;
        bx = s * sw + (r - by * sw);
    } else {
        const int tw = nbx - full * sw;   // width of the last, narrower strip
        const int r = L - full * per;
        by = r / tw;
        bx = full * sw + (r - by * tw);
    }
}

// Addressing of the hot kernels: one velocity plane holds N values, fewer
// than 2^32 bytes (checked on the host), so a node is addressed as the plane's
// uniform base pointer (scalar registers) plus a 32-bit per-lane byte offset,
// the global-load form with a scalar base and a 32-bit vector offset.
// The state is device global memory; the accesses say so, so that pointers
// read from memory (the batched work list's items) also take global rather
// than flat loads and stores.
template <typename T>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, uint32_t off)
{
    return *(const __attribute__((address_space(1))) T*)((const char*)base + off);
}
template <typename T>
__device__ __forceinline__ void st_off(T* __restrict__ base, uint32_t off, T v)
{
    *(__attribute__((address_space(1))) T*)((char*)base + off) = v;
}
// the same store marked non-temporal.  Measured per kernel: the two-step
// kernels of one grid gain with it at 8192^2 (D2Q25 5%, D2Q13 3%, D2Q9
// FP64 1.7%, FP32 0.3%; 256^2 unchanged), and so do the FP64 D3Q19 marches
// at 320^3 (3-5%); the FP32 D3Q19 marches and the batched sweep lost 4%,
// so they keep the plain store.
template <typename T>
__device__ __forceinline__ void st_off_nt(T* __restrict__ base, uint32_t off, T v)
{
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T*)((char*)base + off));
}

// ---------------------------------------------------------------- D2Q9 ----
// Pull the nine shifted distributions of node (x, y): value b comes from
// (x - cx_b, y - cy_b).  xo[0..2] are the byte offsets of columns x-1, x,
// x+1 and yo[0..2] those of rows y-1, y, y+1 (wrapped).
template <typename T>
__device__ __forceinline__ void pull_d2q9(const T* __restrict__ f, int64_t n, const uint32_t (&xo)[3],
                                          const uint32_t (&yo)[3], T (&g)[9])
{
#pragma unroll
    for (int b = 0; b < 9; ++b)
        g[b] = ld_off(f + b * n, yo[1 - D2Q9::cy[b]] + xo[1 - D2Q9::cx[b]]);
}

// byte offsets of the wrapped neighbours of coordinate v in [0, n): k-1, k, k+1
template <typename T>
__device__ __forceinline__ void nbr_offsets(int v, int n, uint32_t stride, uint32_t (&o)[3])
{
    o[0] = (uint32_t)(v == 0 ? n - 1 : v - 1) * stride;
    o[1] = (uint32_t)v * stride;
    o[2] = (uint32_t)(v == n - 1 ? 0 : v + 1) * stride;
}

template <typename T>
__device__ __forceinline__ T sum9(const T (&g)[9])
{
    return ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
}

// Guo-forced BGK collision (Sec. 2, Eq. (3)-(4)) on shifted values.
// drho = rho - rho_ref = sum_b g_b;  u = (sum_b g_b c_b + F/2) / rho.
template <typename T>
__device__ __forceinline__ void collide_d2q9_srt(T (&g)[9], T drho, T Fx, T Fy, const StepArgs<T>& a)
{
    const T rho = a.rho_ref + drho;
    const T jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const T jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const T inv = fast_rcp(rho);
    const T ux = (jx + T(0.5) * Fx) * inv;
    const T uy = (jy + T(0.5) * Fy) * inv;
    const T usq = T(1.5) * (ux * ux + uy * uy);
    const T uF = ux * Fx + uy * Fy;
    const T om = a.omega, gu = a.guo;
    // Velocities b and b + 2 (b = 1, 2, 5, 6) are opposite.  Over such a
    // pair the relaxed equilibrium plus the Guo source, om feq + gu phihat,
    // splits into a part even in c and a part odd in c:
    //   even  w [K0 + cu (a1 cu + a2 cF)],  K0 = om (drho - rho usq) - 3 gu u.F,
    //         a1 = 4.5 om rho, a2 = 9 gu;
    //   odd   w (b1 cu + b2 cF),            b1 = 3 om rho, b2 = 3 gu,
    // with cu = c.u and cF = c.F formed once per pair, and
    //   g*_{+-} = g_{+-} + (even +- odd - om g_{+-}).
    // Collision conserves mass exactly; the rest population closes the
    // balance in difference form, g0* = g0 + sum_{b>=1} (g_b - g_b*): the
    // increments are small, so the node's mass keeps only the rounding of
    // the stored g0* (not that of two 9-term sums of O(rho) values).
    const T K0 = om * (drho - rho * usq) - T(3) * gu * uF;
    const T a1 = T(4.5) * om * rho, a2 = T(9) * gu;
    const T b1 = T(3) * om * rho, b2 = T(3) * gu;
    T dm = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int bp = k < 2 ? 1 + k : 3 + k;   // 1, 2, 5, 6
        const int bm = bp + 2;                  // 3, 4, 7, 8
        const T cu = T(D2Q9::cx[bp]) * ux + T(D2Q9::cy[bp]) * uy;
        const T cF = T(D2Q9::cx[bp]) * Fx + T(D2Q9::cy[bp]) * Fy;
        const T w = T(D2Q9::w[bp]);
        const T S = w * (K0 + cu * (a1 * cu + a2 * cF));
        const T A = w * (b1 * cu + b2 * cF);
        const T gp = g[bp], gm = g[bm];
        const T np = gp + ((S + A) - om * gp);
        const T nm = gm + ((S - A) - om * gm);
        dm += (gp - np) + (gm - nm);
        g[bp] = np;
        g[bm] = nm;
    }
    g[0] += dm;
}

constexpr bool d2q9_opposite_pairs()
{
    for (int bp : {1, 2, 5, 6})
        if (D2Q9::cx[bp + 2] != -D2Q9::cx[bp] || D2Q9::cy[bp + 2] != -D2Q9::cy[bp] ||
            D2Q9::w[bp + 2] != D2Q9::w[bp])
            return false;
    return true;
}
static_assert(d2q9_opposite_pairs(), "D2Q9 velocity order: b and b + 2 must be opposite for b = 1, 2, 5, 6");

// --------------------------------------------------------------- D3Q19 ----
template <typename T>
__device__ __forceinline__ T sum19(const T (&g)[19])
{
    T s0 = (g[0] + g[1]) + (g[2] + g[3]);
    T s1 = (g[4] + g[5]) + (g[6] + g[7]);
    T s2 = (g[8] + g[9]) + (g[10] + g[11]);
    T s3 = (g[12] + g[13]) + (g[14] + g[15]);
    T s4 = (g[16] + g[17]) + g[18];
    return ((s0 + s1) + (s2 + s3)) + s4;
}

// Guo-forced collision for D3Q19.  MRT is written as BGK at the ghost rate
// plus corrections on the six viscous moments:
//   f* = f - s_g n + (1 - s_g/2) phihat
//        + sum_{k in bulk, shear} (s_g - s_k) [m_k . (n + phihat/2)] m_k / |m_k|^2
// with n = f - feq and m_k the (mutually orthogonal) moment vectors
//   bulk:  19 c^2 - 30                     (|m|^2 = 2394)
//   shear: 2cx^2 - cy^2 - cz^2 (36), cy^2 - cz^2 (12), cx cy, cy cz, cx cz (4).
// The conserved moments drop out because m.(n + phihat/2) = 0 for rho and j.
// This equals M^-1 S M with the rates grouped as conserved / bulk / shear /
// ghost; with all rates 1/tau it is exactly the BGK step.
// velocities b and b + 1 (b odd) are opposite: the collision below pairs them
constexpr bool d3q19_opposite_pairs()
{
    for (int b = 1; b < 19; b += 2)
        if (D3Q19::cx[b + 1] != -D3Q19::cx[b] || D3Q19::cy[b + 1] != -D3Q19::cy[b] ||
            D3Q19::cz[b + 1] != -D3Q19::cz[b] || D3Q19::w[b + 1] != D3Q19::w[b])
            return false;
    return true;
}
static_assert(d3q19_opposite_pairs(), "D3Q19 velocity order must list opposite pairs");

template <typename T, bool MRT>
__device__ __forceinline__ void collide_d3q19(T (&g)[19], T drho, T Fx, T Fy, T Fz, const StepArgs<T>& a)
{
    // The moving velocities come in pairs (b, b + 1), b odd, with
    // c_{b+1} = -c_b.  Over a pair, feq and phihat split into a part even in
    // c (the same for both) and a part odd in c (opposite signs):
    //   feq   = w [drho + rho (4.5 (c.u)^2 - 1.5 u^2)]  +-  3 w rho (c.u)
    //   phihat = w [9 (c.u)(c.F) - 3 u.F]                +-  3 w (c.F)
    // and every moment vector above is even in c, so the moments need only
    // the pair sums.  Each pair's c.u and c.F are formed once.
    using L = D3Q19;
    const T rho = a.rho_ref + drho;
    T jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
    for (int b = 1; b < 19; b += 2) {
        const T d = g[b] - g[b + 1];
        if (L::cx[b] > 0) jx += d; else if (L::cx[b] < 0) jx -= d;
        if (L::cy[b] > 0) jy += d; else if (L::cy[b] < 0) jy -= d;
        if (L::cz[b] > 0) jz += d; else if (L::cz[b] < 0) jz -= d;
    }
    const T inv = fast_rcp(rho);
    const T ux = (jx + T(0.5) * Fx) * inv;
    const T uy = (jy + T(0.5) * Fy) * inv;
    const T uz = (jz + T(0.5) * Fz) * inv;
    const T usq = T(1.5) * (ux * ux + uy * uy + uz * uz);
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    // mass closure through the rest population in difference form (see
    // collide_d2q9_srt): dm = sum_{b>=1} (g_b - g_b*), g0* = g0 + dm
    T dm = T(0);
    if (!MRT) {
        // om feq + gu phihat over a pair, even and odd parts as in the D2Q9
        // collision: w [K0 + cu (a1 cu + a2 cF)] and w (b1 cu + b2 cF)
        const T om = a.omega, gu = a.guo;
        const T K0 = om * (drho - rho * usq) - T(3) * gu * uF;
        const T a1 = T(4.5) * om * rho, a2 = T(9) * gu;
        const T b1 = T(3) * om * rho, b2 = T(3) * gu;
#pragma unroll
        for (int b = 1; b < 19; b += 2) {
            const T cu = T(L::cx[b]) * ux + T(L::cy[b]) * uy + T(L::cz[b]) * uz;
            const T cF = T(L::cx[b]) * Fx + T(L::cy[b]) * Fy + T(L::cz[b]) * Fz;
            const T w = T(L::w[b]);
            const T S = w * (K0 + cu * (a1 * cu + a2 * cF));
            const T A = w * (b1 * cu + b2 * cF);
            const T gp = g[b], gm = g[b + 1];
            const T np = gp + ((S + A) - om * gp);
            const T nm = gm + ((S - A) - om * gm);
            dm += (gp - np) + (gm - nm);
            g[b] = np;
            g[b + 1] = nm;
        }
        g[0] += dm;
    } else {
        // BGK at the ghost rate sg with the Guo source (1 - sg/2) phihat, plus
        // for each moment k of the bulk and shear groups
        //   (sg - s_k) [m_k . v] m_k / |m_k|^2,  v = f - feq + phihat / 2.
        // Pass 1 forms the moments m_k . v; every m_k is even in c, so a pair
        // enters through v_b + v_{b+1} = (g_b + g_{b+1}) - 2 feq_even + phihat_even
        //   = (g_b + g_{b+1}) - w [V0 + 9 cu (rho cu - cF)],
        //   V0 = 2 (drho - rho usq) + 3 u.F.
        // Pass 2 applies BGK, source and the (even) moment correction d of the
        // pair in one increment: g*_{+-} = g_{+-} + ((even + d) +- odd - sg g_{+-}),
        // even and odd as in the SRT branch with om -> sg, gu -> 1 - sg/2.
        const T sg = a.s_ghost;
        const T gh = T(1) - T(0.5) * sg;
        // the rest population enters only the bulk moment (19 c^2 - 30 = -30)
        const T w0 = T(L::w[0]);
        const T v0 = (g[0] - w0 * (drho - rho * usq)) + T(0.5) * (w0 * (T(-3) * uF));
        const T V0 = T(2) * (drho - rho * usq) + T(3) * uF;
        T mb = T(-30) * v0, m1 = T(0), m2 = T(0), m3 = T(0), m4 = T(0), m5 = T(0);
        T cuv[9], cFv[9];
#pragma unroll
        for (int b = 1; b < 19; b += 2) {
            const int cx = L::cx[b], cy = L::cy[b], cz = L::cz[b];
            const T cu = T(cx) * ux + T(cy) * uy + T(cz) * uz;
            const T cF = T(cx) * Fx + T(cy) * Fy + T(cz) * Fz;
            cuv[b / 2] = cu;
            cFv[b / 2] = cF;
            const T vs = (g[b] + g[b + 1]) - T(L::w[b]) * (V0 + T(9) * cu * (rho * cu - cF));
            const int c2 = cx * cx + cy * cy + cz * cz;
            mb += T(19 * c2 - 30) * vs;
            const int p1 = 2 * cx * cx - cy * cy - cz * cz, p2 = cy * cy - cz * cz;
            if (p1) m1 += T(p1) * vs;
            if (p2) m2 += T(p2) * vs;
            if (cx * cy) m3 += T(cx * cy) * vs;
            if (cy * cz) m4 += T(cy * cz) * vs;
            if (cx * cz) m5 += T(cx * cz) * vs;
        }
        const T kb = (sg - a.s_bulk) * mb * T(1.0 / 2394.0);
        const T ks = sg - a.omega;
        const T k1 = ks * m1 * T(1.0 / 36.0), k2 = ks * m2 * T(1.0 / 12.0);
        const T k3 = ks * m3 * T(0.25), k4 = ks * m4 * T(0.25), k5 = ks * m5 * T(0.25);
        const T K0 = sg * (drho - rho * usq) - T(3) * gh * uF;
        const T a1 = T(4.5) * sg * rho, a2 = T(9) * gh;
        const T b1 = T(3) * sg * rho, b2 = T(3) * gh;
#pragma unroll
        for (int b = 1; b < 19; b += 2) {
            const int cx = L::cx[b], cy = L::cy[b], cz = L::cz[b];
            const int c2 = cx * cx + cy * cy + cz * cz;
            T d = kb * T(19 * c2 - 30);
            const int p1 = 2 * cx * cx - cy * cy - cz * cz, p2 = cy * cy - cz * cz;
            if (p1) d += k1 * T(p1);
            if (p2) d += k2 * T(p2);
            if (cx * cy) d += k3 * T(cx * cy);
            if (cy * cz) d += k4 * T(cy * cz);
            if (cx * cz) d += k5 * T(cx * cz);
            const T cu = cuv[b / 2], cF = cFv[b / 2];
            const T w = T(L::w[b]);
            const T Sd = w * (K0 + cu * (a1 * cu + a2 * cF)) + d;
            const T A = w * (b1 * cu + b2 * cF);
            const T gp = g[b], gm = g[b + 1];
            const T np = gp + ((Sd + A) - sg * gp);
            const T nm = gm + ((Sd - A) - sg * gm);
            dm += (gp - np) + (gm - nm);
            g[b] = np;
            g[b + 1] = nm;
        }
        g[0] += dm;
    }
}

// ------------------------------------------------------------ launchers ----
// Fused force + collide + pull-stream step.  `variant` picks a launch shape
// (see kernels_2d.hip / kernels_3d.hip / wide2d.h); returns hipSuccess or an
// error.
hipError_t launch_step_d2q9(const StepArgs<float>& a, int order, int variant, hipStream_t s);
hipError_t launch_step_d2q9(const StepArgs<double>& a, int order, int variant, hipStream_t s);
hipError_t launch_step_d3q19(const StepArgs<float>& a, int order, bool mrt, int variant, hipStream_t s);
hipError_t launch_step_d3q19(const StepArgs<double>& a, int order, bool mrt, int variant, hipStream_t s);
int num_variants_d2q9();
int variant_steps_d2q9(int v);   // time steps one launch of the shape advances (1 or 2)
int num_variants_d3q19();
const char* variant_name_d2q9(int v);
const char* variant_name_d3q19(int v);

// Any-lattice 2D step (D2Q13, D2Q25, and D2Q9 with the exact difference
// method): lattice is the SC_* id, edm selects the forcing.
hipError_t launch_step_wide(int lattice, const StepArgs<float>& a, int order, bool edm, int variant,
                            hipStream_t s);
hipError_t launch_step_wide(int lattice, const StepArgs<double>& a, int order, bool edm, int variant,
                            hipStream_t s);
int num_variants_wide();
int variant_steps_wide(int v);   // 1, or 2 for the shapes that block two steps in time
const char* variant_name_wide(int v);
// per-lattice instantiations (kernels_wide_q*.hip)
hipError_t launch_wide_q9(const StepArgs<float>& a, int order, bool edm, int variant, hipStream_t s);
hipError_t launch_wide_q9(const StepArgs<double>& a, int order, bool edm, int variant, hipStream_t s);
hipError_t launch_wide_q13(const StepArgs<float>& a, int order, bool edm, int variant, hipStream_t s);
hipError_t launch_wide_q13(const StepArgs<double>& a, int order, bool edm, int variant, hipStream_t s);
hipError_t launch_wide_q25(const StepArgs<float>& a, int order, bool edm, int variant, hipStream_t s);
hipError_t launch_wide_q25(const StepArgs<double>& a, int order, bool edm, int variant, hipStream_t s);

// Initial state: g_b(x) = w_b (rho0(x + c_b) - rho_ref), i.e. the pull of
// the next step sees f = feq(rho0, u = 0) everywhere.  lattice: SC_* id.
hipError_t launch_init(int lattice, void* f, int precision, const double* rho0, int nx, int ny, int nz,
                       double rho_ref, hipStream_t s);
// f = feq(rho0, -F / (2 rho0)) with F [D][N] (device doubles), placed like launch_init.
hipError_t launch_init_rest(int lattice, void* f, int precision, const double* rho0, const double* F, int nx,
                            int ny, int nz, double rho_ref, hipStream_t s);

// Observables: macroscopic fields of the current state and FP64 reductions.
constexpr int kObsSlots = 11;  // reduction slots per block (observe.hip)
struct ObsBuffers {
    double* rho;      // [N]
    void* psi;        // [N] in the state precision
    double* j;        // [D][N] sum_b f_b c_b
    double* F;        // [D][N]
    double* u;        // [D][N]
    double* partials; // [nblk][kObsSlots]
    double* result;   // [kObsSlots]
    int nblk;
};
hipError_t launch_macro(int lattice, int precision, const void* f, const void* args, ObsBuffers& ob,
                        hipStream_t s);
hipError_t launch_force(int dim, int precision, int order, const void* args, ObsBuffers& ob,
                        bool with_velocity, hipStream_t s);
hipError_t launch_psi_from_host(int precision, const double* psi_dev_d, void* psi, int64_t n, hipStream_t s);
hipError_t launch_reduce(int dim, ObsBuffers& ob, const uint8_t* solid, int64_t n, hipStream_t s);
// dst[i] = (double)src[i], i < n
hipError_t launch_widen(const float* src, double* dst, int64_t n, hipStream_t s);

// Steady-state check straight from the state, in one pass: each block takes
// tiles of the grid, fills an LDS tile of psi (tile plus the force stencil's
// halo, every node pulled from the state), then for its own nodes forms rho,
// j, F (Eq. (1)) and u = (j + F/2) / rho and accumulates the kObsSlots FP64
// reduction slots; a single-block pass sums the per-block partials in a
// fixed order.  result holds kCheckSlots doubles: the reduction slots, then
// rho and psi at the centre node and at node 0 (the Laplace pressure pair).
// partials: check_blocks(...) rows of kObsSlots doubles.
constexpr int kCheckSlots = kObsSlots + 4;
constexpr int kCheckMaxBlocks = 1024;   // check_blocks() never exceeds it
int check_blocks(int lattice, int64_t nx, int64_t ny, int64_t nz);
hipError_t launch_check(int lattice, int precision, int order, const void* f, const void* args, double* partials,
                        double* result, hipStream_t s);

// Batched D2Q9 step over a (item, tile) work list (kernels_batch.hip).
// Launch shapes of the batched step: 0 one step per launch on 32 x 8 tiles;
// 1-3 two steps per launch (temporal blocking) on 32 x 8, 64 x 16 and
// 32 x 16 tiles.  Work entries are (item, tile) pairs of the shape's tile.
int batch_num_shapes();
int batch_shape_steps(int v);
void batch_shape_tile(int v, int* tw, int* th);
const char* batch_shape_name(int v);
size_t batch_item_bytes(int precision);
void batch_fill_item(void* dst, int precision, const void* a, void* b, int nx, int ny, int order, double gc0,
                     double tau);
hipError_t launch_batch_d2q9(int shape, const void* items, const int2* work, int nwork, int parity, int precision,
                             const void* common, hipStream_t s);
// Steady-state check of every active item (the single-grid check above per
// item): cwork lists (item, 16 x 16 tile) entries, one block each, whose
// partial rows are cwork's indices; citems lists (item, first entry, entry
// count) per active item; results holds kCheckSlots doubles per item.
// Net momentum of an FP64 D2Q9 state (shifted storage, n nodes):
// momentum_blocks() rows of (sum g, sum g c_x, sum g c_y) partials; and the
// shift g_b += 3 w_b rho_x (c_b . u) of every node, which adds rho_x u to its
// momentum and leaves its mass unchanged.
int momentum_blocks();
hipError_t launch_d2q9_mass_momentum(const double* g, int64_t n, double* partial, hipStream_t s);
hipError_t launch_d2q9_momentum_shift(double* g, int64_t n, double rho_ref, double ux, double uy, hipStream_t s);
int batch_check_tile();
hipError_t launch_batch_check(const void* items, const int2* cwork, int ncwork, const int4* citems, int nactive,
                              int parity, int precision, const void* common, double* partials, double* results,
                              hipStream_t s);

}  // namespace sclbm
