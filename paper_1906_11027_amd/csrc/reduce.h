// reduce.h -- node-level pieces of the observation path shared by the
// single-grid and batched kernels: periodic neighbour indices, the moments
// of a pulled node, the interaction force of Eq. (1) at a node from a psi
// array, and the FP64 reduction slots (wavefront xor-shuffles, then LDS
// across the waves of a block).
#pragma once
#include "kernels.h"

namespace sclbm {

template <typename L>
__device__ __forceinline__ void neighbours(int64_t i, int nx, int ny, int nz, int64_t (&zo)[3],
                                           int64_t (&yo)[3], int (&xo)[3])
{
    const int64_t nxy = (int64_t)nx * ny;
    const int z = (int)(i / nxy);
    const int64_t rem = i - (int64_t)z * nxy;
    const int y = (int)(rem / nx);
    const int x = (int)(rem - (int64_t)y * nx);
    xo[0] = x == 0 ? nx - 1 : x - 1;
    xo[1] = x;
    xo[2] = x == nx - 1 ? 0 : x + 1;
    yo[0] = (int64_t)(y == 0 ? ny - 1 : y - 1) * nx;
    yo[1] = (int64_t)y * nx;
    yo[2] = (int64_t)(y == ny - 1 ? 0 : y + 1) * nx;
    zo[0] = (int64_t)(z == 0 ? nz - 1 : z - 1) * nxy;
    zo[1] = (int64_t)z * nxy;
    zo[2] = (int64_t)(z == nz - 1 ? 0 : z + 1) * nxy;
}

// Flat index of node (x, y, z) + (dx, dy, dz) on the periodic grid (any
// offset; used by the lattices that stream over distance 2).
__device__ __forceinline__ int64_t shifted_node(int x, int y, int z, int dx, int dy, int dz, int nx, int ny, int nz)
{
    return ((int64_t)wrap_any(z + dz, nz) * ny + wrap_any(y + dy, ny)) * nx + wrap_any(x + dx, nx);
}

__device__ __forceinline__ void coords(int64_t i, int nx, int ny, int& x, int& y, int& z)
{
    const int64_t nxy = (int64_t)nx * ny;
    z = (int)(i / nxy);
    const int64_t rem = i - (int64_t)z * nxy;
    y = (int)(rem / nx);
    x = (int)(rem - (int64_t)y * nx);
}

// rho - rho_ref and j = sum_b f_b c_b of node i from the pulled
// (pre-collision) state, summed over b in list order.
template <typename T, typename L, int M>
__device__ __forceinline__ void pull_moments(const T* __restrict__ f, const StepArgs<T>& a, int64_t i, T& dr,
                                             T& jx, T& jy, T& jz)
{
    const int64_t n = a.n;
    dr = T(0);
    jx = T(0);
    jy = T(0);
    jz = T(0);
    if (M == 1) {
        int64_t zo[3], yo[3];
        int xo[3];
        neighbours<L>(i, a.nx, a.ny, a.nz, zo, yo, xo);
#pragma unroll
        for (int b = 0; b < L::Q; ++b) {
            const T v = f[b * n + zo[1 - L::cz[b]] + yo[1 - L::cy[b]] + xo[1 - L::cx[b]]];
            dr += v;
            jx += T(L::cx[b]) * v;
            jy += T(L::cy[b]) * v;
            jz += T(L::cz[b]) * v;
        }
    } else {
        int x, y, z;
        coords(i, a.nx, a.ny, x, y, z);
#pragma unroll
        for (int b = 0; b < L::Q; ++b) {
            const T v = f[b * n + shifted_node(x, y, z, -L::cx[b], -L::cy[b], -L::cz[b], a.nx, a.ny, a.nz)];
            dr += v;
            jx += T(L::cx[b]) * v;
            jy += T(L::cy[b]) * v;
            jz += T(L::cz[b]) * v;
        }
    }
}

// Eq. (1) at node i from a psi array, summed over +-e pairs:
// s = sum_pairs w (psi(x + e) - psi(x - e)) e; F = -G c0 psi(x) s.
template <typename T, int D, int ORDER>
__device__ __forceinline__ void force_sum(const T* __restrict__ psi, const StepArgs<T>& a, int64_t i, T (&s)[3])
{
#pragma clang fp contract(off)   // same rounding as force_sum_lds: no fused multiply-adds
    using ST = Stencil<D, ORDER>;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t nxy = (int64_t)nx * ny;
    const int z = (int)(i / nxy);
    const int64_t rem = i - (int64_t)z * nxy;
    const int y = (int)(rem / nx);
    const int x = (int)(rem - (int64_t)y * nx);
    s[0] = s[1] = s[2] = T(0);
#pragma unroll
    for (int p = 0; p < ST::NP; ++p) {
        constexpr PairList P = ST::P;
        const int ex = P.e[p][0], ey = P.e[p][1], ez = P.e[p][2];
        const int64_t ip = (int64_t)wrap_any(z + ez, nz) * nxy + (int64_t)wrap_any(y + ey, ny) * nx +
                           wrap_any(x + ex, nx);
        const int64_t im = (int64_t)wrap_any(z - ez, nz) * nxy + (int64_t)wrap_any(y - ey, ny) * nx +
                           wrap_any(x - ex, nx);
        const T wd = T(P.w[p]) * (psi[ip] - psi[im]);
        s[0] += T(ex) * wd;
        s[1] += T(ey) * wd;
        s[2] += T(ez) * wd;
    }
}

// ------------------------------------------------------------- reduce ----
// partial[blk] = {sum rho, sum rho u_x, sum rho u_y, sum rho u_z,
//                 max |u|, sum |u|, sum |u|^2, count of non-finite nodes,
//                 count of finite fluid nodes, max rho, max -rho}
// (the maxima over finite fluid nodes).  Wall nodes add their rho
// (populations in transit) to the mass only.
constexpr int kNR = kObsSlots;
constexpr int kRedThreads = 256;

__host__ __device__ constexpr bool is_max_slot(int k) { return k == 4 || k == 9 || k == 10; }
__host__ __device__ constexpr double slot_start(int k) { return (k == 9 || k == 10) ? -1e300 : 0.0; }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void block_reduce_store(double (&acc)[kNR], double* out)
{
    __shared__ double red[kRedThreads / 64][kNR];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kNR; ++k) acc[k] = is_max_slot(k) ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < kNR; ++k) red[wv][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < kNR) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int w = 1; w < kRedThreads / 64; ++w) v = is_max_slot(k) ? fmax(v, red[w][k]) : v + red[w][k];
        out[k] = v;
    }
}


// u_d = (j_d + F_d / 2) / rho of a node in FP64, rounded the same way on
// both observation paths (no fused multiply-add)
__device__ __forceinline__ double node_u(double j, double F, double rho)
{
#pragma clang fp contract(off)
    return (j + 0.5 * F) / rho;
}

// One node's share of the slots.  Wall nodes add their rho (populations in
// transit) to the mass only; a fluid node with a non-finite rho or u is
// counted and otherwise left out.
__device__ __forceinline__ void accumulate_node(double (&acc)[kNR], double r, const double (&ud)[3], int dim,
                                                bool wall)
{
#pragma clang fp contract(off)   // |u| rounded alike wherever this is inlined
    if (wall) {
        if (isfinite(r)) acc[0] += r;
        else acc[7] += 1.0;
        return;
    }
    double uu = 0.0;
    bool fin = isfinite(r);
    for (int d = 0; d < dim; ++d) {
        fin = fin && isfinite(ud[d]);
        acc[1 + d] += r * ud[d];
        uu += ud[d] * ud[d];
    }
    if (!fin) {
        acc[7] += 1.0;
        return;
    }
    const double um = sqrt(uu);
    acc[0] += r;
    acc[4] = fmax(acc[4], um);
    acc[5] += um;
    acc[6] += uu;
    acc[8] += 1.0;
    acc[9] = fmax(acc[9], r);
    acc[10] = fmax(acc[10], -r);
}

// Eq. (1) at the centre c of an LDS psi tile with row stride sy and plane
// stride sz, in the pair order and arithmetic of force_sum.
template <typename T, int D, int ORDER>
__device__ __forceinline__ void force_sum_lds(const T* __restrict__ c, int sy, int sz, T (&s)[3])
{
#pragma clang fp contract(off)   // same rounding as force_sum
    using ST = Stencil<D, ORDER>;
    s[0] = s[1] = s[2] = T(0);
#pragma unroll
    for (int p = 0; p < ST::NP; ++p) {
        constexpr PairList P = ST::P;
        const int ex = P.e[p][0], ey = P.e[p][1], ez = P.e[p][2];
        const int off = ez * sz + ey * sy + ex;
        const T wd = T(P.w[p]) * (c[off] - c[-off]);
        s[0] += T(ex) * wd;
        s[1] += T(ey) * wd;
        s[2] += T(ez) * wd;
    }
}

// Tile of the fused steady-state check: one node per thread of a 256-thread
// block, 16 x 16 in 2D and 8 x 8 x 4 in 3D.
template <int D>
struct CheckTile {
    static constexpr int TX = D == 3 ? 8 : 16, TY = D == 3 ? 8 : 16, TZ = D == 3 ? 4 : 1;
};
// LDS psi values the check tile of any order in D dimensions can need
// (radius 3 in 2D, 2 in 3D)
template <int D>
constexpr int check_lds_max()
{
    return D == 3 ? (CheckTile<3>::TX + 4) * (CheckTile<3>::TY + 4) * (CheckTile<3>::TZ + 4)
                  : (CheckTile<2>::TX + 6) * (CheckTile<2>::TY + 6);
}

// One tile of the fused check at origin (x0, y0, z0): psi of the tile and
// its halo of the stencil radius into psi_s (every node pulled from the
// state a.fin; solid nodes take psi_w), then the tile's own nodes' rho, u and
// their share of the reduction slots.  The centre node ic and node 0 also
// leave (rho, psi) in extra[0..1] and extra[2..3].  Every thread of the
// block calls it (barriers inside).
template <typename T, typename L, int M, int ORDER>
__device__ __forceinline__ void check_tile(const StepArgs<T>& a, int x0, int y0, int z0, T* __restrict__ psi_s,
                                           double (&acc)[kNR], int64_t ic, double* __restrict__ extra)
{
    constexpr int D = L::D;
    using CT = CheckTile<D>;
    constexpr int R = Stencil<D, ORDER>::R;
    constexpr int RZ = D == 3 ? R : 0;
    constexpr int LX = CT::TX + 2 * R, LY = CT::TY + 2 * R, LZ = CT::TZ + 2 * RZ;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    __syncthreads();   // the previous tile's force sums are done with psi_s
    for (int i = threadIdx.x; i < LX * LY * LZ; i += blockDim.x) {
        const int lx = i % LX, ly = (i / LX) % LY, lz = i / (LX * LY);
        const int gx = wrap_any(x0 - R + lx, nx), gy = wrap_any(y0 - R + ly, ny), gz = wrap_any(z0 - RZ + lz, nz);
        const int64_t gi = ((int64_t)gz * ny + gy) * nx + gx;
        T dr, jx, jy, jz;
        pull_moments<T, L, M>(a.fin, a, gi, dr, jx, jy, jz);
        psi_s[i] = (a.solid && a.solid[gi]) ? a.psi_w : psi_of(a.rho_ref + dr, a);
    }
    __syncthreads();
    const int tx = threadIdx.x % CT::TX, ty = (threadIdx.x / CT::TX) % CT::TY, tz = threadIdx.x / (CT::TX * CT::TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (threadIdx.x < CT::TX * CT::TY * CT::TZ && x < nx && y < ny && z < nz) {
        const int64_t i = ((int64_t)z * ny + y) * nx + x;
        T dr, j[3];
        pull_moments<T, L, M>(a.fin, a, i, dr, j[0], j[1], j[2]);
        const T r = a.rho_ref + dr;
        const T* c = psi_s + ((tz + RZ) * LY + ty + R) * LX + tx + R;
        T s[3];
        force_sum_lds<T, D, ORDER>(c, LX, LX * LY, s);
        const T pref = -a.gc0 * c[0];
        const bool wall = a.solid && a.solid[i];
        const double rd = (double)r;
        double ud[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double Fd = wall ? 0.0 : (double)(pref * s[d]);
            ud[d] = wall ? 0.0 : node_u((double)j[d], Fd, rd);
        }
        accumulate_node(acc, rd, ud, D, wall);
        if (i == ic) {
            extra[0] = rd;
            extra[1] = (double)c[0];
        }
        if (i == 0) {
            extra[2] = rd;
            extra[3] = (double)c[0];
        }
    }
}

}  // namespace sclbm
