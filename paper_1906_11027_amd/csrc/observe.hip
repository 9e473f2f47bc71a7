// observe.hip -- initial state, macroscopic fields, stand-alone force and the
// FP64 reductions (mass, momentum, maximum / mean / rms |u|) for gfx950.
//
// These run once per K steps, so they favour simplicity: one kernel per
// quantity over flat node ranges.  Reductions accumulate in FP64 whatever
// the state precision, reduce a wavefront with xor-shuffles, combine the
// waves of a block through LDS, and sum the per-block partials in a second
// single-block pass in a fixed order (deterministic for a given grid).
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

// ---------------------------------------------------------------- init ----
template <typename T, typename L, int M>
__global__ void k_init(T* __restrict__ f, const double* __restrict__ rho0, int nx, int ny, int nz,
                       double rho_ref)
{
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (M == 1) {
            int64_t zo[3], yo[3];
            int xo[3];
            neighbours<L>(i, nx, ny, nz, zo, yo, xo);
#pragma unroll
            for (int b = 0; b < L::Q; ++b) {
                // node x + c_b: the pull of the next step brings this value to it
                const int64_t src = zo[1 + L::cz[b]] + yo[1 + L::cy[b]] + xo[1 + L::cx[b]];
                f[b * n + i] = (T)(L::w[b] * (rho0[src] - rho_ref));
            }
        } else {
            int x, y, z;
            coords(i, nx, ny, x, y, z);
#pragma unroll
            for (int b = 0; b < L::Q; ++b) {
                const int64_t src = shifted_node(x, y, z, L::cx[b], L::cy[b], L::cz[b], nx, ny, nz);
                f[b * n + i] = (T)(L::w[b] * (rho0[src] - rho_ref));
            }
        }
    }
}

// Rest start: the equilibrium of velocity v = -F / (2 rho) at every node,
// so that (sum_b f_b c_b + F/2) / rho = 0.  Same placement as k_init; the
// shifted value w_b [(rho - rho_ref) + rho (c.v / cs2 + (c.v)^2 / (2 cs2^2)
// - v.v / (2 cs2))] is formed in double before the store.
template <typename T, typename L, int M>
__global__ void k_init_rest(T* __restrict__ f, const double* __restrict__ rho0, const double* __restrict__ F,
                            int nx, int ny, int nz, double rho_ref)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const double ics2 = 1.0 / L::cs2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t zo[3] = {0, 0, 0}, yo[3] = {0, 0, 0};
        int xo[3] = {0, 0, 0};
        int x = 0, y = 0, z = 0;
        if constexpr (M == 1)
            neighbours<L>(i, nx, ny, nz, zo, yo, xo);
        else
            coords(i, nx, ny, x, y, z);
#pragma unroll
        for (int b = 0; b < L::Q; ++b) {
            int64_t src;
            if constexpr (M == 1)
                src = zo[1 + L::cz[b]] + yo[1 + L::cy[b]] + xo[1 + L::cx[b]];
            else
                src = shifted_node(x, y, z, L::cx[b], L::cy[b], L::cz[b], nx, ny, nz);
            const double r = rho0[src];
            const double h = -0.5 / r;
            const double vx = h * F[src];
            const double vy = h * F[n + src];
            const double vz = L::D == 3 ? h * F[2 * n + src] : 0.0;
            const double cv = L::cx[b] * vx + L::cy[b] * vy + L::cz[b] * vz;
            const double vv = vx * vx + vy * vy + vz * vz;
            const double e = cv * ics2 + 0.5 * cv * cv * ics2 * ics2 - 0.5 * vv * ics2;
            f[b * n + i] = (T)(L::w[b] * ((r - rho_ref) + r * e));
        }
    }
}

// --------------------------------------------------------------- macro ----
// rho, psi and j = sum_b f_b c_b of the pulled (pre-collision) state.
template <typename T, typename L, int M>
__global__ void k_macro(const T* __restrict__ f, StepArgs<T> a, double* __restrict__ rho,
                        T* __restrict__ psi, double* __restrict__ j)
{
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T dr = T(0), jx = T(0), jy = T(0), jz = T(0);
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
        const T r = a.rho_ref + dr;
        rho[i] = (double)r;
        psi[i] = (a.solid && a.solid[i]) ? a.psi_w : psi_of(r, a);
        j[i] = (double)jx;
        j[n + i] = (double)jy;
        if (L::D == 3) j[2 * n + i] = (double)jz;
    }
}

// --------------------------------------------------------------- force ----
// Eq. (1) from a psi array, summed over +-e pairs; optionally the velocity
// u = (j + F/2) / rho of the observed state.
template <typename T, int D, int ORDER>
__global__ void k_force(const T* __restrict__ psi, StepArgs<T> a, double* __restrict__ F,
                        const double* __restrict__ rho, const double* __restrict__ j,
                        double* __restrict__ u)
{
    using ST = Stencil<D, ORDER>;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t n = a.n;
    const int64_t nxy = (int64_t)nx * ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(i / nxy);
        const int64_t rem = i - (int64_t)z * nxy;
        const int y = (int)(rem / nx);
        const int x = (int)(rem - (int64_t)y * nx);
        T s[3] = {T(0), T(0), T(0)};
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
        const T pref = -a.gc0 * psi[i];
        const bool wall = a.solid && a.solid[i];   // no force or velocity inside a wall
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double Fd = wall ? 0.0 : (double)(pref * s[d]);
            F[d * n + i] = Fd;
            if (u) u[d * n + i] = wall ? 0.0 : (j[d * n + i] + 0.5 * Fd) / rho[i];
        }
    }
}

template <typename T>
__global__ void k_psi_convert(const double* __restrict__ src, T* __restrict__ dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (T)src[i];
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

__global__ void __launch_bounds__(kRedThreads)
k_reduce_partials(const double* __restrict__ rho, const double* __restrict__ u, const uint8_t* __restrict__ solid,
                  int dim, int64_t n, double* __restrict__ partials)
{
    double acc[kNR];
#pragma unroll
    for (int k = 0; k < kNR; ++k) acc[k] = slot_start(k);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double r = rho[i];
        if (solid && solid[i]) {
            if (isfinite(r)) acc[0] += r;
            else acc[7] += 1.0;
            continue;
        }
        double uu = 0.0;
        bool fin = isfinite(r);
        for (int d = 0; d < dim; ++d) {
            const double ud = u[d * n + i];
            fin = fin && isfinite(ud);
            acc[1 + d] += r * ud;
            uu += ud * ud;
        }
        if (!fin) {
            acc[7] += 1.0;
            continue;
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
    block_reduce_store(acc, partials + (int64_t)blockIdx.x * kNR);
}

__global__ void __launch_bounds__(kRedThreads)
k_reduce_final(const double* __restrict__ partials, int nblk, double* __restrict__ out)
{
    double acc[kNR];
#pragma unroll
    for (int k = 0; k < kNR; ++k) acc[k] = slot_start(k);
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        const double* p = partials + (int64_t)b * kNR;
#pragma unroll
        for (int k = 0; k < kNR; ++k) acc[k] = is_max_slot(k) ? fmax(acc[k], p[k]) : acc[k] + p[k];
    }
    block_reduce_store(acc, out);
}

// ----------------------------------------------------------- launchers ----
static int grid_for(int64_t n, int threads)
{
    int64_t b = (n + threads - 1) / threads;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename T>
static hipError_t init_t(int lattice, T* f, const double* rho0, int nx, int ny, int nz, double rho_ref,
                         hipStream_t s)
{
    const int g = grid_for((int64_t)nx * ny * nz, 256);
    switch (lattice) {
    case 0: hipLaunchKernelGGL((k_init<T, D2Q9, 1>), g, 256, 0, s, f, rho0, nx, ny, nz, rho_ref); break;
    case 1: hipLaunchKernelGGL((k_init<T, D3Q19, 1>), g, 256, 0, s, f, rho0, nx, ny, nz, rho_ref); break;
    case 2: hipLaunchKernelGGL((k_init<T, D2Q13, 2>), g, 256, 0, s, f, rho0, nx, ny, nz, rho_ref); break;
    case 3: hipLaunchKernelGGL((k_init<T, D2Q25, 2>), g, 256, 0, s, f, rho0, nx, ny, nz, rho_ref); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init(int lattice, void* f, int precision, const double* rho0, int nx, int ny, int nz,
                       double rho_ref, hipStream_t s)
{
    return precision == 0 ? init_t<float>(lattice, (float*)f, rho0, nx, ny, nz, rho_ref, s)
                          : init_t<double>(lattice, (double*)f, rho0, nx, ny, nz, rho_ref, s);
}

template <typename T>
static hipError_t init_rest_t(int lattice, T* f, const double* rho0, const double* F, int nx, int ny, int nz,
                              double rho_ref, hipStream_t s)
{
    const int g = grid_for((int64_t)nx * ny * nz, 256);
    switch (lattice) {
    case 0: hipLaunchKernelGGL((k_init_rest<T, D2Q9, 1>), g, 256, 0, s, f, rho0, F, nx, ny, nz, rho_ref); break;
    case 1: hipLaunchKernelGGL((k_init_rest<T, D3Q19, 1>), g, 256, 0, s, f, rho0, F, nx, ny, nz, rho_ref); break;
    case 2: hipLaunchKernelGGL((k_init_rest<T, D2Q13, 2>), g, 256, 0, s, f, rho0, F, nx, ny, nz, rho_ref); break;
    case 3: hipLaunchKernelGGL((k_init_rest<T, D2Q25, 2>), g, 256, 0, s, f, rho0, F, nx, ny, nz, rho_ref); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init_rest(int lattice, void* f, int precision, const double* rho0, const double* F, int nx,
                            int ny, int nz, double rho_ref, hipStream_t s)
{
    return precision == 0 ? init_rest_t<float>(lattice, (float*)f, rho0, F, nx, ny, nz, rho_ref, s)
                          : init_rest_t<double>(lattice, (double*)f, rho0, F, nx, ny, nz, rho_ref, s);
}

template <typename T>
static hipError_t macro_t(int lattice, const T* f, const StepArgs<T>& a, ObsBuffers& ob, hipStream_t s)
{
    const int g = grid_for(a.n, 256);
    T* psi = (T*)ob.psi;
    switch (lattice) {
    case 0: hipLaunchKernelGGL((k_macro<T, D2Q9, 1>), g, 256, 0, s, f, a, ob.rho, psi, ob.j); break;
    case 1: hipLaunchKernelGGL((k_macro<T, D3Q19, 1>), g, 256, 0, s, f, a, ob.rho, psi, ob.j); break;
    case 2: hipLaunchKernelGGL((k_macro<T, D2Q13, 2>), g, 256, 0, s, f, a, ob.rho, psi, ob.j); break;
    case 3: hipLaunchKernelGGL((k_macro<T, D2Q25, 2>), g, 256, 0, s, f, a, ob.rho, psi, ob.j); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_macro(int lattice, int precision, const void* f, const void* args, ObsBuffers& ob,
                        hipStream_t s)
{
    if (precision == 0) return macro_t<float>(lattice, (const float*)f, *(const StepArgs<float>*)args, ob, s);
    return macro_t<double>(lattice, (const double*)f, *(const StepArgs<double>*)args, ob, s);
}

template <typename T, int D>
static hipError_t force_d(int order, const StepArgs<T>& a, ObsBuffers& ob, bool vel, hipStream_t s)
{
    const int g = grid_for(a.n, 256);
    const T* psi = (const T*)ob.psi;
    double* u = vel ? ob.u : nullptr;
    switch (order) {
    case 4: hipLaunchKernelGGL((k_force<T, D, 4>), g, 256, 0, s, psi, a, ob.F, ob.rho, ob.j, u); break;
    case 6: hipLaunchKernelGGL((k_force<T, D, 6>), g, 256, 0, s, psi, a, ob.F, ob.rho, ob.j, u); break;
    case 8: hipLaunchKernelGGL((k_force<T, D, 8>), g, 256, 0, s, psi, a, ob.F, ob.rho, ob.j, u); break;
    case 10:
        if (D != 2) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_force<T, 2, 10>), g, 256, 0, s, psi, a, ob.F, ob.rho, ob.j, u);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_force(int dim, int precision, int order, const void* args, ObsBuffers& ob,
                        bool with_velocity, hipStream_t s)
{
    if (precision == 0) {
        const StepArgs<float>& a = *(const StepArgs<float>*)args;
        return dim == 2 ? force_d<float, 2>(order, a, ob, with_velocity, s)
                        : force_d<float, 3>(order, a, ob, with_velocity, s);
    }
    const StepArgs<double>& a = *(const StepArgs<double>*)args;
    return dim == 2 ? force_d<double, 2>(order, a, ob, with_velocity, s)
                    : force_d<double, 3>(order, a, ob, with_velocity, s);
}

hipError_t launch_psi_from_host(int precision, const double* psi_dev_d, void* psi, int64_t n, hipStream_t s)
{
    const int g = grid_for(n, 256);
    if (precision == 0)
        hipLaunchKernelGGL(k_psi_convert<float>, g, 256, 0, s, psi_dev_d, (float*)psi, n);
    else
        hipLaunchKernelGGL(k_psi_convert<double>, g, 256, 0, s, psi_dev_d, (double*)psi, n);
    return hipGetLastError();
}

hipError_t launch_reduce(int dim, ObsBuffers& ob, const uint8_t* solid, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_partials, ob.nblk, kRedThreads, 0, s, ob.rho, ob.u, solid, dim, n, ob.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, 1, kRedThreads, 0, s, ob.partials, ob.nblk, ob.result);
    return hipGetLastError();
}

}  // namespace sclbm
