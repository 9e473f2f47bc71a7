// observe.hip -- initial state, macroscopic fields, stand-alone force and the
// FP64 reductions (mass, momentum, maximum / mean / rms |u|) for gfx950.
//
// These run once per K steps, so they favour simplicity: one kernel per
// quantity over flat node ranges.  Reductions accumulate in FP64 whatever
// the state precision, reduce a wavefront with xor-shuffles, combine the
// waves of a block through LDS, and sum the per-block partials in a second
// single-block pass in a fixed order (deterministic for a given grid).
#include "reduce.h"

namespace sclbm {

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
// rho, psi and j of the pulled state as fields.
template <typename T, typename L, int M>
__global__ void k_macro(const T* __restrict__ f, StepArgs<T> a, double* __restrict__ rho,
                        T* __restrict__ psi, double* __restrict__ j)
{
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T dr, jx, jy, jz;
        pull_moments<T, L, M>(f, a, i, dr, jx, jy, jz);
        const T r = a.rho_ref + dr;
        rho[i] = (double)r;
        psi[i] = (a.solid && a.solid[i]) ? a.psi_w : psi_of(r, a);
        j[i] = (double)jx;
        j[n + i] = (double)jy;
        if (L::D == 3) j[2 * n + i] = (double)jz;
    }
}

// --------------------------------------------------------------- force ----
// The force field, and optionally the velocity u = (j + F/2) / rho of the
// observed state.
template <typename T, int D, int ORDER>
__global__ void k_force(const T* __restrict__ psi, StepArgs<T> a, double* __restrict__ F,
                        const double* __restrict__ rho, const double* __restrict__ j,
                        double* __restrict__ u)
{
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T s[3];
        force_sum<T, D, ORDER>(psi, a, i, s);
        const T pref = -a.gc0 * psi[i];
        const bool wall = a.solid && a.solid[i];   // no force or velocity inside a wall
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double Fd = wall ? 0.0 : (double)(pref * s[d]);
            F[d * n + i] = Fd;
            if (u) u[d * n + i] = wall ? 0.0 : node_u(j[d * n + i], Fd, rho[i]);
        }
    }
}

// an FP32 state widened exactly to FP64 (same storage shift)
__global__ void k_widen(const float* __restrict__ src, double* __restrict__ dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

template <typename T>
__global__ void k_psi_convert(const double* __restrict__ src, T* __restrict__ dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (T)src[i];
}

// ------------------------------------------------------------- reduce ----
__global__ void __launch_bounds__(kRedThreads)
k_reduce_partials(const double* __restrict__ rho, const double* __restrict__ u, const uint8_t* __restrict__ solid,
                  int dim, int64_t n, double* __restrict__ partials)
{
    double acc[kNR];
#pragma unroll
    for (int k = 0; k < kNR; ++k) acc[k] = slot_start(k);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double ud[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < dim; ++d) ud[d] = u[d * n + i];
        accumulate_node(acc, rho[i], ud, dim, solid && solid[i]);
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


// ------------------------------------------------------------- check ----
// Fused steady-state check: blocks take the grid's check tiles in turn
// (at most kCheckMaxBlocks blocks, so the partials stay a bounded size).

template <typename T, typename L, int M, int ORDER>
__global__ void __launch_bounds__(kRedThreads)
k_check(StepArgs<T> a, int ntx, int nty, int ntz, int64_t ic, double* __restrict__ partials,
        double* __restrict__ extra)
{
    using CT = CheckTile<L::D>;
    __shared__ T psi_s[check_lds_max<L::D>()];
    double acc[kNR];
#pragma unroll
    for (int k = 0; k < kNR; ++k) acc[k] = slot_start(k);
    const int ntiles = ntx * nty * ntz;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int bx = t % ntx, by = (t / ntx) % nty, bz = t / (ntx * nty);
        check_tile<T, L, M, ORDER>(a, bx * CT::TX, by * CT::TY, bz * CT::TZ, psi_s, acc, ic, extra);
    }
    block_reduce_store(acc, partials + (int64_t)blockIdx.x * kNR);
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

hipError_t launch_widen(const float* src, double* dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_widen, grid_for(n, 256), 256, 0, s, src, dst, n);
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

static void check_tiles(int lattice, int64_t nx, int64_t ny, int64_t nz, int64_t& tx, int64_t& ty, int64_t& tz)
{
    const bool d3 = lattice == 1;
    const int TX = d3 ? CheckTile<3>::TX : CheckTile<2>::TX, TY = d3 ? CheckTile<3>::TY : CheckTile<2>::TY;
    const int TZ = d3 ? CheckTile<3>::TZ : CheckTile<2>::TZ;
    tx = (nx + TX - 1) / TX;
    ty = (ny + TY - 1) / TY;
    tz = (nz + TZ - 1) / TZ;
}

int check_blocks(int lattice, int64_t nx, int64_t ny, int64_t nz)
{
    int64_t tx, ty, tz;
    check_tiles(lattice, nx, ny, nz, tx, ty, tz);
    const int64_t t = tx * ty * tz;
    return (int)(t < kCheckMaxBlocks ? t : kCheckMaxBlocks);
}

template <typename T, typename L, int M, int ORDER>
static hipError_t check_launch(const StepArgs<T>& a, double* partials, double* result, hipStream_t s)
{
    int64_t tx, ty, tz;
    check_tiles(L::D == 3 ? 1 : 0, a.nx, a.ny, a.nz, tx, ty, tz);
    const int nb = check_blocks(L::D == 3 ? 1 : 0, a.nx, a.ny, a.nz);
    const int64_t ic = (int64_t)(a.nx / 2) + (int64_t)a.nx * ((int64_t)(a.ny / 2) + (int64_t)a.ny * (a.nz / 2));
    hipLaunchKernelGGL((k_check<T, L, M, ORDER>), nb, kRedThreads, 0, s, a, (int)tx, (int)ty, (int)tz, ic,
                       partials, result + kObsSlots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, 1, kRedThreads, 0, s, partials, nb, result);
    return hipGetLastError();
}

template <typename T, typename L, int M>
static hipError_t check_order(int order, const StepArgs<T>& a, double* partials, double* result, hipStream_t s)
{
    switch (order) {
    case 4: return check_launch<T, L, M, 4>(a, partials, result, s);
    case 6: return check_launch<T, L, M, 6>(a, partials, result, s);
    case 8: return check_launch<T, L, M, 8>(a, partials, result, s);
    case 10:
        if constexpr (L::D == 2) return check_launch<T, L, M, 10>(a, partials, result, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t check_t(int lattice, int order, const T* f, const StepArgs<T>& args, double* partials,
                          double* result, hipStream_t s)
{
    StepArgs<T> a = args;
    a.fin = f;
    switch (lattice) {
    case 0: return check_order<T, D2Q9, 1>(order, a, partials, result, s);
    case 1: return check_order<T, D3Q19, 1>(order, a, partials, result, s);
    case 2: return check_order<T, D2Q13, 2>(order, a, partials, result, s);
    case 3: return check_order<T, D2Q25, 2>(order, a, partials, result, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_check(int lattice, int precision, int order, const void* f, const void* args, double* partials,
                        double* result, hipStream_t s)
{
    if (precision == 0)
        return check_t<float>(lattice, order, (const float*)f, *(const StepArgs<float>*)args, partials, result, s);
    return check_t<double>(lattice, order, (const double*)f, *(const StepArgs<double>*)args, partials, result, s);
}

}  // namespace sclbm
