// sc_lbm.cpp -- host side of the C ABI declared in include/sc_lbm.h.
//
// Owns the two state buffers (or borrows the caller's), enqueues the fused
// step kernels on one stream, captures runs of steps into HIP graphs (one
// per parity of the current buffer, since a graph freezes its kernel
// arguments), and turns the FP64 reductions into sc_lbm_obs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/sc_lbm.h"
#include "kernels.h"

using namespace sclbm;

namespace {

constexpr int kGraphSteps = 32;   // steps per captured graph (even)
// automatic batched launch shapes (batch_shape_*), two steps per launch:
// FP32 on 32 x 16 tiles with 512 threads (72.7 GLUPS on the 64-droplet
// sweep, against 63 for the 64 x 16 and 32 x 8 tiles), FP64 on 64 x 16
// tiles with 1024 threads (34.5 GLUPS, against 28-29 for 32 x 8 and
// 32 x 16); sc_lbm_batch_autotune measures them all
constexpr int kBatchShapeFP32 = 3;
constexpr int kBatchShapeFP64 = 2;
constexpr int kFloorWindow = 50;   // checks the FP32 resolution rule fits a line to
constexpr int kFloorHorizon = 300; // checks ahead over which that line's drift must stay in the band

struct ObsState {
    bool ready = false;
    ObsBuffers b{};
};

}  // namespace

struct sc_lbm {
    sc_lbm_params p;
    int dim = 2, q = 9;
    int64_t n = 0;
    size_t tsize = 4;
    void* f[2] = {nullptr, nullptr};
    bool own_f = false;
    int cur = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t step = 0;
    int variant = 0;
    StepArgs<float> af{};
    StepArgs<double> ad{};
    ObsState obs;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    bool graph_failed = false;
    double last_max_u = -1.0;
    double umax_hist[kFloorWindow] = {};   // max|u| of the last checks (FP32 resolution rule)
    int64_t umax_n = 0;          // checks recorded since the last reset
    int conv_by = 0;             // rule that stopped the last sc_lbm_step: 1 tol, 2 FP32 floor
    int tol_hits = 0;            // consecutive checks with a change below tol
    uint8_t* solid = nullptr;   // device wall mask [N] (null: no walls)
    // steady-state check: per-block partials and the result block on the
    // device, the result's pinned host copy, and graphs of K steps followed
    // by the check (one per buffer parity at the start of the K steps)
    double* chk_partials = nullptr;
    double* chk_result = nullptr;
    double* chk_host = nullptr;
    hipGraphExec_t gchunk[2] = {nullptr, nullptr};
    int gchunk_end[2] = {0, 1};   // buffer holding the state after gchunk[k]
    double* scratch = nullptr;    // this device's copy of the file-scope scratch array (null if not found)
};

static thread_local char g_detail[256] = "";

static void set_detail(const char* where, hipError_t e)
{
    std::snprintf(g_detail, sizeof(g_detail), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
}

// map a HIP status to an SC_E_* code, recording where it happened
static int hip_err_at(hipError_t e, const char* where)
{
    if (e == hipSuccess) return SC_OK;
    set_detail(where, e);
    return e == hipErrorOutOfMemory ? SC_E_NOMEM : SC_E_DEVICE;
}
#define hip_err(e) hip_err_at((e), __func__)

// ---- lattice facts used on the host ---------------------------------------
static int lattice_q(int lattice)
{
    switch (lattice) {
    case SC_D2Q9: return 9;
    case SC_D3Q19: return 19;
    case SC_D2Q13: return 13;
    case SC_D2Q25: return 25;
    default: return 0;
    }
}
static int lattice_dim(int lattice) { return lattice == SC_D3Q19 ? 3 : 2; }
static double lattice_cs2(int lattice)
{
    return lattice == SC_D2Q13 ? D2Q13::cs2 : (lattice == SC_D2Q25 ? D2Q25::cs2 : 1.0 / 3.0);
}

// Kernel families: the D2Q9 Guo kernels, the D3Q19 kernels, and the
// any-lattice 2D kernels (D2Q13, D2Q25, D2Q9 with the exact difference method).
enum Family { kFamD2Q9 = 0, kFamD3Q19 = 1, kFamWide = 2 };
static Family family_of(const sc_lbm_params& p)
{
    if (p.lattice == SC_D3Q19) return kFamD3Q19;
    if (p.lattice == SC_D2Q9 && p.forcing == SC_GUO) return kFamD2Q9;
    return kFamWide;
}
// With walls every 2D lattice runs the any-lattice kernels.
static Family handle_family(const sc_lbm* h) { return h->solid ? kFamWide : family_of(h->p); }

static int family_variants(Family f)
{
    return f == kFamD2Q9 ? num_variants_d2q9() : (f == kFamD3Q19 ? num_variants_d3q19() : num_variants_wide());
}

namespace sclbm {
static const char* const kShapesWide[] = {"wide64x8r2",     "wide32x8r1",     "wide64x16r4",
                                          "wide64x16r2",    "wide128x16r2",   "wide256x8r2",
                                          "wide2x32x8t256", "wide2x64x8t512", "wide2x64x16t1024",
                                          "wide2x128x8t1024", "wide2x64x8t1024", "wide2x64x12t768",
                                          "wide2x64x12t1024", "wide2x64x16t768", "wide2x128x12t1024"};
int num_variants_wide() { return (int)(sizeof(kShapesWide) / sizeof(kShapesWide[0])); }
// shapes 6.. advance two steps per launch (no walls)
int variant_steps_wide(int v) { return v >= 6 ? 2 : 1; }
const char* variant_name_wide(int v) { return (v >= 0 && v < num_variants_wide()) ? kShapesWide[v] : "?"; }

template <typename T>
static hipError_t wide_dispatch(int lattice, const StepArgs<T>& a, int order, bool edm, int variant, hipStream_t s)
{
    switch (lattice) {
    case SC_D2Q9: return launch_wide_q9(a, order, edm, variant, s);
    case SC_D2Q13: return launch_wide_q13(a, order, edm, variant, s);
    case SC_D2Q25: return launch_wide_q25(a, order, edm, variant, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_step_wide(int lattice, const StepArgs<float>& a, int order, bool edm, int variant, hipStream_t s)
{
    return wide_dispatch<float>(lattice, a, order, edm, variant, s);
}
hipError_t launch_step_wide(int lattice, const StepArgs<double>& a, int order, bool edm, int variant, hipStream_t s)
{
    return wide_dispatch<double>(lattice, a, order, edm, variant, s);
}
}  // namespace sclbm

extern "C" void sc_lbm_default_params(sc_lbm_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->lattice = SC_D2Q9;
    p->nx = 64;
    p->ny = 64;
    p->nz = 1;
    p->order = 4;
    p->psi_kind = SC_PSI_EXP;
    p->G = -5.0;
    p->c0 = 1.0 / 3.0;
    p->psi0 = 1.0;
    p->rho_psi = 1.0;
    p->tau = 1.0;
    p->collision = SC_SRT;
    p->precision = SC_FP32_SHIFTED;
    p->s_bulk = 1.2;
    p->s_ghost = 1.2;
    p->rho_ref = SC_RHO_REF_AUTO;
    p->obs_every = 100;
    p->variant = -1;
}

// Checks everything but the variant index.
static int validate_problem(const sc_lbm_params* p)
{
    if (!p) return SC_E_INVAL;
    if (lattice_q(p->lattice) == 0) return SC_E_INVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return SC_E_INVAL;
    const int dim = lattice_dim(p->lattice);
    if (dim == 2 && p->nz != 1) return SC_E_INVAL;
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    // one velocity plane must stay below 4 GiB (32-bit byte offsets in the kernels)
    const int64_t ts = p->precision == SC_FP64 ? 8 : 4;
    if (n * ts >= ((int64_t)1 << 32)) return SC_E_UNSUPPORTED;
    if (dim == 2) {
        if (p->order != 4 && p->order != 6 && p->order != 8 && p->order != 10) return SC_E_INVAL;
    } else {
        if (p->order != 4 && p->order != 6 && p->order != 8) return SC_E_UNSUPPORTED;
    }
    if (p->psi_kind != SC_PSI_EXP && p->psi_kind != SC_PSI_IDENTITY && p->psi_kind != SC_PSI_PR) return SC_E_INVAL;
    if (p->collision != SC_SRT && p->collision != SC_MRT) return SC_E_INVAL;
    if (p->collision == SC_MRT && p->lattice != SC_D3Q19) return SC_E_UNSUPPORTED;
    if (p->forcing != SC_GUO && p->forcing != SC_EDM) return SC_E_INVAL;
    if (p->forcing == SC_EDM && (dim != 2 || p->collision != SC_SRT)) return SC_E_UNSUPPORTED;
    if (p->psi_kind == SC_PSI_PR) {
        const double v[5] = {p->eos_a, p->eos_b, p->eos_R, p->eos_T, p->eos_alpha};
        for (double x : v)
            if (!std::isfinite(x)) return SC_E_INVAL;
        if (!(p->eos_b > 0.0) || !(p->eos_R > 0.0) || !(p->eos_T > 0.0) || p->eos_a < 0.0 || p->eos_alpha < 0.0)
            return SC_E_INVAL;
        if (!(p->G * p->c0 != 0.0)) return SC_E_INVAL;
    }
    if (p->precision != SC_FP32_SHIFTED && p->precision != SC_FP64) return SC_E_INVAL;
    if (!std::isfinite(p->G) || !std::isfinite(p->c0) || !std::isfinite(p->rho_ref)) return SC_E_INVAL;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return SC_E_INVAL;
    if (p->psi_kind == SC_PSI_EXP && (!(p->rho_psi > 0.0) || !std::isfinite(p->psi0))) return SC_E_INVAL;
    if (p->collision == SC_MRT) {
        if (!(p->s_bulk > 0.0 && p->s_bulk < 2.0) || !(p->s_ghost > 0.0 && p->s_ghost < 2.0)) return SC_E_INVAL;
    }
    if (p->obs_every < 0) return SC_E_INVAL;
    if (p->init != SC_INIT_EQUILIBRIUM && p->init != SC_INIT_REST) return SC_E_INVAL;
    return SC_OK;
}

static int validate(const sc_lbm_params* p)
{
    const int rc = validate_problem(p);
    if (rc != SC_OK) return rc;
    if (p->variant < -1 || p->variant >= family_variants(family_of(*p))) return SC_E_INVAL;
    return SC_OK;
}

extern "C" size_t sc_lbm_state_bytes(const sc_lbm_params* p)
{
    if (validate(p) != SC_OK) return 0;
    const size_t q = (size_t)lattice_q(p->lattice);
    const size_t ts = p->precision == SC_FP64 ? 8 : 4;
    return q * (size_t)p->nx * p->ny * p->nz * ts;
}

extern "C" int sc_lbm_num_variants(const sc_lbm_params* p)
{
    if (validate_problem(p) != SC_OK) return 0;
    return family_variants(family_of(*p));
}

// Time steps one launch of the handle's shape advances (the two-step D2Q9
// shapes fuse two steps per launch).
static int steps_per_launch(const sc_lbm* h)
{
    switch (handle_family(h)) {
    case kFamD2Q9: return variant_steps_d2q9(h->variant);
    case kFamWide: return h->solid ? 1 : variant_steps_wide(h->variant);
    default: return 1;
    }
}

extern "C" int sc_lbm_steps_per_launch(const sc_lbm* h) { return h ? steps_per_launch(h) : 0; }

extern "C" const char* sc_lbm_variant_name(const sc_lbm* h)
{
    if (!h) return "";
    switch (handle_family(h)) {
    case kFamD2Q9: return variant_name_d2q9(h->variant);
    case kFamD3Q19: return variant_name_d3q19(h->variant);
    default: return variant_name_wide(h->variant);
    }
}

template <typename T>
static void fill_args(sc_lbm* h, StepArgs<T>& a)
{
    const sc_lbm_params& p = h->p;
    a.fin = nullptr;
    a.fout = nullptr;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.n = h->n;
    a.gc0 = (T)(p.G * p.c0);
    a.omega = (T)(1.0 / p.tau);
    a.guo = (T)(1.0 - 0.5 / p.tau);
    a.rho_ref = (T)p.rho_ref;
    a.psi0 = (T)p.psi0;
    a.inv_rho_psi = (T)(p.psi_kind == SC_PSI_EXP ? 1.0 / p.rho_psi : 1.0);
    a.psi_kind = p.psi_kind;
    a.s_bulk = (T)p.s_bulk;
    a.s_ghost = (T)p.s_ghost;
    a.cs2 = (T)lattice_cs2(p.lattice);
    const bool pr = p.psi_kind == SC_PSI_PR;
    a.eos_RT = (T)(pr ? p.eos_R * p.eos_T : 0.0);
    a.eos_b = (T)(pr ? p.eos_b : 0.0);
    a.eos_aa = (T)(pr ? p.eos_a * p.eos_alpha : 0.0);
    a.eos_k = (T)(pr ? 2.0 / (p.G * p.c0) : 0.0);
}

// ---- launch-shape autotuning --------------------------------------------
// Tuned choices are kept per (lattice, order, precision, collision, grid) in
// process memory and, when SC_LBM_TUNE_CACHE names a file, in that file (one
// "lattice order precision collision forcing nx ny nz variant ms" line per
// entry; entries whose variant is out of range for their family are dropped).
struct TuneKey {
    int lattice, order, precision, collision, forcing, nx, ny, nz;
    bool operator==(const TuneKey& o) const
    {
        return lattice == o.lattice && order == o.order && precision == o.precision && collision == o.collision &&
               forcing == o.forcing && nx == o.nx && ny == o.ny && nz == o.nz;
    }
};
struct TuneEntry {
    TuneKey k;
    int variant;
    double ms;
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;
static bool g_tune_loaded = false;

static TuneKey tune_key(const sc_lbm_params& p)
{
    return TuneKey{p.lattice, p.order, p.precision, p.collision, p.forcing, p.nx, p.ny, p.nz};
}

static Family family_of_key(const TuneKey& k)
{
    sc_lbm_params p{};
    p.lattice = k.lattice;
    p.forcing = k.forcing;
    return family_of(p);
}

static void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("SC_LBM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    TuneEntry e;
    while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %lf", &e.k.lattice, &e.k.order, &e.k.precision,
                       &e.k.collision, &e.k.forcing, &e.k.nx, &e.k.ny, &e.k.nz, &e.variant, &e.ms) == 10)
        if (e.variant >= 0 && e.variant < family_variants(family_of_key(e.k))) g_tune.push_back(e);
    std::fclose(f);
}

static int tune_lookup(const sc_lbm_params& p)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    const TuneKey k = tune_key(p);
    for (const TuneEntry& e : g_tune)
        if (e.k == k) return e.variant;
    return -1;
}

static void tune_store(const sc_lbm_params& p, int variant, double ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    const TuneKey k = tune_key(p);
    bool found = false;
    for (TuneEntry& e : g_tune)
        if (e.k == k) {
            e.variant = variant;
            e.ms = ms;
            found = true;
        }
    if (!found) g_tune.push_back(TuneEntry{k, variant, ms});
    const char* path = std::getenv("SC_LBM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    for (const TuneEntry& e : g_tune)
        std::fprintf(f, "%d %d %d %d %d %d %d %d %d %.6g\n", e.k.lattice, e.k.order, e.k.precision, e.k.collision,
                     e.k.forcing, e.k.nx, e.k.ny, e.k.nz, e.variant, e.ms);
    std::fclose(f);
}

static int auto_variant(const sc_lbm_params& p, int64_t n)
{
    const int tuned = tune_lookup(p);
    if (tuned >= 0) return tuned;
    switch (family_of(p)) {
    case kFamD2Q9: return n < (int64_t)1 << 20 ? 2 : 0;   // tile32x8r1 / tile64x16r4
    // march64x8r1h16pf1; in FP64 its 512-thread blocks leave 256 registers
    // a lane and the E6/E8 MRT step spills, so FP64 takes the 256-thread
    // march32x16h16, which keeps its window in registers
    case kFamD3Q19: return p.precision == SC_FP64 ? 0 : 7;
    default:
        if (n < (int64_t)1 << 20) return 1;                    // wide32x8r1
        // wide128x16r2; its 1024-thread blocks spill the FP64 D2Q25 step, which
        // takes wide64x8r2 (512 threads)
        return (p.precision == SC_FP64 && p.lattice == SC_D2Q25) ? 0 : 4;
    }
}

static void drop_graphs(sc_lbm* h)
{
    for (int k = 0; k < 2; ++k) {
        if (h->gexec[k]) hipGraphExecDestroy(h->gexec[k]);
        if (h->gchunk[k]) hipGraphExecDestroy(h->gchunk[k]);
        h->gexec[k] = nullptr;
        h->gchunk[k] = nullptr;
    }
}

static void release(sc_lbm* h)
{
    if (!h) return;
    drop_graphs(h);
    hipFree(h->chk_partials);
    hipFree(h->chk_result);
    if (h->chk_host) hipHostFree(h->chk_host);
    if (h->obs.ready) {
        ObsBuffers& b = h->obs.b;
        hipFree(b.rho);
        hipFree(b.psi);
        hipFree(b.j);
        hipFree(b.F);
        hipFree(b.u);
        hipFree(b.partials);
        hipFree(b.result);
    }
    if (h->own_f) {
        hipFree(h->f[0]);
        hipFree(h->f[1]);
    }
    if (h->own_stream && h->stream) hipStreamDestroy(h->stream);
    hipFree(h->solid);
    delete h;
}

static int ensure_obs(sc_lbm* h);
static const void* args_ptr(sc_lbm* h);

// Appends about `budget` evenly strided finite densities of one initial
// field (all of them when it is smaller; rho = 1 everywhere for a NULL field).
static void sample_density(const double* rho, int64_t n, int64_t budget, std::vector<double>& out)
{
    const int64_t stride = std::max<int64_t>(1, n / std::max<int64_t>(1, budget));
    for (int64_t i = 0; i < n; i += stride) {
        const double r = rho ? rho[i] : 1.0;
        if (std::isfinite(r)) out.push_back(r);  // sc_lbm_create rejects the field
    }
}

// The shift SC_RHO_REF_AUTO picks: the median of the sampled densities.  A
// state stored as f - w rho_ref is rounded relative to |rho - rho_ref|, so
// centring it on the density most nodes hold (the surrounding phase of a
// droplet or a bubble) keeps their rounding, and the velocity noise it feeds,
// smallest.
static double median_density(std::vector<double>& v)
{
    if (v.empty()) return 1.0;
    const size_t mid = v.size() / 2;
    std::nth_element(v.begin(), v.begin() + mid, v.end());
    return std::max(0.0, v[mid]);
}

constexpr int64_t kShiftSamples = (int64_t)1 << 20;

// ---- scratch of the allocation-free check ---------------------------------
// One array per device, made when the library is loaded and held until the
// process ends: room for the per-block partials of the fused check at its
// largest grid (kCheckMaxBlocks rows) and its result block.  In host code
// `scratch` names a host-side stand-in; kernels receive the device address
// from hipGetSymbolAddress, looked up once per device.
constexpr int kScratchDoubles = kCheckMaxBlocks * kObsSlots + kCheckSlots;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be current;
// nullptr (with the HIP error recorded) if it cannot be found.
static double* device_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            set_detail("hipGetSymbolAddress(scratch)", e);
            return nullptr;
        }
        g_scratch[dev] = (double*)ptr;
    }
    return g_scratch[dev];
}

extern "C" int sc_lbm_create(const sc_lbm_params* p, const double* rho_init, void* dev_a, void* dev_b,
                             void* hip_stream, sc_lbm** out)
{
    int rc = validate(p);
    if (rc != SC_OK) return rc;
    if (!out) return SC_E_INVAL;
    if ((dev_a == nullptr) != (dev_b == nullptr) || (dev_a && dev_a == dev_b)) return SC_E_INVAL;
    sc_lbm* h = new (std::nothrow) sc_lbm();
    if (!h) return SC_E_NOMEM;
    h->p = *p;
    if (h->p.obs_every == 0) h->p.obs_every = 100;
    h->dim = lattice_dim(p->lattice);
    h->q = lattice_q(p->lattice);
    h->n = (int64_t)p->nx * p->ny * p->nz;
    h->tsize = p->precision == SC_FP64 ? 8 : 4;
    h->variant = p->variant >= 0 ? p->variant : auto_variant(*p, h->n);
    if (rho_init) {
        for (int64_t i = 0; i < h->n; ++i)
            if (!std::isfinite(rho_init[i])) {
                delete h;
                return SC_E_INVAL;
            }
    }
    if (h->p.rho_ref < 0.0) {
        try {
            std::vector<double> smp;
            sample_density(rho_init, h->n, kShiftSamples, smp);
            h->p.rho_ref = median_density(smp);
        } catch (const std::bad_alloc&) {
            delete h;
            return SC_E_NOMEM;
        }
    }
    int ndev = 0;
    hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev < 1) {
        set_detail("hipGetDeviceCount", de == hipSuccess ? hipErrorNoDevice : de);
        delete h;
        return SC_E_DEVICE;
    }
    // set-up of the allocation-free check on the current device (the one
    // the handle's buffers and stream belong to)
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) h->scratch = device_scratch(dev);
    hipError_t e;
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreate(&h->stream);
        if (e != hipSuccess) {
            delete h;
            return hip_err(e);
        }
        h->own_stream = true;
    }
    const size_t bytes = sc_lbm_state_bytes(p);
    if (dev_a) {
        h->f[0] = dev_a;
        h->f[1] = dev_b;
    } else {
        h->own_f = true;
        e = hipMalloc(&h->f[0], bytes);
        if (e == hipSuccess) e = hipMalloc(&h->f[1], bytes);
        if (e != hipSuccess) {
            rc = hip_err(e);
            release(h);
            return rc;
        }
    }
    fill_args(h, h->af);
    fill_args(h, h->ad);
    // initial state from rho_init (or rho = 1)
    double* rho_d = nullptr;
    e = hipMalloc(&rho_d, sizeof(double) * h->n);
    if (e != hipSuccess) {
        rc = hip_err(e);
        release(h);
        return rc;
    }
    std::vector<double> ones;
    const double* src = rho_init;
    if (!src) {
        try {
            ones.assign(h->n, 1.0);
        } catch (const std::bad_alloc&) {
            hipFree(rho_d);
            release(h);
            return SC_E_NOMEM;
        }
        src = ones.data();
    }
    const char* where = "hipMemcpyAsync(rho_init)";
    e = hipMemcpyAsync(rho_d, src, sizeof(double) * h->n, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        where = "init kernel";
        e = launch_init(p->lattice, h->f[0], p->precision, rho_d, p->nx, p->ny, p->nz, h->p.rho_ref, h->stream);
    }
    if (e == hipSuccess && p->init == SC_INIT_REST) {
        // F of psi(rho_init) from the equilibrium state just written, then
        // the populations again at the equilibrium of -F / (2 rho)
        rc = ensure_obs(h);
        if (rc != SC_OK) {
            hipFree(rho_d);
            release(h);
            return rc;
        }
        ObsBuffers& b = h->obs.b;
        where = "rest initialisation";
        e = launch_macro(p->lattice, p->precision, h->f[0], args_ptr(h), b, h->stream);
        if (e == hipSuccess) e = launch_force(h->dim, p->precision, p->order, args_ptr(h), b, false, h->stream);
        if (e == hipSuccess)
            e = launch_init_rest(p->lattice, h->f[0], p->precision, rho_d, b.F, p->nx, p->ny, p->nz,
                                 h->p.rho_ref, h->stream);
    }
    if (e == hipSuccess) {
        where = "hipStreamSynchronize(create)";
        e = hipStreamSynchronize(h->stream);
    }
    hipFree(rho_d);
    if (e != hipSuccess) {
        rc = hip_err_at(e, where);
        release(h);
        return rc;
    }
    *out = h;
    return SC_OK;
}

extern "C" void sc_lbm_destroy(sc_lbm* h)
{
    if (!h) return;
    hipStreamSynchronize(h->stream);
    release(h);
}

extern "C" void* sc_lbm_state_ptr(sc_lbm* h) { return h ? h->f[h->cur] : nullptr; }

extern "C" void* sc_lbm_stream(sc_lbm* h) { return h ? (void*)h->stream : nullptr; }

extern "C" double sc_lbm_rho_ref(const sc_lbm* h) { return h ? h->p.rho_ref : std::nan(""); }


// single-step D2Q9 shape used for the odd step of a two-step shape
constexpr int kSingleStepD2Q9 = 2;   // tile32x8r1

template <typename T>
static hipError_t launch_family(sc_lbm* h, const StepArgs<T>& a, bool single = false)
{
    const sc_lbm_params& p = h->p;
    switch (handle_family(h)) {
    case kFamD2Q9:
        return launch_step_d2q9(a, p.order, single && variant_steps_d2q9(h->variant) != 1 ? kSingleStepD2Q9 : h->variant,
                                h->stream);
    case kFamD3Q19: return launch_step_d3q19(a, p.order, p.collision == SC_MRT, h->variant, h->stream);
    default: {
        // the odd step of a two-step shape, and every step with walls, take a
        // one-step shape of the same tiling scale
        int v = h->variant;
        if ((single || h->solid) && variant_steps_wide(v) != 1) v = h->n < ((int64_t)1 << 20) ? 1 : 4;
        return launch_step_wide(p.lattice, a, p.order, p.forcing == SC_EDM, v, h->stream);
    }
    }
}

// one fused launch from f[from] into f[from ^ 1] (no swap): steps_per_launch(h)
// steps, or exactly one step when `single` is set
static hipError_t enqueue_step(sc_lbm* h, int from, bool single = false)
{
    const sc_lbm_params& p = h->p;
    if (p.precision == SC_FP32_SHIFTED) {
        StepArgs<float> a = h->af;
        a.fin = (const float*)h->f[from];
        a.fout = (float*)h->f[from ^ 1];
        return launch_family(h, a, single);
    }
    StepArgs<double> a = h->ad;
    a.fin = (const double*)h->f[from];
    a.fout = (double*)h->f[from ^ 1];
    return launch_family(h, a, single);
}

static hipError_t build_graph(sc_lbm* h, int from)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    const int launches = kGraphSteps / steps_per_launch(h);   // even: the graph keeps the buffer parity
    for (int k = 0; k < launches && le == hipSuccess; ++k) le = enqueue_step(h, from ^ (k & 1));
    e = hipStreamEndCapture(h->stream, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec[from], g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    return e;
}

// enqueue `count` steps (asynchronous)
static hipError_t run_steps(sc_lbm* h, int64_t count)
{
    hipError_t e = hipSuccess;
    while (count >= kGraphSteps && !h->graph_failed) {
        if (!h->gexec[h->cur]) {
            e = build_graph(h, h->cur);
            if (e != hipSuccess) {
                // capture unsupported on this stream: fall back to plain launches
                (void)hipGetLastError();
                h->graph_failed = true;
                break;
            }
        }
        e = hipGraphLaunch(h->gexec[h->cur], h->stream);
        if (e != hipSuccess) return e;
        count -= kGraphSteps;
        h->step += kGraphSteps;
    }
    const int spl = steps_per_launch(h);
    while (count > 0) {
        const bool single = count < spl;
        e = enqueue_step(h, h->cur, single);
        if (e != hipSuccess) return e;
        const int adv = single ? 1 : spl;
        h->cur ^= 1;
        h->step += adv;
        count -= adv;
    }
    return hipSuccess;
}

// enqueue `count` steps as direct launches starting from buffer `from`;
// *end receives the buffer that then holds the state
static hipError_t enqueue_steps(sc_lbm* h, int from, int64_t count, int* end)
{
    const int spl = steps_per_launch(h);
    int p = from;
    while (count > 0) {
        const bool single = count < spl;
        hipError_t e = enqueue_step(h, p, single);
        if (e != hipSuccess) return e;
        p ^= 1;
        count -= single ? 1 : spl;
    }
    *end = p;
    return hipSuccess;
}

static int ensure_check(sc_lbm* h)
{
    if (h->chk_host) return SC_OK;
    const int nb = check_blocks(h->p.lattice, h->p.nx, h->p.ny, h->p.nz);
    hipError_t e = hipMalloc(&h->chk_partials, sizeof(double) * kObsSlots * nb);
    if (e == hipSuccess) e = hipMalloc(&h->chk_result, sizeof(double) * kCheckSlots);
    if (e == hipSuccess) e = hipHostMalloc(&h->chk_host, sizeof(double) * kCheckSlots, hipHostMallocDefault);
    if (e != hipSuccess) {
        hipFree(h->chk_partials);
        hipFree(h->chk_result);
        h->chk_partials = h->chk_result = nullptr;
        h->chk_host = nullptr;
        return hip_err(e);
    }
    return SC_OK;
}

// the fused check of buffer `buf` into the given partials and result
// block, and the result's copy to host memory `dst` (asynchronous)
static hipError_t enqueue_check_into(sc_lbm* h, int buf, double* partials, double* result, double* dst)
{
    hipError_t e = launch_check(h->p.lattice, h->p.precision, h->p.order, h->f[buf], args_ptr(h), partials,
                                result, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dst, result, sizeof(double) * kCheckSlots, hipMemcpyDeviceToHost, h->stream);
    return e;
}

static hipError_t enqueue_check(sc_lbm* h, int buf)
{
    return enqueue_check_into(h, buf, h->chk_partials, h->chk_result, h->chk_host);
}

// K steps and the check of their result as one graph replay (built on first
// use per start buffer); falls back to direct launches when the stream does
// not capture.  Advances h->cur and h->step.
static hipError_t run_chunk(sc_lbm* h, int64_t K)
{
    const int from = h->cur;
    if (!h->graph_failed && !h->gchunk[from]) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            int end = from;
            hipError_t le = enqueue_steps(h, from, K, &end);
            if (le == hipSuccess) le = enqueue_check(h, end);
            e = hipStreamEndCapture(h->stream, &g);
            if (le != hipSuccess) e = le;
            if (e == hipSuccess) e = hipGraphInstantiate(&h->gchunk[from], g, nullptr, nullptr, 0);
            if (g) hipGraphDestroy(g);
            h->gchunk_end[from] = end;
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->gchunk[from] = nullptr;
            h->graph_failed = true;
        }
    }
    hipError_t e;
    if (h->gchunk[from]) {
        e = hipGraphLaunch(h->gchunk[from], h->stream);
        if (e != hipSuccess) return e;
        h->cur = h->gchunk_end[from];
    } else {
        int end = from;
        e = enqueue_steps(h, from, K, &end);
        if (e == hipSuccess) e = enqueue_check(h, end);
        if (e != hipSuccess) return e;
        h->cur = end;
    }
    h->step += K;
    return hipSuccess;
}

static int ensure_obs(sc_lbm* h)
{
    if (h->obs.ready) return SC_OK;
    ObsBuffers& b = h->obs.b;
    const int64_t n = h->n;
    b.nblk = (int)std::min<int64_t>(1024, (n + 255) / 256);
    if (b.nblk < 1) b.nblk = 1;
    hipError_t e = hipMalloc(&b.rho, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&b.psi, h->tsize * n);
    if (e == hipSuccess) e = hipMalloc(&b.j, sizeof(double) * 3 * n);
    if (e == hipSuccess) e = hipMalloc(&b.F, sizeof(double) * 3 * n);
    if (e == hipSuccess) e = hipMalloc(&b.u, sizeof(double) * 3 * n);
    if (e == hipSuccess) e = hipMalloc(&b.partials, sizeof(double) * kObsSlots * b.nblk);
    if (e == hipSuccess) e = hipMalloc(&b.result, sizeof(double) * kObsSlots);
    if (e != hipSuccess) {
        hipFree(b.rho);
        hipFree(b.psi);
        hipFree(b.j);
        hipFree(b.F);
        hipFree(b.u);
        hipFree(b.partials);
        hipFree(b.result);
        b = ObsBuffers{};
        return hip_err(e);
    }
    h->obs.ready = true;
    return SC_OK;
}

static const void* args_ptr(sc_lbm* h) { return h->p.precision == SC_FP64 ? (const void*)&h->ad : (const void*)&h->af; }

static void fill_obs(const sc_lbm* h, const double* res, double rin, double rout, double psi_in, double psi_out,
                     sc_lbm_obs* o);

// fields + reductions of the current state; fills obs (except convergence fields)
static int observe_core(sc_lbm* h, sc_lbm_obs* o)
{
    int rc = ensure_obs(h);
    if (rc != SC_OK) return rc;
    ObsBuffers& b = h->obs.b;
    const sc_lbm_params& p = h->p;
    hipError_t e = launch_macro(p.lattice, p.precision, h->f[h->cur], args_ptr(h), b, h->stream);
    if (e == hipSuccess) e = launch_force(h->dim, p.precision, p.order, args_ptr(h), b, true, h->stream);
    if (e == hipSuccess) e = launch_reduce(h->dim, b, h->solid, h->n, h->stream);
    double res[kObsSlots];
    if (e == hipSuccess) e = hipMemcpyAsync(res, b.result, sizeof(res), hipMemcpyDeviceToHost, h->stream);
    const int64_t ic = (int64_t)(p.nx / 2) + (int64_t)p.nx * ((int64_t)(p.ny / 2) + (int64_t)p.ny * (p.nz / 2));
    double rin = 0, rout = 0;
    double psi_pair[2] = {0, 0};
    float psi_pair_f[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(&rin, b.rho + ic, sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&rout, b.rho, sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (p.precision == SC_FP64) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(&psi_pair[0], (double*)b.psi + ic, 8, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&psi_pair[1], (double*)b.psi, 8, hipMemcpyDeviceToHost, h->stream);
    } else {
        if (e == hipSuccess)
            e = hipMemcpyAsync(&psi_pair_f[0], (float*)b.psi + ic, 4, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&psi_pair_f[1], (float*)b.psi, 4, hipMemcpyDeviceToHost, h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(e);
    if (p.precision != SC_FP64) {
        psi_pair[0] = psi_pair_f[0];
        psi_pair[1] = psi_pair_f[1];
    }
    fill_obs(h, res, rin, rout, psi_pair[0], psi_pair[1], o);
    return SC_OK;
}

// sc_lbm_obs (all but converged_by) from the reduction slots and the
// (rho, psi) pair at the centre node and node 0
static void fill_obs(const sc_lbm* h, const double* res, double rin, double rout, double psi_in, double psi_out,
                     sc_lbm_obs* o)
{
    const sc_lbm_params& p = h->p;
    const double cs2 = lattice_cs2(p.lattice);
    const double pin = cs2 * rin + 0.5 * p.G * p.c0 * psi_in * psi_in;
    const double pout = cs2 * rout + 0.5 * p.G * p.c0 * psi_out * psi_out;
    std::memset(o, 0, sizeof(*o));
    o->step = h->step;
    o->mass = res[0];
    o->mom[0] = res[1];
    o->mom[1] = res[2];
    o->mom[2] = res[3];
    o->max_u = res[4];
    const double nfin = res[8];   // finite fluid nodes
    o->rho_max = nfin > 0 ? res[9] : std::nan("");
    o->rho_min = nfin > 0 ? -res[10] : std::nan("");
    o->mean_u = nfin > 0 ? res[5] / nfin : 0.0;
    o->l2_u = nfin > 0 ? std::sqrt(res[6] / nfin) : 0.0;
    o->nonfinite = (int64_t)res[7];
    o->rho_in = rin;
    o->rho_out = rout;
    o->p_in = pin;
    o->p_out = pout;
    o->dp = pin - pout;
    double vol = (rin != rout) ? (res[0] - (double)h->n * rout) / (rin - rout) : 0.0;
    if (vol < 0) vol = 0;
    o->radius = h->dim == 2 ? std::sqrt(vol / M_PI) : std::cbrt(3.0 * vol / (4.0 * M_PI));
    o->d_max_u = h->last_max_u >= 0 ? std::fabs(o->max_u - h->last_max_u) : -1.0;
    o->status = o->nonfinite ? SC_E_NONFINITE : SC_OK;
}

// the observables of a check result block (kCheckSlots doubles)
static void obs_from_check(const sc_lbm* h, const double* res, sc_lbm_obs* o)
{
    fill_obs(h, res, res[kObsSlots], res[kObsSlots + 2], res[kObsSlots + 1], res[kObsSlots + 3], o);
}

// sum_b |c_b| w_b of each lattice
static double lattice_cw(int lattice)
{
    switch (lattice) {
    case SC_D2Q9: return 4.0 / 9.0 + 4.0 * std::sqrt(2.0) / 36.0;
    case SC_D3Q19: return 6.0 / 18.0 + 12.0 * std::sqrt(2.0) / 36.0;
    case SC_D2Q13: return 4.0 * (8.0 / 75.0) + 4.0 * std::sqrt(2.0) / 25.0 + 4.0 * 2.0 / 300.0;
    case SC_D2Q25:
        return 4.0 * (16.0 / 147.0) + 4.0 * std::sqrt(2.0) * (16.0 / 315.0) + 4.0 * 2.0 / 105.0 +
               8.0 * std::sqrt(5.0) * (8.0 / 2205.0) + 4.0 * std::sqrt(8.0) / 8820.0;
    default: return 1.0;
    }
}

// Smallest change of max|u| an FP32 state resolves: each stored
// g_b = f_b - w_b rho_ref is rounded to 2^-24 of its size, at most
// w_b max(1, |rho - rho_ref|); u = (sum_b g_b c_b + F/2) / rho sums them with
// weights |c_b| and divides by rho.  Taken with a factor 4 for the sums, and
// never below 4 ulp of max|u| itself.
static double fp32_u_floor(const sc_lbm_params& p, const sc_lbm_obs& o)
{
    const double ulp4 = 4.0 * o.max_u * 1.1920928955078125e-7;
    if (!(o.rho_min > 0.0)) return ulp4;
    const double big = std::max(1.0, std::max(std::fabs(o.rho_max - p.rho_ref), std::fabs(o.rho_min - p.rho_ref)));
    return std::max(ulp4, 4.0 * 5.9604644775390625e-8 * lattice_cw(p.lattice) * big / o.rho_min);
}

// Records this check's max|u|.  An FP32 run is at its resolution when the
// max|u| of its last 50 checks scatter around their least-squares line by
// no more than one band of fp32_u_floor, and that line, carried on for 300
// more checks, moves by less than the band too.  Round-off noise of the
// state stays inside the band; a drift of d per check shows as a slope and
// keeps the run going down to d ~ band / 300 (droplets have slow modes that
// drift by ~1e-8 per check for 10^4 - 10^5 steps).  Measured on the sweep's
// droplets against their FP64 runs, this stops where a flat 100-check band
// did, 30% sooner, with the same steady max|u|.
static bool fp32_at_resolution(sc_lbm* h, const sc_lbm_obs& o)
{
    h->umax_hist[h->umax_n % kFloorWindow] = o.max_u;
    ++h->umax_n;
    if (h->p.precision != SC_FP32_SHIFTED || h->umax_n < kFloorWindow) return false;
    // the window in time order, t centred on its middle
    double v[kFloorWindow], mean = 0.0;
    for (int k = 0; k < kFloorWindow; ++k) {
        v[k] = h->umax_hist[(h->umax_n + k) % kFloorWindow];
        mean += v[k];
    }
    mean /= kFloorWindow;
    double stt = 0.0, sty = 0.0;
    for (int k = 0; k < kFloorWindow; ++k) {
        const double t = k - 0.5 * (kFloorWindow - 1);
        stt += t * t;
        sty += t * (v[k] - mean);
    }
    const double slope = sty / stt;
    double lo = 1e300, hi = -1e300;
    for (int k = 0; k < kFloorWindow; ++k) {
        const double r = v[k] - mean - slope * (k - 0.5 * (kFloorWindow - 1));
        lo = std::min(lo, r);
        hi = std::max(hi, r);
    }
    const double band = fp32_u_floor(h->p, o);
    return hi - lo <= band && std::fabs(slope) * kFloorHorizon <= band;
}

static void reset_convergence(sc_lbm* h)
{
    h->last_max_u = -1.0;
    h->umax_n = 0;
    h->conv_by = 0;
    h->tol_hits = 0;
}

// The tolerance rule: |max_u - previous max_u| < tol.  An FP32 state's
// round-off moves max_u by ~1e-7 per check near a steady state, so a single
// check (or a turning point of max_u) can fall below a small tol by chance;
// FP32 runs need it on 3 consecutive checks.
static bool tol_rule(sc_lbm* h, const sc_lbm_obs& o, double tol)
{
    const bool below = o.d_max_u >= 0 && o.d_max_u < tol;
    h->tol_hits = below ? h->tol_hits + 1 : 0;
    return h->p.precision == SC_FP64 ? below : h->tol_hits >= 3;
}

extern "C" int sc_lbm_step(sc_lbm* h, int64_t max_steps, double tol, int64_t* steps_done)
{
    if (!h || max_steps < 0 || !(tol >= 0.0)) return SC_E_INVAL;
    const int64_t start = h->step;
    h->conv_by = 0;
    if (tol == 0.0) {
        hipError_t e = run_steps(h, max_steps);
        if (steps_done) *steps_done = h->step - start;
        return hip_err(e);
    }
    const int64_t K = h->p.obs_every;
    int64_t left = max_steps;
    int rc = ensure_check(h);
    while (rc == SC_OK && left > 0) {
        // K steps and the fused check of their result as one graph replay,
        // then one wait for the result block in pinned host memory
        hipError_t e;
        if (left >= K) {
            e = run_chunk(h, K);
            left -= K;
        } else {
            e = run_steps(h, left);
            if (e == hipSuccess) e = enqueue_check(h, h->cur);
            left = 0;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            rc = hip_err(e);
            break;
        }
        sc_lbm_obs o;
        obs_from_check(h, h->chk_host, &o);
        if (o.nonfinite) {
            rc = SC_E_NONFINITE;
            break;
        }
        const bool floor = fp32_at_resolution(h, o);
        const bool tol_ok = tol_rule(h, o, tol);
        h->conv_by = tol_ok ? 1 : (floor ? 2 : 0);
        const bool done = tol_ok || floor;
        h->last_max_u = o.max_u;
        if (done) break;
    }
    if (steps_done) *steps_done = h->step - start;
    return rc;
}

extern "C" int sc_lbm_check(sc_lbm* h, sc_lbm_obs* obs)
{
    if (!h || !obs) return SC_E_INVAL;
    int rc = ensure_check(h);
    if (rc != SC_OK) return rc;
    hipError_t e = enqueue_check(h, h->cur);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(e);
    obs_from_check(h, h->chk_host, obs);
    obs->converged_by = h->conv_by;
    return obs->nonfinite ? SC_E_NONFINITE : SC_OK;
}

extern "C" int sc_lbm_check_noalloc(sc_lbm* h, sc_lbm_obs* obs)
{
    if (!h || !obs) return SC_E_INVAL;
    if (!h->scratch) return SC_E_DEVICE;   // hipGetSymbolAddress failed at creation (detail recorded)
    const int nb = check_blocks(h->p.lattice, h->p.nx, h->p.ny, h->p.nz);
    if ((int64_t)nb * kObsSlots + kCheckSlots > kScratchDoubles) {
        std::snprintf(g_detail, sizeof(g_detail), "sc_lbm_check_noalloc: %d partial rows exceed the scratch (%d)",
                      nb, kCheckMaxBlocks);
        return SC_E_UNSUPPORTED;
    }
    // the partials are written in full by every block and the result block
    // by the final pass and the two pressure nodes: nothing to clear
    double* partials = h->scratch;
    double* result = h->scratch + (size_t)nb * kObsSlots;
    double res[kCheckSlots];
    hipError_t e = enqueue_check_into(h, h->cur, partials, result, res);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(e);
    obs_from_check(h, res, obs);
    obs->converged_by = h->conv_by;
    return obs->nonfinite ? SC_E_NONFINITE : SC_OK;
}

extern "C" int sc_lbm_observe(sc_lbm* h, sc_lbm_obs* obs, double* rho_out, double* u_out, void* f_out)
{
    if (!h) return SC_E_INVAL;
    sc_lbm_obs o;
    int rc = observe_core(h, &o);
    if (rc != SC_OK) return rc;
    o.converged_by = h->conv_by;
    ObsBuffers& b = h->obs.b;
    hipError_t e = hipSuccess;
    if (rho_out) e = hipMemcpyAsync(rho_out, b.rho, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && u_out)
        e = hipMemcpyAsync(u_out, b.u, sizeof(double) * h->dim * h->n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && f_out)
        e = hipMemcpyAsync(f_out, h->f[h->cur], h->tsize * h->q * h->n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(e);
    if (obs) *obs = o;
    return o.nonfinite ? SC_E_NONFINITE : SC_OK;
}

extern "C" int sc_lbm_force(sc_lbm* h, const double* psi_in, double* F_out)
{
    if (!h || !F_out) return SC_E_INVAL;
    int rc = ensure_obs(h);
    if (rc != SC_OK) return rc;
    ObsBuffers& b = h->obs.b;
    const sc_lbm_params& p = h->p;
    hipError_t e = hipSuccess;
    if (psi_in) {
        // stage the doubles in the u buffer, then convert to the state precision
        e = hipMemcpyAsync(b.u, psi_in, sizeof(double) * h->n, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = launch_psi_from_host(p.precision, b.u, b.psi, h->n, h->stream);
    } else {
        e = launch_macro(p.lattice, p.precision, h->f[h->cur], args_ptr(h), b, h->stream);
    }
    if (e == hipSuccess) e = launch_force(h->dim, p.precision, p.order, args_ptr(h), b, false, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(F_out, b.F, sizeof(double) * h->dim * h->n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return hip_err(e);
}

extern "C" int sc_lbm_set_state(sc_lbm* h, const void* f_in, int64_t step)
{
    if (!h || !f_in || step < 0) return SC_E_INVAL;
    hipError_t e = hipMemcpyAsync(h->f[h->cur], f_in, h->tsize * h->q * h->n, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(e);
    h->step = step;
    reset_convergence(h);
    return SC_OK;
}

// psi of the virtual wall density in FP64 (the kernels take it as a value)
static double host_psi(const sc_lbm_params& p, double rho)
{
    if (p.psi_kind == SC_PSI_IDENTITY) return rho;
    if (p.psi_kind == SC_PSI_PR) {
        const double br = p.eos_b * rho;
        const double pr = rho * p.eos_R * p.eos_T / (1.0 - br) -
                          p.eos_a * p.eos_alpha * rho * rho / (1.0 + 2.0 * br - br * br);
        const double arg = 2.0 * (pr - lattice_cs2(p.lattice) * rho) / (p.G * p.c0);
        return arg > 0.0 ? std::sqrt(arg) : 0.0;
    }
    return p.psi0 * (1.0 - std::exp(-rho / p.rho_psi));
}

extern "C" int sc_lbm_set_walls(sc_lbm* h, const uint8_t* solid, double rho_w)
{
    if (!h || !std::isfinite(rho_w)) return SC_E_INVAL;
    if (h->dim != 2) return SC_E_UNSUPPORTED;
    hipError_t e = hipStreamSynchronize(h->stream);   // kernels in flight may read the old mask
    if (e != hipSuccess) return hip_err(e);
    drop_graphs(h);   // captured graphs hold the old kernel arguments
    const Family before = handle_family(h);
    if (!solid) {
        hipFree(h->solid);
        h->solid = nullptr;
    } else {
        if (!h->solid) {
            e = hipMalloc(&h->solid, (size_t)h->n);
            if (e != hipSuccess) {
                h->solid = nullptr;
                return hip_err(e);
            }
        }
        e = hipMemcpyAsync(h->solid, solid, (size_t)h->n, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_err(e);
    }
    const double pw = host_psi(h->p, rho_w);
    h->af.solid = h->solid;
    h->ad.solid = h->solid;
    h->af.psi_w = (float)pw;
    h->ad.psi_w = pw;
    // a change of kernel family invalidates the launch shape index: back in
    // the parameters' own family take the requested (or tuned / automatic)
    // shape, in the any-lattice family its automatic one
    const Family now = handle_family(h);
    if (now != before) {
        if (now == family_of(h->p))
            h->variant = h->p.variant >= 0 ? h->p.variant : auto_variant(h->p, h->n);
        else
            h->variant = h->n < ((int64_t)1 << 20) ? 1 : 4;   // wide32x8r1 / wide128x16r2
    }
    reset_convergence(h);
    return SC_OK;
}

extern "C" const char* sc_lbm_last_error_detail(void) { return g_detail; }

extern "C" const char* sc_lbm_strerror(int code)
{
    switch (code) {
    case SC_OK: return "ok";
    case SC_E_INVAL: return "invalid argument";
    case SC_E_NOMEM: return "out of memory";
    case SC_E_DEVICE: return "HIP device or runtime error";
    case SC_E_UNSUPPORTED: return "unsupported parameter combination";
    case SC_E_NONFINITE: return "non-finite value in the state";
    default: return "unknown error";
    }
}

// =========================================================================
// Batched sweeps: many D2Q9 items advanced by one launch per step.
// =========================================================================

struct sc_lbm_batch {
    int n = 0;
    int precision = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<sc_lbm*> items;
    void* pool = nullptr;
    void* desc = nullptr;
    int2* work = nullptr;
    int nwork = 0;
    int work_cap = 0;
    // launch shape (batch_shape_*): one step per launch over `work`, or two
    // per launch over `work2` (its own tile size, tiles of an item in strip
    // order), with one-step launches over `work` for an odd remainder
    int shape = 0;
    int2* work2 = nullptr;
    std::vector<int> tiles2x, tiles2y;
    int nwork2 = 0;
    std::vector<int> tiles;       // tiles per item
    std::vector<int> active;      // 1 while the item is stepped
    std::vector<int> conv_by;     // 0 running, 1 tol rule, 2 FP32 floor, -1 non-finite
    int parity = 0;
    int64_t step = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    bool graph_failed = false;
    StepArgs<float> cf{};
    StepArgs<double> cd{};
    // steady-state check: (item, tile) entries, (item, first entry, count)
    // per active item, per-entry partials, per-item result rows on the
    // device and their pinned host copy; graphs of K steps plus the check
    int2* cwork = nullptr;
    int ncwork = 0;
    int4* citems = nullptr;
    int nactive = 0;
    std::vector<int> ctiles;      // check tiles per item
    double* cpartials = nullptr;
    double* cresults = nullptr;
    double* chost = nullptr;
    hipGraphExec_t gchunk[2] = {nullptr, nullptr};
    int gchunk_end[2] = {0, 1};
};

static void batch_drop_graphs(sc_lbm_batch* b)
{
    for (int k = 0; k < 2; ++k) {
        if (b->gexec[k]) hipGraphExecDestroy(b->gexec[k]);
        if (b->gchunk[k]) hipGraphExecDestroy(b->gchunk[k]);
        b->gexec[k] = nullptr;
        b->gchunk[k] = nullptr;
    }
}

static void batch_release(sc_lbm_batch* b)
{
    if (!b) return;
    batch_drop_graphs(b);
    hipFree(b->cwork);
    hipFree(b->citems);
    hipFree(b->cpartials);
    hipFree(b->cresults);
    if (b->chost) hipHostFree(b->chost);
    for (sc_lbm* h : b->items)
        if (h) release(h);
    hipFree(b->pool);
    hipFree(b->desc);
    hipFree(b->work);
    hipFree(b->work2);
    if (b->own_stream && b->stream) hipStreamDestroy(b->stream);
    delete b;
}

constexpr int kBatchStrip = 8;   // tile columns per strip of the two-step work list

static int batch_rebuild_work(sc_lbm_batch* b)
{
    std::vector<int2> w, w2, cw;
    std::vector<int4> ci;
    for (int i = 0; i < b->n; ++i)
        if (b->active[i]) {
            for (int t = 0; t < b->tiles[i]; ++t) w.push_back(make_int2(i, t));
            if (b->work2) {
                // strip order: strips of kStrip tile columns, rows down each strip
                const int ntx = b->tiles2x[i], nty = b->tiles2y[i];
                for (int x0 = 0; x0 < ntx; x0 += kBatchStrip)
                    for (int by = 0; by < nty; ++by)
                        for (int bx = x0; bx < std::min(ntx, x0 + kBatchStrip); ++bx)
                            w2.push_back(make_int2(i, by * ntx + bx));
            }
            ci.push_back(make_int4(i, (int)cw.size(), b->ctiles[i], 0));
            for (int t = 0; t < b->ctiles[i]; ++t) cw.push_back(make_int2(i, t));
        }
    b->nwork = (int)w.size();
    b->nwork2 = (int)w2.size();
    b->ncwork = (int)cw.size();
    b->nactive = (int)ci.size();
    batch_drop_graphs(b);
    if (w.empty()) return SC_OK;
    hipError_t e = hipMemcpyAsync(b->work, w.data(), sizeof(int2) * w.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && b->work2)
        e = hipMemcpyAsync(b->work2, w2.data(), sizeof(int2) * w2.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->cwork, cw.data(), sizeof(int2) * cw.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->citems, ci.data(), sizeof(int4) * ci.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return hip_err(e);
}

// one step of the active items from buffer parity `parity`
static hipError_t batch_enqueue(sc_lbm_batch* b, int parity)
{
    const void* common = b->precision == SC_FP64 ? (const void*)&b->cd : (const void*)&b->cf;
    return launch_batch_d2q9(0, b->desc, b->work, b->nwork, parity, b->precision, common, b->stream);
}

// enqueue `count` steps for the active items as direct launches, from
// parity `from` (two per launch where the shape blocks two steps); *end
// receives the parity after them
static hipError_t batch_enqueue_steps(sc_lbm_batch* b, int from, int64_t count, int* end)
{
    const void* common = b->precision == SC_FP64 ? (const void*)&b->cd : (const void*)&b->cf;
    int p = from;
    if (batch_shape_steps(b->shape) == 2)
        for (; count >= 2; count -= 2) {
            hipError_t e = launch_batch_d2q9(b->shape, b->desc, b->work2, b->nwork2, p, b->precision, common,
                                             b->stream);
            if (e != hipSuccess) return e;
            p ^= 1;
        }
    for (; count > 0; --count) {
        hipError_t e = batch_enqueue(b, p);
        if (e != hipSuccess) return e;
        p ^= 1;
    }
    *end = p;
    return hipSuccess;
}

// the fused check of every active item's buffer `parity` and the copy of
// the result rows to pinned host memory (asynchronous)
static hipError_t batch_enqueue_check(sc_lbm_batch* b, int parity)
{
    const void* common = b->precision == SC_FP64 ? (const void*)&b->cd : (const void*)&b->cf;
    hipError_t e = launch_batch_check(b->desc, b->cwork, b->ncwork, b->citems, b->nactive, parity, b->precision,
                                      common, b->cpartials, b->cresults, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->chost, b->cresults, sizeof(double) * kCheckSlots * b->n, hipMemcpyDeviceToHost,
                           b->stream);
    return e;
}

// the active items now hold their state in buffer b->parity, `advanced`
// steps on (each item counts its own steps: items retired and brought back
// by sc_lbm_batch_promote differ)
static void batch_sync_items(sc_lbm_batch* b, int64_t advanced)
{
    for (int i = 0; i < b->n; ++i)
        if (b->active[i]) {
            b->items[i]->cur = b->parity;
            b->items[i]->step += advanced;
        }
}

// enqueue `count` steps for the active items (asynchronous): graphs of
// kGraphSteps steps (an even number of launches, so a graph keeps the buffer
// parity), the remainder as direct launches
static hipError_t batch_run(sc_lbm_batch* b, int64_t count)
{
    hipError_t e = hipSuccess;
    const int64_t start = b->step;
    while (count >= kGraphSteps && !b->graph_failed && b->nwork > 0) {
        if (!b->gexec[b->parity]) {
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                int end = b->parity;
                hipError_t le = batch_enqueue_steps(b, b->parity, kGraphSteps, &end);
                e = hipStreamEndCapture(b->stream, &g);
                if (le != hipSuccess) e = le;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec[b->parity], g, nullptr, nullptr, 0);
            if (g) hipGraphDestroy(g);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                b->gexec[b->parity] = nullptr;
                b->graph_failed = true;
                break;
            }
        }
        e = hipGraphLaunch(b->gexec[b->parity], b->stream);
        if (e != hipSuccess) return e;
        count -= kGraphSteps;
        b->step += kGraphSteps;
    }
    if (count > 0) {
        int end = b->parity;
        e = batch_enqueue_steps(b, b->parity, count, &end);
        if (e != hipSuccess) return e;
        b->parity = end;
        b->step += count;
    }
    batch_sync_items(b, b->step - start);
    return hipSuccess;
}

// K steps of the active items and their check as one graph replay (built
// on first use per start parity, dropped when the work list changes)
static hipError_t batch_run_chunk(sc_lbm_batch* b, int64_t K)
{
    const int from = b->parity;
    if (!b->graph_failed && !b->gchunk[from]) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            int end = from;
            hipError_t le = batch_enqueue_steps(b, from, K, &end);
            if (le == hipSuccess) le = batch_enqueue_check(b, end);
            e = hipStreamEndCapture(b->stream, &g);
            if (le != hipSuccess) e = le;
            if (e == hipSuccess) e = hipGraphInstantiate(&b->gchunk[from], g, nullptr, nullptr, 0);
            if (g) hipGraphDestroy(g);
            b->gchunk_end[from] = end;
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b->gchunk[from] = nullptr;
            b->graph_failed = true;
        }
    }
    hipError_t e;
    if (b->gchunk[from]) {
        e = hipGraphLaunch(b->gchunk[from], b->stream);
        if (e != hipSuccess) return e;
        b->parity = b->gchunk_end[from];
    } else {
        int end = from;
        e = batch_enqueue_steps(b, from, K, &end);
        if (e == hipSuccess) e = batch_enqueue_check(b, end);
        if (e != hipSuccess) return e;
        b->parity = end;
    }
    b->step += K;
    batch_sync_items(b, K);
    return hipSuccess;
}

extern "C" int sc_lbm_batch_create(const sc_lbm_params* items, int32_t n, const double* const* rho_init,
                                   void* hip_stream, sc_lbm_batch** out)
{
    if (!items || n < 1 || !out) return SC_E_INVAL;
    for (int i = 0; i < n; ++i) {
        int rc = validate(&items[i]);
        if (rc != SC_OK) return rc;
        if (items[i].lattice != SC_D2Q9 || items[i].collision != SC_SRT || items[i].forcing != SC_GUO ||
            items[i].psi_kind == SC_PSI_PR)
            return SC_E_UNSUPPORTED;
        if (items[i].precision != items[0].precision || items[i].psi_kind != items[0].psi_kind ||
            items[i].psi0 != items[0].psi0 || items[i].rho_psi != items[0].rho_psi ||
            items[i].rho_ref != items[0].rho_ref)
            return SC_E_INVAL;
    }
    std::vector<sc_lbm_params> its;
    try {
        its.assign(items, items + n);
        if (items[0].rho_ref < 0.0) {
            std::vector<double> smp;
            for (int i = 0; i < n; ++i)
                sample_density(rho_init ? rho_init[i] : nullptr, (int64_t)items[i].nx * items[i].ny,
                               std::max<int64_t>(1, kShiftSamples / n), smp);
            const double shift = median_density(smp);
            for (auto& it : its) it.rho_ref = shift;
        }
    } catch (const std::bad_alloc&) {
        return SC_E_NOMEM;
    }
    sc_lbm_batch* b = new (std::nothrow) sc_lbm_batch();
    if (!b) return SC_E_NOMEM;
    b->n = n;
    b->precision = items[0].precision;
    hipError_t e;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreate(&b->stream);
        if (e != hipSuccess) {
            delete b;
            return hip_err(e);
        }
        b->own_stream = true;
    }
    std::vector<size_t> off(n);
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        off[i] = total;
        total += 2 * ((sc_lbm_state_bytes(&items[i]) + 255) / 256 * 256);
    }
    e = hipMalloc(&b->pool, total);
    if (e == hipSuccess) e = hipMalloc(&b->desc, batch_item_bytes(b->precision) * n);
    int64_t ntiles = 0;
    int tw = 0, th = 0;
    batch_shape_tile(0, &tw, &th);
    for (int i = 0; i < n; ++i) {
        const int t = ((items[i].nx + tw - 1) / tw) * ((items[i].ny + th - 1) / th);
        b->tiles.push_back(t);
        ntiles += t;
    }
    b->shape = (items[0].variant >= 0 && items[0].variant < batch_num_shapes())
                   ? items[0].variant
                   : (b->precision == SC_FP64 ? kBatchShapeFP64 : kBatchShapeFP32);
    int64_t ntiles2 = 0;
    if (batch_shape_steps(b->shape) == 2) {
        int t2w = 0, t2h = 0;
        batch_shape_tile(b->shape, &t2w, &t2h);
        for (int i = 0; i < n; ++i) {
            b->tiles2x.push_back((items[i].nx + t2w - 1) / t2w);
            b->tiles2y.push_back((items[i].ny + t2h - 1) / t2h);
            ntiles2 += (int64_t)b->tiles2x.back() * b->tiles2y.back();
        }
    }
    int64_t nctiles = 0;
    const int ct = batch_check_tile();
    for (int i = 0; i < n; ++i) {
        const int t = ((items[i].nx + ct - 1) / ct) * ((items[i].ny + ct - 1) / ct);
        b->ctiles.push_back(t);
        nctiles += t;
    }
    if (ntiles > 0x7fffffff || nctiles > 0x7fffffff || ntiles2 > 0x7fffffff) e = hipErrorInvalidValue;
    if (e == hipSuccess && ntiles2 > 0) e = hipMalloc(&b->work2, sizeof(int2) * (size_t)ntiles2);
    b->work_cap = (int)ntiles;
    if (e == hipSuccess) e = hipMalloc(&b->work, sizeof(int2) * (size_t)ntiles);
    if (e == hipSuccess) e = hipMalloc(&b->cwork, sizeof(int2) * (size_t)nctiles);
    if (e == hipSuccess) e = hipMalloc(&b->citems, sizeof(int4) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&b->cpartials, sizeof(double) * kObsSlots * (size_t)nctiles);
    if (e == hipSuccess) e = hipMalloc(&b->cresults, sizeof(double) * kCheckSlots * (size_t)n);
    if (e == hipSuccess) e = hipHostMalloc(&b->chost, sizeof(double) * kCheckSlots * (size_t)n, hipHostMallocDefault);
    if (e != hipSuccess) {
        int rc = hip_err(e);
        batch_release(b);
        return rc;
    }
    std::vector<unsigned char> desc(batch_item_bytes(b->precision) * n);
    for (int i = 0; i < n; ++i) {
        char* base = (char*)b->pool + off[i];
        const size_t half = (sc_lbm_state_bytes(&items[i]) + 255) / 256 * 256;
        sc_lbm* h = nullptr;
        int rc = sc_lbm_create(&its[i], rho_init ? rho_init[i] : nullptr, base, base + half, b->stream, &h);
        if (rc != SC_OK) {
            batch_release(b);
            return rc;
        }
        b->items.push_back(h);
        batch_fill_item(desc.data() + batch_item_bytes(b->precision) * i, b->precision, base, base + half,
                        items[i].nx, items[i].ny, items[i].order, items[i].G * items[i].c0, items[i].tau);
    }
    b->active.assign(n, 1);
    b->conv_by.assign(n, 0);
    fill_args(b->items[0], b->cf);
    fill_args(b->items[0], b->cd);
    e = hipMemcpyAsync(b->desc, desc.data(), desc.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    int rc = hip_err(e);
    if (rc == SC_OK) rc = batch_rebuild_work(b);
    if (rc != SC_OK) {
        batch_release(b);
        return rc;
    }
    *out = b;
    return SC_OK;
}

extern "C" int sc_lbm_batch_step(sc_lbm_batch* b, int64_t max_steps, double tol, int64_t* steps_done)
{
    if (!b || max_steps < 0 || !(tol >= 0.0)) return SC_E_INVAL;
    const int64_t start = b->step;
    int rc = SC_OK;
    if (tol == 0.0) {
        rc = hip_err(batch_run(b, max_steps));
        if (steps_done) *steps_done = b->step - start;
        return rc;
    }
    const int64_t K = b->items[0]->p.obs_every;
    int64_t left = max_steps;
    while (left > 0 && b->nwork > 0) {
        // K steps of every active item and the fused check of each as one
        // graph replay, then one wait for all result rows
        hipError_t e;
        if (left >= K) {
            e = batch_run_chunk(b, K);
            left -= K;
        } else {
            e = batch_run(b, left);
            if (e == hipSuccess) e = batch_enqueue_check(b, b->parity);
            left = 0;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        rc = hip_err(e);
        if (rc != SC_OK) break;
        bool changed = false;
        for (int i = 0; i < b->n; ++i) {
            if (!b->active[i]) continue;
            sc_lbm* h = b->items[i];
            sc_lbm_obs o;
            obs_from_check(h, b->chost + (size_t)kCheckSlots * i, &o);
            int by = 0;
            const bool floor = fp32_at_resolution(h, o);
            const bool tol_ok = tol_rule(h, o, tol);
            if (o.nonfinite) by = -1;
            else if (tol_ok) by = 1;
            else if (floor) by = 2;
            h->last_max_u = o.max_u;
            if (by != 0) {
                b->active[i] = 0;
                b->conv_by[i] = by;
                changed = true;
            }
        }
        if (changed) {
            rc = batch_rebuild_work(b);
            if (rc != SC_OK) break;
        }
    }
    if (steps_done) *steps_done = b->step - start;
    return rc;
}

extern "C" int sc_lbm_batch_observe(sc_lbm_batch* b, int32_t item, sc_lbm_obs* obs, double* rho_out,
                                    double* u_out)
{
    if (!b || item < 0 || item >= b->n) return SC_E_INVAL;
    int rc = sc_lbm_observe(b->items[item], obs, rho_out, u_out, nullptr);
    if (obs) {
        obs->converged_by = b->conv_by[item] > 0 ? b->conv_by[item] : 0;
        if (b->conv_by[item] < 0) obs->status = SC_E_NONFINITE;
    }
    return rc;
}

extern "C" int sc_lbm_batch_status(sc_lbm_batch* b, int32_t item, int64_t* steps, int32_t* converged_by)
{
    if (!b || item < 0 || item >= b->n) return SC_E_INVAL;
    if (steps) *steps = b->items[item]->step;
    if (converged_by) *converged_by = b->conv_by[item];
    return SC_OK;
}

extern "C" int32_t sc_lbm_batch_active(sc_lbm_batch* b)
{
    if (!b) return 0;
    int32_t k = 0;
    for (int v : b->active) k += v;
    return k;
}

// free a handle's observation buffers (sized for its state precision)
static void drop_obs(sc_lbm* h)
{
    if (!h->obs.ready) return;
    ObsBuffers& o = h->obs.b;
    hipFree(o.rho);
    hipFree(o.psi);
    hipFree(o.j);
    hipFree(o.F);
    hipFree(o.u);
    hipFree(o.partials);
    hipFree(o.result);
    o = ObsBuffers{};
    h->obs.ready = false;
}

// Take the net momentum out of every widened item's state.  The step
// conserves momentum exactly, and every batch item starts with none (f at
// rest, and the interaction forces sum to zero on the periodic grid); the
// FP32 stage's rounding has gathered a little (a drift of ~1e-8 per step on
// the sweep's droplets), which the FP64 state would keep: its droplet would
// then cross the lattice and its max |u| keep changing, so the literal rule
// is never met.  Each node's populations take the equilibrium change of the
// uniform velocity -J/M at its own density; masses are unchanged.
static hipError_t batch_remove_momentum(sc_lbm_batch* b)
{
    const int nb = momentum_blocks();
    double* part = nullptr;
    hipError_t e = hipMalloc(&part, sizeof(double) * 3 * nb);
    std::vector<double> hp(3 * (size_t)nb);
    for (int i = 0; i < b->n && e == hipSuccess; ++i) {
        sc_lbm* h = b->items[i];
        double* g = (double*)h->f[h->cur];
        e = launch_d2q9_mass_momentum(g, h->n, part, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hp.data(), part, sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) break;
        double m = 0.0, jx = 0.0, jy = 0.0;
        for (int k = 0; k < nb; ++k) {
            m += hp[3 * k];
            jx += hp[3 * k + 1];
            jy += hp[3 * k + 2];
        }
        const double M = m + h->p.rho_ref * (double)h->n;
        if (!(M > 0.0) || !std::isfinite(M) || !std::isfinite(jx) || !std::isfinite(jy)) continue;   // quarantined
        e = launch_d2q9_momentum_shift(g, h->n, h->p.rho_ref, -jx / M, -jy / M, b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    hipFree(part);
    return e;
}

extern "C" int sc_lbm_batch_promote(sc_lbm_batch* b)
{
    if (!b || b->precision != SC_FP32_SHIFTED) return SC_E_INVAL;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_err(e);
    const int n = b->n;
    // FP64 buffers for every item, carved from one allocation like the FP32 ones
    std::vector<size_t> off(n), half(n);
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        const sc_lbm* h = b->items[i];
        half[i] = ((size_t)h->q * (size_t)h->n * 8 + 255) / 256 * 256;
        off[i] = total;
        total += 2 * half[i];
    }
    const int shape = kBatchShapeFP64;
    int t2w = 0, t2h = 0;
    batch_shape_tile(shape, &t2w, &t2h);
    std::vector<int> t2x(n), t2y(n);
    int64_t ntiles2 = 0;
    for (int i = 0; i < n; ++i) {
        t2x[i] = (b->items[i]->p.nx + t2w - 1) / t2w;
        t2y[i] = (b->items[i]->p.ny + t2h - 1) / t2h;
        ntiles2 += (int64_t)t2x[i] * t2y[i];
    }
    void* pool = nullptr;
    void* desc = nullptr;
    int2* work2 = nullptr;
    e = hipMalloc(&pool, total);
    if (e == hipSuccess) e = hipMalloc(&desc, batch_item_bytes(SC_FP64) * n);
    if (e == hipSuccess) e = hipMalloc(&work2, sizeof(int2) * (size_t)ntiles2);
    if (e != hipSuccess) {
        hipFree(pool);
        hipFree(desc);
        hipFree(work2);
        return hip_err(e);
    }
    std::vector<unsigned char> dd(batch_item_bytes(SC_FP64) * n);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        sc_lbm* h = b->items[i];
        double* a0 = (double*)((char*)pool + off[i]);
        double* a1 = (double*)((char*)pool + off[i] + half[i]);
        e = launch_widen((const float*)h->f[h->cur], a0, (int64_t)h->q * h->n, b->stream);
        drop_graphs(h);
        drop_obs(h);
        h->p.precision = SC_FP64;
        h->tsize = 8;
        h->f[0] = a0;
        h->f[1] = a1;
        h->cur = 0;
        fill_args(h, h->af);
        fill_args(h, h->ad);
        reset_convergence(h);
        batch_fill_item(dd.data() + batch_item_bytes(SC_FP64) * i, SC_FP64, a0, a1, h->p.nx, h->p.ny, h->p.order,
                        h->p.G * h->p.c0, h->p.tau);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(desc, dd.data(), dd.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = batch_remove_momentum(b);
    if (e != hipSuccess) {
        // the items may already point into the new pool: keep it (freed with the batch)
        hipFree(b->pool);
        b->pool = pool;
        hipFree(desc);
        hipFree(work2);
        return hip_err(e);
    }
    batch_drop_graphs(b);
    hipFree(b->pool);
    hipFree(b->desc);
    hipFree(b->work2);
    b->pool = pool;
    b->desc = desc;
    b->work2 = work2;
    b->tiles2x = t2x;
    b->tiles2y = t2y;
    b->shape = shape;
    b->precision = SC_FP64;
    b->parity = 0;
    fill_args(b->items[0], b->cd);
    for (int i = 0; i < n; ++i)
        if (b->conv_by[i] > 0) {   // retired by a convergence rule: back to work
            b->active[i] = 1;
            b->conv_by[i] = 0;
        }
    return batch_rebuild_work(b);
}

extern "C" const char* sc_lbm_batch_variant_name(const sc_lbm_batch* b) { return b ? batch_shape_name(b->shape) : ""; }

extern "C" int32_t sc_lbm_batch_num_variants(void) { return batch_num_shapes(); }

// Batched shape tuner: one scratch batch of the caller's items per shape
// (rho = 1 everywhere: the kernels do the same work whatever the values),
// each timed as sc_lbm_batch_step runs it -- a warm-up graph that also
// builds it, then the best of three runs of whole 32-step graphs.
extern "C" int sc_lbm_batch_autotune(const sc_lbm_params* items, int32_t n, int32_t steps, int32_t* best_variant,
                                     double* best_ms)
{
    if (!items || n < 1 || steps < 1) return SC_E_INVAL;
    const int64_t per_rep = ((std::max<int64_t>(steps, kGraphSteps) + kGraphSteps - 1) / kGraphSteps) * kGraphSteps;
    std::vector<sc_lbm_params> q(items, items + n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return hip_err(e);
    }
    int rc = SC_OK, best = -1;
    double bms = 1e300;
    for (int v = 0; v < batch_num_shapes() && rc == SC_OK; ++v) {
        q[0].variant = v;
        sc_lbm_batch* b = nullptr;
        rc = sc_lbm_batch_create(q.data(), n, nullptr, nullptr, &b);
        if (rc != SC_OK) break;
        e = batch_run(b, kGraphSteps);
        double per = 1e300;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, b->stream);
            if (e == hipSuccess) e = batch_run(b, per_rep);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) per = std::min(per, (double)ms / per_rep);
        }
        sc_lbm_batch_destroy(b);
        if (e != hipSuccess) {
            rc = hip_err(e);
            break;
        }
        if (per < bms) {
            bms = per;
            best = v;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc != SC_OK) return rc;
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = bms;
    return SC_OK;
}

extern "C" double sc_lbm_batch_rho_ref(const sc_lbm_batch* b)
{
    return (b && !b->items.empty()) ? b->items[0]->p.rho_ref : std::nan("");
}

extern "C" void sc_lbm_batch_destroy(sc_lbm_batch* b)
{
    if (!b) return;
    hipStreamSynchronize(b->stream);
    batch_release(b);
}

// =========================================================================
// Autotuner: time every launch shape on the caller's problem statement.
// =========================================================================
extern "C" int sc_lbm_autotune(const sc_lbm_params* p, int32_t steps, int32_t* best_variant, double* best_ms)
{
    int rc = validate(p);
    if (rc != SC_OK) return rc;
    if (steps < 1) return SC_E_INVAL;
    const int nv = family_variants(family_of(*p));
    int best = -1;
    double bms = 1e300;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return hip_err(e);
    }
    // one state pair for all candidates; each is timed the way sc_lbm_step
    // runs it (graph replay): a warm-up graph that also builds it, then the
    // best of three runs of whole graphs
    const int64_t per_rep = ((std::max<int64_t>(steps, kGraphSteps) + kGraphSteps - 1) / kGraphSteps) * kGraphSteps;
    sc_lbm_params q = *p;
    q.variant = 0;
    sc_lbm* h = nullptr;
    rc = sc_lbm_create(&q, nullptr, nullptr, nullptr, nullptr, &h);
    if (rc == SC_OK) {
        for (int v = 0; v < nv && rc == SC_OK; ++v) {
            h->variant = v;
            drop_graphs(h);
            e = run_steps(h, kGraphSteps);
            double per = 1e300;
            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, h->stream);
                if (e == hipSuccess) e = run_steps(h, per_rep);
                if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess) per = std::min(per, (double)ms / per_rep);
            }
            if (e != hipSuccess) {
                rc = hip_err(e);
                break;
            }
            if (per < bms) {
                bms = per;
                best = v;
            }
        }
        sc_lbm_destroy(h);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc != SC_OK) return rc;
    tune_store(*p, best, bms);
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = bms;
    return SC_OK;
}
