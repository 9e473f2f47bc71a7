// Calls the C ABI's entry points that validate their arguments before any
// device work, for a build whose host code has -fsanitize=address,undefined:
// parameter defaults and sizes, every rejection of sc_lbm_create /
// sc_lbm_batch_create / sc_lbm_autotune, NULL handles everywhere, the
// network kernels' size checks.  No GPU is needed.  Prints "ok" and exits 0
// when every call returned what the header says.  Test infrastructure only.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../../include/sc_lbm.h"

static int fails = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

int main()
{
    sc_lbm_params p;
    sc_lbm_default_params(&p);
    sc_lbm_default_params(nullptr);
    CHECK(sc_lbm_state_bytes(&p) == (size_t)9 * 64 * 64 * 4);
    CHECK(sc_lbm_num_variants(&p) > 0);
    sc_lbm_params q = p;
    q.lattice = SC_D3Q19;
    q.nz = 8;
    CHECK(sc_lbm_num_variants(&q) > 0);
    q = p;
    q.lattice = SC_D2Q25;
    CHECK(sc_lbm_num_variants(&q) > 0);
    for (int c = 1; c >= -6; --c) CHECK(sc_lbm_strerror(c) != nullptr && std::strlen(sc_lbm_strerror(c)) > 0);
    CHECK(sc_lbm_last_error_detail() != nullptr);

    // rejections before any device call
    sc_lbm* h = nullptr;
    const double rho[4] = {1.0, 1.0, 1.0, 1.0};
    struct Bad {
        const char* what;
        void (*edit)(sc_lbm_params&);
        int rc;
    };
    const Bad bad[] = {
        {"lattice", [](sc_lbm_params& x) { x.lattice = 9; }, SC_E_INVAL},
        {"nx", [](sc_lbm_params& x) { x.nx = 0; }, SC_E_INVAL},
        {"2D nz", [](sc_lbm_params& x) { x.nz = 2; }, SC_E_INVAL},
        {"order", [](sc_lbm_params& x) { x.order = 5; }, SC_E_INVAL},
        {"3D E10", [](sc_lbm_params& x) { x.lattice = SC_D3Q19; x.nz = 4; x.order = 10; }, SC_E_UNSUPPORTED},
        {"tau", [](sc_lbm_params& x) { x.tau = 0.5; }, SC_E_INVAL},
        {"tau NaN", [](sc_lbm_params& x) { x.tau = NAN; }, SC_E_INVAL},
        {"G inf", [](sc_lbm_params& x) { x.G = INFINITY; }, SC_E_INVAL},
        {"2D MRT", [](sc_lbm_params& x) { x.collision = SC_MRT; }, SC_E_UNSUPPORTED},
        {"3D EDM", [](sc_lbm_params& x) { x.lattice = SC_D3Q19; x.nz = 4; x.forcing = SC_EDM; }, SC_E_UNSUPPORTED},
        {"psi kind", [](sc_lbm_params& x) { x.psi_kind = 7; }, SC_E_INVAL},
        {"P-R b", [](sc_lbm_params& x) { x.psi_kind = SC_PSI_PR; x.eos_b = 0.0; }, SC_E_INVAL},
        {"precision", [](sc_lbm_params& x) { x.precision = 3; }, SC_E_INVAL},
        {"MRT rate", [](sc_lbm_params& x) { x.lattice = SC_D3Q19; x.nz = 4; x.collision = SC_MRT; x.s_bulk = 2.5; },
         SC_E_INVAL},
        {"obs_every", [](sc_lbm_params& x) { x.obs_every = -1; }, SC_E_INVAL},
        {"init", [](sc_lbm_params& x) { x.init = 4; }, SC_E_INVAL},
        {"variant", [](sc_lbm_params& x) { x.variant = 999; }, SC_E_INVAL},
        {"plane over 4 GiB", [](sc_lbm_params& x) { x.nx = 1 << 15; x.ny = 1 << 15; }, SC_E_UNSUPPORTED},
    };
    for (const Bad& b : bad) {
        sc_lbm_params x = p;
        b.edit(x);
        const int rc = sc_lbm_create(&x, nullptr, nullptr, nullptr, nullptr, &h);
        if (rc != b.rc) std::fprintf(stderr, "create(%s) returned %d\n", b.what, rc);
        CHECK(rc == b.rc && h == nullptr);
        CHECK(sc_lbm_state_bytes(&x) == 0 || b.rc == SC_OK);
    }
    int dummy = 0;
    CHECK(sc_lbm_create(nullptr, nullptr, nullptr, nullptr, nullptr, &h) == SC_E_INVAL);
    CHECK(sc_lbm_create(&p, nullptr, nullptr, nullptr, nullptr, nullptr) == SC_E_INVAL);
    CHECK(sc_lbm_create(&p, rho, &dummy, nullptr, nullptr, &h) == SC_E_INVAL);   // one buffer only
    CHECK(sc_lbm_create(&p, rho, &dummy, &dummy, nullptr, &h) == SC_E_INVAL);    // the same buffer twice
    sc_lbm_params nanp = p;
    nanp.nx = nanp.ny = 2;
    const double rho_nan[4] = {1.0, NAN, 1.0, 1.0};
    CHECK(sc_lbm_create(&nanp, rho_nan, nullptr, nullptr, nullptr, &h) == SC_E_INVAL);

    // NULL handles
    int64_t done = 0;
    sc_lbm_obs o;
    double buf[16];
    CHECK(sc_lbm_step(nullptr, 10, 0.0, &done) == SC_E_INVAL);
    CHECK(sc_lbm_observe(nullptr, &o, nullptr, nullptr, nullptr) == SC_E_INVAL);
    CHECK(sc_lbm_check(nullptr, &o) == SC_E_INVAL);
    CHECK(sc_lbm_check_noalloc(nullptr, &o) == SC_E_INVAL);
    CHECK(sc_lbm_force(nullptr, nullptr, buf) == SC_E_INVAL);
    CHECK(sc_lbm_set_state(nullptr, buf, 0) == SC_E_INVAL);
    CHECK(sc_lbm_set_walls(nullptr, nullptr, 1.0) == SC_E_INVAL);
    CHECK(sc_lbm_state_ptr(nullptr) == nullptr && sc_lbm_stream(nullptr) == nullptr);
    CHECK(std::isnan(sc_lbm_rho_ref(nullptr)) && sc_lbm_steps_per_launch(nullptr) == 0);
    CHECK(std::strcmp(sc_lbm_variant_name(nullptr), "") == 0);
    sc_lbm_destroy(nullptr);

    // batches
    sc_lbm_batch* b = nullptr;
    sc_lbm_params items[2] = {p, p};
    CHECK(sc_lbm_batch_create(nullptr, 2, nullptr, nullptr, &b) == SC_E_INVAL);
    CHECK(sc_lbm_batch_create(items, 0, nullptr, nullptr, &b) == SC_E_INVAL);
    items[1].precision = SC_FP64;
    CHECK(sc_lbm_batch_create(items, 2, nullptr, nullptr, &b) == SC_E_INVAL);   // mixed precision
    items[1] = p;
    items[1].forcing = SC_EDM;
    CHECK(sc_lbm_batch_create(items, 2, nullptr, nullptr, &b) == SC_E_UNSUPPORTED);
    items[1] = p;
    items[1].lattice = SC_D2Q13;
    CHECK(sc_lbm_batch_create(items, 2, nullptr, nullptr, &b) == SC_E_UNSUPPORTED);
    CHECK(b == nullptr);
    CHECK(sc_lbm_batch_step(nullptr, 10, 0.0, &done) == SC_E_INVAL);
    CHECK(sc_lbm_batch_observe(nullptr, 0, &o, nullptr, nullptr) == SC_E_INVAL);
    CHECK(sc_lbm_batch_status(nullptr, 0, &done, &dummy) == SC_E_INVAL);
    CHECK(sc_lbm_batch_promote(nullptr) == SC_E_INVAL);
    CHECK(sc_lbm_batch_active(nullptr) == 0 && std::isnan(sc_lbm_batch_rho_ref(nullptr)));
    CHECK(std::strcmp(sc_lbm_batch_variant_name(nullptr), "") == 0 && sc_lbm_batch_num_variants() > 1);
    sc_lbm_batch_destroy(nullptr);

    // autotune rejections
    int32_t best = 0;
    double ms = 0;
    sc_lbm_params bt = p;
    bt.tau = 0.2;
    CHECK(sc_lbm_autotune(&bt, 32, &best, &ms) == SC_E_INVAL);
    CHECK(sc_lbm_autotune(&p, 0, &best, &ms) == SC_E_INVAL);

    // network kernels: sizes and pointers are checked before any launch
    float f[4];
    uint16_t w16[4];
    double d[4];
    CHECK(sc_nn_conv3x3_fwd(nullptr, w16, f, f, 1, 1, 32, 4, 4, nullptr) == SC_E_INVAL);
    CHECK(sc_nn_conv3x3_fwd(f, w16, f, f, 1, 33, 32, 4, 4, nullptr) == SC_E_INVAL);   // cin > 32
    CHECK(sc_nn_conv3x3_fwd(f, w16, f, f, 1, 5, 7, 4, 4, nullptr) == SC_E_INVAL);     // cout not 1 or 32
    CHECK(sc_nn_conv3x3_fwd(f, w16, f, f, 0, 5, 32, 4, 4, nullptr) == SC_E_INVAL);    // batch 0
    CHECK(sc_nn_conv3x3_bwd_data(f, w16, w16, f, 1, 5, 32, 4, 4, nullptr) == SC_E_INVAL);   // cin must be 32
    CHECK(sc_nn_bwd_weight_scratch_floats(32, 32, 4) > 0);
    CHECK(sc_nn_start_field(f, d, d, d, 1, 4, 5, 1.0f, 0.0, 2.0, nullptr) == SC_E_INVAL);    // h != w
    CHECK(sc_nn_start_field(f, d, d, d, 1, 4, 4, 1.0f, 2.0, 0.0, nullptr) == SC_E_INVAL);    // lo > hi

    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
