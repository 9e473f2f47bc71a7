/*
 * Exercises every entry point of the FP64 oracle (oracle/sc_oracle.c, built
 * into this program) on tiny periodic grids, for a build with
 * -fsanitize=address,undefined: each lattice and force-stencil order, SRT and
 * MRT, Guo and the exact difference method, the three pseudo-potentials, the
 * rest start and walls.  Prints "ok" and exits 0 when every call succeeded;
 * the sanitizers abort on the first memory error or undefined behaviour.
 * Test infrastructure only.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int lattice, nx, ny, nz, order;
    double G, c0;
    int psi_kind;
    double psi0, rho_psi, tau;
    int collision;
    double s_bulk, s_ghost;
    int forcing;
    double pr_a, pr_b, pr_R, pr_T, pr_alpha;
    int init;
} orc_params;
typedef struct orc_sim orc_sim;

int orc_lattice(int lattice, int *dim, int *q, int (*c)[3], double *w, double *cs2);
int orc_stencil(int dim, int order, int (*e)[3], double *w);
orc_sim *orc_create(const orc_params *p, const double *rho0);
void orc_destroy(orc_sim *s);
int orc_set_walls(orc_sim *s, const unsigned char *solid, double rho_w);
void orc_step(orc_sim *s, long nsteps);
void orc_fields(orc_sim *s, double *rho, double *psi, double *F, double *u);
void orc_get_f(const orc_sim *s, double *f);
void orc_set_f(orc_sim *s, const double *f);
int orc_force(const orc_params *p, const double *psi, double *F);
int orc_mrt_basis(const orc_sim *s, double *M, double *norm, double *S);
int orc_num_threads(void);

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__);    \
            ++fails;                                                    \
        }                                                               \
    } while (0)

static void run(int lattice, int nx, int ny, int nz, int order, int collision, int forcing, int psi_kind, int init,
                int walls)
{
    orc_params p = {0};
    p.lattice = lattice;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.order = order;
    p.G = psi_kind == 2 ? -1.0 : -5.0;
    p.c0 = 1.0 / 3.0;
    p.psi_kind = psi_kind;
    p.psi0 = 1.0;
    p.rho_psi = 1.0;
    p.tau = 0.9;
    p.collision = collision;
    p.s_bulk = 0.7;
    p.s_ghost = 1.6;
    p.forcing = forcing;
    p.pr_a = 2.0 / 49.0;
    p.pr_b = 2.0 / 21.0;
    p.pr_R = 1.0;
    p.pr_T = 0.85 * 0.0729190;
    p.pr_alpha = 1.05;
    p.init = init;
    const long n = (long)nx * ny * nz;
    const int dim = nz > 1 ? 3 : 2;
    double *rho = malloc(sizeof(double) * n), *out = malloc(sizeof(double) * (2 + 2 * 3) * n);
    double *f = malloc(sizeof(double) * 25 * n);
    unsigned char *solid = calloc((size_t)n, 1);
    for (long i = 0; i < n; ++i) rho[i] = (psi_kind == 2 ? 0.5 : 1.0) + 0.3 * sin(0.7 * (double)i);
    orc_sim *s = orc_create(&p, rho);
    CHECK(s != NULL);
    if (!s) goto done;
    if (walls) {
        for (long i = 0; i < nx; ++i) solid[i] = 1;
        CHECK(orc_set_walls(s, solid, 1.2) == 0);
    }
    orc_step(s, 3);
    orc_fields(s, out, out + n, out + 2 * n, out + (2 + dim) * n);   /* rho, psi, F[dim], u[dim] */
    orc_get_f(s, f);
    orc_set_f(s, f);
    orc_step(s, 1);
    if (collision == 1) {
        double M[19 * 19], nn[19], S[19];
        CHECK(orc_mrt_basis(s, M, nn, S) == 0);
    }
    for (long i = 0; i < (2 + 2 * dim) * n; ++i) CHECK(isfinite(out[i]));
    CHECK(orc_force(&p, rho, out) == 0);
    orc_destroy(s);
done:
    free(rho);
    free(out);
    free(f);
    free(solid);
}

int main(void)
{
    int c[25][3], e[96][3], dim, q;
    double w[96], cs2;
    for (int l = 0; l < 4; ++l) CHECK(orc_lattice(l, &dim, &q, c, w, &cs2) == 0);
    CHECK(orc_lattice(7, &dim, &q, c, w, &cs2) != 0);
    for (int o = 4; o <= 10; o += 2) CHECK(orc_stencil(2, o, e, w) > 0);
    for (int o = 4; o <= 8; o += 2) CHECK(orc_stencil(3, o, e, w) > 0);
    CHECK(orc_stencil(3, 10, e, w) <= 0);
    for (int o = 4; o <= 10; o += 2) {
        run(0, 9, 7, 1, o, 0, 0, 0, 0, 0);     /* D2Q9 Guo */
        run(0, 9, 7, 1, o, 0, 1, 1, 1, 1);     /* D2Q9 EDM, psi = rho, rest start, walls */
        run(2, 11, 6, 1, o, 0, 1, 2, 0, 1);    /* D2Q13 EDM, Peng-Robinson, walls */
        run(3, 12, 5, 1, o, 0, 0, 0, 1, 0);    /* D2Q25 Guo, rest start */
        run(3, 3, 2, 1, o, 0, 1, 2, 0, 0);     /* D2Q25 on a grid narrower than its stencils */
    }
    for (int o = 4; o <= 8; o += 2) {
        run(1, 5, 4, 3, o, 0, 0, 0, 0, 0);     /* D3Q19 SRT */
        run(1, 5, 4, 3, o, 1, 0, 0, 1, 0);     /* D3Q19 MRT, rest start */
    }
    CHECK(orc_num_threads() >= 1);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
