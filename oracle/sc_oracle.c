/*
 * sc_oracle.c -- plain FP64 CPU stepper for the Shan-Chen pseudo-potential
 * lattice Boltzmann method (Peng, Ayala, Ayala & Wang, "Isotropy and spurious
 * currents in pseudo-potential multiphase lattice Boltzmann models").
 *
 * TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the CPU
 * baseline leg of bench.py may load this library.  It shares no code, header
 * or table with the GPU library; every constant below is written out here.
 *
 * One time step, for every node x of a periodic grid (lattice units,
 * dt = dx = 1), in the order the method defines it:
 *   1. rho   = sum_b f_b                                   (zeroth moment)
 *   2. psi   = psi(rho)                                    (Sec. 3, psi(rho))
 *   3. F     = -G c0 psi(x) sum_a w_a psi(x + e_a) e_a      (Sec. 2, Eq. (1))
 *   4. u     = (sum_b f_b c_b + F/2) / rho                  (Sec. 4, Eq. (7))
 *   5. feq_b = rho w_b [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)]
 *      phi_b = (1 - 1/(2 tau)) w_b [(c-u)/cs2 + (c.u) c/cs2^2] . F
 *                                                          (Sec. 2, Eq. (4))
 *   6. SRT:  f*_b = f_b - (f_b - feq_b)/tau + phi_b        (Sec. 2, Eq. (3))
 *      MRT:  m = M f;  m* = m - S (m - meq) + (I - S/2) M phihat;  f* = M^-1 m*
 *   7. f_b(x + c_b, t+1) = f*_b(x, t)                      (Sec. 2, Eq. (3))
 *
 * Solid walls (Sec. 3, droplet on a flat wall), when a solid mask is set:
 * solid nodes take part in the interaction force with the pseudo-potential
 * of a virtual wall density, psi(rho_w); instead of steps 4-6 a solid node
 * applies the standard (full-way) bounce-back, f*_b = f_{-b}: whatever
 * streamed into it is sent back along the link it came from, whatever its
 * length.  Solid nodes start like every node from feq(rho_init, 0) and hold
 * the populations in transit through the wall; streaming, bounce-back and
 * the fluid collision all conserve the total of the populations.
 *
 * No blocking, fusion or reordering beyond the above; the only parallelism
 * is an OpenMP split of independent node loops, which does not change any
 * result.  Build with -ffp-contract=off so no FMA changes the rounding.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Grids below this many nodes run their node loops on one thread: the
 * fork/join of a parallel region costs more than their work (no result
 * depends on the thread count). */
#define ORC_OMP_MIN_NODES 16384

#define ORC_D2Q9 0
#define ORC_D3Q19 1
#define ORC_D2Q13 2
#define ORC_D2Q25 3

typedef struct {
    int lattice;            /* ORC_D2Q9, ORC_D3Q19, ORC_D2Q13, ORC_D2Q25 */
    int nx, ny, nz;         /* nz = 1 for 2D */
    int order;              /* force-stencil isotropy order 4, 6, 8, 10 */
    double G, c0;           /* F = -G c0 psi sum_a what_a psi(x+e_a) e_a */
    int psi_kind;           /* 0: psi0 (1 - exp(-rho/rho_psi)); 1: psi = rho;
                               2: from the Peng-Robinson EOS (Sec. 3) */
    double psi0, rho_psi;
    double tau;
    int collision;          /* 0 SRT, 1 MRT (3D lattices) */
    double s_bulk, s_ghost; /* MRT rates of the c^2 moment and the ghosts */
    int forcing;            /* 0 Guo (Sec. 2, Eq. (4)); 1 exact difference method */
    double pr_a, pr_b, pr_R, pr_T, pr_alpha;  /* P-R EOS: a, b, R, T, alpha(T) */
    int init;               /* 0: f = feq(rho0, 0); 1: at rest in the forced
                               sense, f = feq(rho0, -F / (2 rho0)) */
} orc_params;

typedef struct {
    orc_params p;
    int dim, q;
    long n;
    int c[25][3];
    double w[25];
    double cs2;
    int ns;                 /* force stencil size */
    int e[96][3];
    double ew[96];
    double M[19][19];       /* MRT basis rows (3D only) */
    double Mnorm[19];       /* |row|^2 */
    double S[19];           /* relaxation rate per moment */
    double *f, *ftmp, *rho, *psi, *F;
    int opp[25];            /* index of -c_b */
    unsigned char *solid;   /* solid mask [N] or NULL */
    double psi_w;           /* psi(rho_w) of the solid nodes */
} orc_sim;

/* ------------------------------------------------------------------------ */
/* Velocity sets.  D2Q9/D2Q13/D2Q25: Sec. 3, Table 1 (weights by |c|^2).    */
/* D3Q19: the standard cube lattice Sec. 3 lists among 4th-order sets.      */
/* Vectors are enumerated by shell then lexicographically.                  */
/* ------------------------------------------------------------------------ */

static int add_shell(int dim, int n2, double w, int (*c)[3], double *wt, int k)
{
    int m = 3;
    for (int a = -m; a <= m; ++a)
        for (int b = -m; b <= m; ++b)
            for (int d = (dim == 3 ? -m : 0); d <= (dim == 3 ? m : 0); ++d)
                if (a * a + b * b + d * d == n2) {
                    c[k][0] = a; c[k][1] = b; c[k][2] = d;
                    wt[k] = w;
                    ++k;
                }
    return k;
}

int orc_lattice(int lattice, int *dim, int *q, int (*c)[3], double *w, double *cs2)
{
    int k = 0;
    switch (lattice) {
    case ORC_D2Q9:
        *dim = 2; *cs2 = 1.0 / 3.0;
        k = add_shell(2, 0, 4.0 / 9.0, c, w, k);
        k = add_shell(2, 1, 1.0 / 9.0, c, w, k);
        k = add_shell(2, 2, 1.0 / 36.0, c, w, k);
        break;
    case ORC_D2Q13:
        *dim = 2; *cs2 = 2.0 / 5.0;
        k = add_shell(2, 0, 2.0 / 5.0, c, w, k);
        k = add_shell(2, 1, 8.0 / 75.0, c, w, k);
        k = add_shell(2, 2, 1.0 / 25.0, c, w, k);
        k = add_shell(2, 4, 1.0 / 300.0, c, w, k);
        break;
    case ORC_D2Q25:
        *dim = 2; *cs2 = 4.0 / 7.0;
        k = add_shell(2, 0, 72.0 / 245.0, c, w, k);
        k = add_shell(2, 1, 16.0 / 147.0, c, w, k);
        k = add_shell(2, 2, 16.0 / 315.0, c, w, k);
        k = add_shell(2, 4, 1.0 / 105.0, c, w, k);
        k = add_shell(2, 5, 8.0 / 2205.0, c, w, k);
        k = add_shell(2, 8, 1.0 / 8820.0, c, w, k);
        break;
    case ORC_D3Q19:
        *dim = 3; *cs2 = 1.0 / 3.0;
        k = add_shell(3, 0, 1.0 / 3.0, c, w, k);
        k = add_shell(3, 1, 1.0 / 18.0, c, w, k);
        k = add_shell(3, 2, 1.0 / 36.0, c, w, k);
        break;
    default:
        return -1;
    }
    *q = k;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Force stencils (Sec. 2, Eq. (1)).  Normalised weights what(|e|^2) with   */
/* sum what e_x^2 = 1 and isotropic moment tensors up to the stated rank.   */
/* The weights are the exact solution of those isotropy conditions.         */
/* ------------------------------------------------------------------------ */

int orc_stencil(int dim, int order, int (*e)[3], double *w)
{
    int k = 0;
    if (dim == 2) {
        switch (order) {
        case 4:
            k = add_shell(2, 1, 1.0 / 3.0, e, w, k);
            k = add_shell(2, 2, 1.0 / 12.0, e, w, k);
            break;
        case 6:
            k = add_shell(2, 1, 4.0 / 15.0, e, w, k);
            k = add_shell(2, 2, 1.0 / 10.0, e, w, k);
            k = add_shell(2, 4, 1.0 / 120.0, e, w, k);
            break;
        case 8:
            k = add_shell(2, 1, 4.0 / 21.0, e, w, k);
            k = add_shell(2, 2, 4.0 / 45.0, e, w, k);
            k = add_shell(2, 4, 1.0 / 60.0, e, w, k);
            k = add_shell(2, 5, 2.0 / 315.0, e, w, k);
            k = add_shell(2, 8, 1.0 / 5040.0, e, w, k);
            break;
        case 10:
            k = add_shell(2, 1, 262.0 / 1785.0, e, w, k);
            k = add_shell(2, 2, 93.0 / 1190.0, e, w, k);
            k = add_shell(2, 4, 7.0 / 340.0, e, w, k);
            k = add_shell(2, 5, 6.0 / 595.0, e, w, k);
            k = add_shell(2, 8, 9.0 / 9520.0, e, w, k);
            k = add_shell(2, 9, 2.0 / 5355.0, e, w, k);
            k = add_shell(2, 10, 1.0 / 7140.0, e, w, k);
            break;
        default:
            return -1;
        }
    } else if (dim == 3) {
        switch (order) {
        case 4:
            k = add_shell(3, 1, 1.0 / 6.0, e, w, k);
            k = add_shell(3, 2, 1.0 / 12.0, e, w, k);
            break;
        case 6:
            k = add_shell(3, 1, 2.0 / 15.0, e, w, k);
            k = add_shell(3, 2, 1.0 / 15.0, e, w, k);
            k = add_shell(3, 3, 1.0 / 60.0, e, w, k);
            k = add_shell(3, 4, 1.0 / 120.0, e, w, k);
            break;
        case 8:
            k = add_shell(3, 1, 4.0 / 45.0, e, w, k);
            k = add_shell(3, 2, 1.0 / 21.0, e, w, k);
            k = add_shell(3, 3, 2.0 / 105.0, e, w, k);
            k = add_shell(3, 4, 5.0 / 504.0, e, w, k);
            k = add_shell(3, 5, 1.0 / 315.0, e, w, k);
            k = add_shell(3, 6, 1.0 / 630.0, e, w, k);
            k = add_shell(3, 8, 1.0 / 5040.0, e, w, k);
            break;
        default:
            return -1;
        }
    } else {
        return -1;
    }
    return k;
}

/* ------------------------------------------------------------------------ */
/* MRT moment basis for D3Q19.  Gram-Schmidt (unweighted inner product) of  */
/* monomials ordered by degree; groups: 0-3 conserved (rho, j), 4 the trace */
/* c^2 (bulk), 5-9 the traceless second moments (shear, rate 1/tau),        */
/* 10-18 the remaining non-hydrodynamic moments.                            */
/* ------------------------------------------------------------------------ */

static double mono(int k, const int *c)
{
    double x = c[0], y = c[1], z = c[2];
    double r2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return r2;
    case 5: return 2 * x * x - y * y - z * z;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return x * z;
    case 10: return r2 * r2;
    case 11: return r2 * x;
    case 12: return r2 * y;
    case 13: return r2 * z;
    case 14: return r2 * (2 * x * x - y * y - z * z);
    case 15: return r2 * (y * y - z * z);
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    case 18: return (x * x - y * y) * z;
    }
    return 0.0;
}

static void build_mrt(orc_sim *s)
{
    int q = s->q;
    for (int k = 0; k < q; ++k) {
        double v[19];
        for (int b = 0; b < q; ++b) v[b] = mono(k, s->c[b]);
        for (int j = 0; j < k; ++j) {
            double num = 0.0;
            for (int b = 0; b < q; ++b) num += v[b] * s->M[j][b];
            for (int b = 0; b < q; ++b) v[b] -= num / s->Mnorm[j] * s->M[j][b];
        }
        double nn = 0.0;
        for (int b = 0; b < q; ++b) nn += v[b] * v[b];
        for (int b = 0; b < q; ++b) s->M[k][b] = v[b];
        s->Mnorm[k] = nn;
    }
    for (int k = 0; k < q; ++k) {
        if (k < 4) s->S[k] = 0.0;
        else if (k == 4) s->S[k] = s->p.s_bulk;
        else if (k < 10) s->S[k] = 1.0 / s->p.tau;
        else s->S[k] = s->p.s_ghost;
    }
}

/* ------------------------------------------------------------------------ */

/* Peng-Robinson pressure (Sec. 3):
 *   p = rho R T / (1 - b rho) - a alpha rho^2 / (1 + 2 b rho - b^2 rho^2) */
static double p_pr(const orc_params *p, double rho)
{
    return rho * p->pr_R * p->pr_T / (1.0 - p->pr_b * rho)
           - p->pr_a * p->pr_alpha * rho * rho / (1.0 + 2.0 * p->pr_b * rho - p->pr_b * p->pr_b * rho * rho);
}

static double psi_of_cs(const orc_params *p, double rho, double cs2)
{
    if (p->psi_kind == 1) return rho;
    if (p->psi_kind == 2) {
        /* Sec. 3: psi = sqrt(2 (p - cs2 rho) / (G cs'^2)), cs'^2 = c0 here */
        double arg = 2.0 * (p_pr(p, rho) - cs2 * rho) / (p->G * p->c0);
        return arg > 0.0 ? sqrt(arg) : 0.0;
    }
    return p->psi0 * (1.0 - exp(-rho / p->rho_psi));
}

static long wrap(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

static long node_at(const orc_sim *s, long x, long y, long z)
{
    return wrap(x, s->p.nx) + s->p.nx * (wrap(y, s->p.ny) + s->p.ny * wrap(z, s->p.nz));
}

/* The force operator of Eq. (1) applied to an arbitrary psi field. */
static void force_from_psi(const orc_sim *s, const double *psi, double *F)
{
    const long n = s->n;
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    /* threads take whole rows (z, y); every node's sum is the same either way */
#pragma omp parallel for collapse(2) schedule(static) if (n >= ORC_OMP_MIN_NODES)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long i = x + nx * (y + ny * z);
                double acc[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < s->ns; ++a) {
                    double pn = psi[node_at(s, x + s->e[a][0], y + s->e[a][1], z + s->e[a][2])];
                    for (int d = 0; d < 3; ++d) acc[d] += s->ew[a] * pn * s->e[a][d];
                }
                for (int d = 0; d < s->dim; ++d)
                    F[d * n + i] = -s->p.G * s->p.c0 * psi[i] * acc[d];
            }
}

static void macro(orc_sim *s)
{
    const long n = s->n;
#pragma omp parallel for schedule(static) if (n >= ORC_OMP_MIN_NODES)
    for (long i = 0; i < n; ++i) {
        double r = 0.0;
        for (int b = 0; b < s->q; ++b) r += s->f[b * n + i];
        s->rho[i] = r;
        s->psi[i] = (s->solid && s->solid[i]) ? s->psi_w : psi_of_cs(&s->p, r, s->cs2);
    }
    force_from_psi(s, s->psi, s->F);
}

static void velocity(const orc_sim *s, long i, double *u)
{
    const long n = s->n;
    for (int d = 0; d < 3; ++d) u[d] = 0.0;
    for (int b = 0; b < s->q; ++b)
        for (int d = 0; d < s->dim; ++d) u[d] += s->f[b * n + i] * s->c[b][d];
    for (int d = 0; d < s->dim; ++d) u[d] = (u[d] + 0.5 * s->F[d * n + i]) / s->rho[i];
}

static void feq_of(const orc_sim *s, double rho, const double *u, double *feq)
{
    const double cs2 = s->cs2;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int b = 0; b < s->q; ++b) {
        double cu = s->c[b][0] * u[0] + s->c[b][1] * u[1] + s->c[b][2] * u[2];
        feq[b] = rho * s->w[b] * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

/* Exact difference method (the forcing used in the paper's experiments,
 * Sec. 3): relax towards feq(rho, v) with v = sum f c / rho, then add the
 * change of the equilibrium under the velocity increment F / rho:
 *   f* = f - (f - feq(rho, v)) / tau + feq(rho, v + F/rho) - feq(rho, v). */
static void collide_edm(const orc_sim *s, long i, double *fstar)
{
    const long n = s->n;
    double rho = s->rho[i];
    double v[3] = {0.0, 0.0, 0.0}, v2[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < s->q; ++b)
        for (int d = 0; d < s->dim; ++d) v[d] += s->f[b * n + i] * s->c[b][d];
    for (int d = 0; d < s->dim; ++d) {
        v[d] /= rho;
        v2[d] = v[d] + s->F[d * n + i] / rho;
    }
    double fe[25], fe2[25];
    feq_of(s, rho, v, fe);
    feq_of(s, rho, v2, fe2);
    for (int b = 0; b < s->q; ++b) {
        double f = s->f[b * n + i];
        fstar[b] = f - (f - fe[b]) / s->p.tau + (fe2[b] - fe[b]);
    }
}

static void collide_node(const orc_sim *s, long i, double *fstar)
{
    const long n = s->n;
    if (s->solid && s->solid[i]) {
        /* full-way bounce-back: reverse what arrived */
        for (int b = 0; b < s->q; ++b) fstar[b] = s->f[s->opp[b] * n + i];
        return;
    }
    const double cs2 = s->cs2, tau = s->p.tau;
    if (s->p.forcing == 1) {
        collide_edm(s, i, fstar);
        return;
    }
    double u[3], Fv[3] = {0.0, 0.0, 0.0};
    velocity(s, i, u);
    for (int d = 0; d < s->dim; ++d) Fv[d] = s->F[d * n + i];
    double rho = s->rho[i];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double feq[25], phihat[25];
    for (int b = 0; b < s->q; ++b) {
        double cu = s->c[b][0] * u[0] + s->c[b][1] * u[1] + s->c[b][2] * u[2];
        feq[b] = rho * s->w[b] * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
        double t = 0.0;
        for (int d = 0; d < 3; ++d)
            t += ((s->c[b][d] - u[d]) / cs2 + cu * s->c[b][d] / (cs2 * cs2)) * Fv[d];
        phihat[b] = s->w[b] * t;
    }
    if (s->p.collision == 0) {
        for (int b = 0; b < s->q; ++b) {
            double f = s->f[b * n + i];
            fstar[b] = f - (f - feq[b]) / tau + (1.0 - 1.0 / (2.0 * tau)) * phihat[b];
        }
    } else {
        double m[19], meq[19], mph[19], ms[19];
        for (int k = 0; k < s->q; ++k) {
            m[k] = meq[k] = mph[k] = 0.0;
            for (int b = 0; b < s->q; ++b) {
                m[k] += s->M[k][b] * s->f[b * n + i];
                meq[k] += s->M[k][b] * feq[b];
                mph[k] += s->M[k][b] * phihat[b];
            }
            ms[k] = m[k] - s->S[k] * (m[k] - meq[k]) + (1.0 - 0.5 * s->S[k]) * mph[k];
        }
        for (int b = 0; b < s->q; ++b) {
            double v = 0.0;
            for (int k = 0; k < s->q; ++k) v += s->M[k][b] * ms[k] / s->Mnorm[k];
            fstar[b] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                      */
/* ------------------------------------------------------------------------ */

orc_sim *orc_create(const orc_params *p, const double *rho0)
{
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->p = *p;
    if (orc_lattice(p->lattice, &s->dim, &s->q, s->c, s->w, &s->cs2) != 0) goto fail;
    if (s->dim == 2) s->p.nz = 1;
    s->ns = orc_stencil(s->dim, p->order, s->e, s->ew);
    if (s->ns <= 0) goto fail;
    if (p->collision == 1) {
        if (s->q != 19 || p->forcing != 0) goto fail;
        build_mrt(s);
    }
    for (int b = 0; b < s->q; ++b)
        for (int k = 0; k < s->q; ++k)
            if (s->c[k][0] == -s->c[b][0] && s->c[k][1] == -s->c[b][1] && s->c[k][2] == -s->c[b][2]) s->opp[b] = k;
    s->n = (long)s->p.nx * s->p.ny * s->p.nz;
    s->f = (double *)malloc(sizeof(double) * s->q * s->n);
    s->ftmp = (double *)malloc(sizeof(double) * s->q * s->n);
    s->rho = (double *)malloc(sizeof(double) * s->n);
    s->psi = (double *)malloc(sizeof(double) * s->n);
    s->F = (double *)malloc(sizeof(double) * 3 * s->n);
    if (!s->f || !s->ftmp || !s->rho || !s->psi || !s->F) goto fail;
    /* initial state: f = feq(rho0, u = 0) = w rho0 */
    for (int b = 0; b < s->q; ++b)
        for (long i = 0; i < s->n; ++i) s->f[b * s->n + i] = s->w[b] * rho0[i];
    macro(s);
    if (p->init == 1) {
        /* The forcing schemes report u = (sum f c + F/2) / rho; starting
         * from the equilibrium of v = -F / (2 rho) makes that zero.  rho is
         * unchanged (the equilibrium keeps the density), so F is too. */
        double v[3], fe[25];
        for (long i = 0; i < s->n; ++i) {
            for (int d = 0; d < 3; ++d) v[d] = d < s->dim ? -s->F[d * s->n + i] / (2.0 * rho0[i]) : 0.0;
            feq_of(s, rho0[i], v, fe);
            for (int b = 0; b < s->q; ++b) s->f[b * s->n + i] = fe[b];
        }
        macro(s);
    } else if (p->init != 0) {
        goto fail;
    }
    return s;
fail:
    if (s) {
        free(s->f); free(s->ftmp); free(s->rho); free(s->psi); free(s->F);
        free(s);
    }
    return NULL;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->f); free(s->ftmp); free(s->rho); free(s->psi); free(s->F); free(s->solid);
    free(s);
}

/* Solid mask [N] (nonzero = solid) and virtual wall density rho_w; NULL
 * removes the walls.  The populations are left as they are. */
int orc_set_walls(orc_sim *s, const unsigned char *solid, double rho_w)
{
    free(s->solid);
    s->solid = NULL;
    if (solid) {
        s->solid = (unsigned char *)malloc(s->n);
        if (!s->solid) return -1;
        for (long i = 0; i < s->n; ++i) s->solid[i] = solid[i] ? 1 : 0;
        s->psi_w = psi_of_cs(&s->p, rho_w, s->cs2);
    }
    macro(s);
    return 0;
}

void orc_step(orc_sim *s, long nsteps)
{
    const long n = s->n;
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    for (long t = 0; t < nsteps; ++t) {
        macro(s);
#pragma omp parallel for collapse(2) schedule(static) if (n >= ORC_OMP_MIN_NODES)
        for (long z = 0; z < nz; ++z)
            for (long y = 0; y < ny; ++y)
                for (long x = 0; x < nx; ++x) {
                    long i = x + nx * (y + ny * z);
                    double fstar[25];
                    collide_node(s, i, fstar);
                    for (int b = 0; b < s->q; ++b)
                        s->ftmp[b * n + node_at(s, x + s->c[b][0], y + s->c[b][1], z + s->c[b][2])] = fstar[b];
                }
        double *tmp = s->f; s->f = s->ftmp; s->ftmp = tmp;
    }
    macro(s);
}

/* Fields at the current time: rho[N], psi[N], F[dim][N], u[dim][N] (each nullable). */
void orc_fields(orc_sim *s, double *rho, double *psi, double *F, double *u)
{
    const long n = s->n;
    macro(s);
    if (rho) memcpy(rho, s->rho, sizeof(double) * n);
    if (psi) memcpy(psi, s->psi, sizeof(double) * n);
    if (F) for (int d = 0; d < s->dim; ++d) memcpy(F + d * n, s->F + d * n, sizeof(double) * n);
    if (u) {
        for (long i = 0; i < n; ++i) {
            double uv[3] = {0.0, 0.0, 0.0};
            if (!(s->solid && s->solid[i])) velocity(s, i, uv);
            for (int d = 0; d < s->dim; ++d) u[d * n + i] = uv[d];
        }
    }
    if (F && s->solid)
        for (long i = 0; i < n; ++i)
            if (s->solid[i])
                for (int d = 0; d < s->dim; ++d) F[d * n + i] = 0.0;
}

void orc_get_f(const orc_sim *s, double *f) { memcpy(f, s->f, sizeof(double) * s->q * s->n); }
void orc_set_f(orc_sim *s, const double *f) { memcpy(s->f, f, sizeof(double) * s->q * s->n); macro(s); }

/* Eq. (1) on a caller-supplied psi: F[dim][N]. */
int orc_force(const orc_params *p, const double *psi, double *F)
{
    orc_sim s;
    memset(&s, 0, sizeof(s));
    s.p = *p;
    if (orc_lattice(p->lattice, &s.dim, &s.q, s.c, s.w, &s.cs2) != 0) return -1;
    if (s.dim == 2) s.p.nz = 1;
    s.ns = orc_stencil(s.dim, p->order, s.e, s.ew);
    if (s.ns <= 0) return -1;
    s.n = (long)s.p.nx * s.p.ny * s.p.nz;
    force_from_psi(&s, psi, F);
    return 0;
}

/* MRT basis as built (rows [19][19], norms [19], rates [19]). */
int orc_mrt_basis(const orc_sim *s, double *M, double *norm, double *S)
{
    if (s->p.collision != 1) return -1;
    for (int k = 0; k < s->q; ++k) {
        for (int b = 0; b < s->q; ++b) M[k * s->q + b] = s->M[k][b];
        norm[k] = s->Mnorm[k];
        S[k] = s->S[k];
    }
    return 0;
}

/* Threads the node loops run on (for reporting CPU timings). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
