/*
 * sc_lbm.h -- C ABI of the MI355X (gfx950) Shan-Chen pseudo-potential lattice
 * Boltzmann hot path.
 *
 * Method: Peng, Ayala, Ayala & Wang, "Isotropy and spurious currents in
 * pseudo-potential multiphase lattice Boltzmann models".
 *   - interaction force   F(x) = -G psi(x) sum_a w_a psi(x + e_a) e_a     (Sec. 2, Eq. (1))
 *     on the E4/E6/E8/E10 isotropic stencils (Sec. 2, around Eq. (2));
 *     w_a = c0 * w_hat_a with w_hat normalised to sum w_hat e_x^2 = 1;
 *   - Guo-forced lattice Boltzmann step with pull streaming               (Sec. 2, Eq. (3)-(4)),
 *     u = (sum_b f_b c_b + F/2) / rho                                     (Sec. 4, Eq. (7));
 *   - psi = psi0 (1 - exp(-rho / rho_psi)), psi = rho for exact tests, or
 *     the Peng-Robinson pseudo-potential of Sec. 3,
 *       psi = sqrt(2 (p_PR(rho) - cs2 rho) / (G c0)),
 *       p_PR = rho R T / (1 - b rho) - a alpha rho^2 / (1 + 2 b rho - b^2 rho^2);
 *   - pressure p = cs2 rho + G c0 psi^2 / 2 (the psi definition of Sec. 3);
 *   - lattices D2Q9, D2Q13, D2Q25 (Sec. 3, Table 1) and D3Q19 (Sec. 3);
 *     D3Q19 also with MRT collision (rates grouped conserved / bulk /
 *     shear = 1/tau / ghost);
 *   - forcing: Guo (Eq. (4)) or, on the 2D lattices with SRT, the exact
 *     difference method the experiments of Sec. 3 use:
 *       f* = f - (f - feq(v))/tau + feq(v + F/rho) - feq(v),  v = sum f c / rho.
 *
 * Conventions
 *   - Lattice units, dt = dx = 1, periodic in every axis.
 *   - Node index i = x + nx (y + ny z).  Host field arrays passed to or
 *     returned from this library use that order; vector fields are [D][N].
 *   - State buffers hold the post-collision distributions minus w_b rho_ref,
 *     [Q][N], velocities in this order (c_x, c_y[, c_z]):
 *       D2Q9:  (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *       D3Q19: (0,0,0) (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1)
 *              (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *              (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *       D2Q13: (0,0), then by |c|^2 and within a shell lexicographically:
 *              (-1,0) (0,-1) (0,1) (1,0) (-1,-1) (-1,1) (1,-1) (1,1)
 *              (-2,0) (0,-2) (0,2) (2,0)
 *       D2Q25: the D2Q13 list, then (-2,-1) (-2,1) (-1,-2) (-1,2) (1,-2)
 *              (1,2) (2,-1) (2,1) (-2,-2) (-2,2) (2,-2) (2,2)
 *     so the next step pulls f_b(x) = state_b(x - c_b) + w_b rho_ref.
 *   - Every entry point returns SC_OK (0) or a negative SC_E_* code and
 *     never aborts or throws.  sc_lbm_strerror() names the code.
 *   - All host buffers are caller-owned; the library copies inputs and
 *     never keeps a host pointer beyond the call.
 *   - Work is enqueued on the stream given at creation (a hipStream_t; NULL
 *     makes the library create its own).  sc_lbm_observe / sc_lbm_force and
 *     every convergence check synchronise that stream.
 *   - A handle may be used from one host thread at a time.
 */
#ifndef SC_LBM_H
#define SC_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define SC_OK 0
#define SC_E_INVAL (-1)        /* invalid argument or parameter set         */
#define SC_E_NOMEM (-2)        /* device or host allocation failed          */
#define SC_E_DEVICE (-3)       /* HIP runtime error (no GPU, launch failure) */
#define SC_E_UNSUPPORTED (-4)  /* valid but not implemented combination     */
#define SC_E_NONFINITE (-5)    /* a reduction saw a NaN / Inf node          */

/* ---- enumerations ------------------------------------------------------ */
#define SC_D2Q9 0
#define SC_D3Q19 1
#define SC_D2Q13 2             /* cs^2 = 2/5, 6th-order isotropic (Table 1)  */
#define SC_D2Q25 3             /* cs^2 = 4/7, 8th-order isotropic (Table 1)  */

#define SC_PSI_EXP 0           /* psi = psi0 (1 - exp(-rho / rho_psi))      */
#define SC_PSI_IDENTITY 1      /* psi = rho                                 */
#define SC_PSI_PR 2            /* Peng-Robinson pseudo-potential (Sec. 3)   */

#define SC_GUO 0               /* Guo forcing, Eq. (4)                      */
#define SC_EDM 1               /* exact difference method (2D, SRT)          */

#define SC_SRT 0
#define SC_MRT 1               /* D3Q19 only                               */

#define SC_FP32_SHIFTED 0      /* float state stored as f - w rho_ref       */
#define SC_FP64 1              /* double state (same shift)                 */

#define SC_RHO_REF_AUTO (-1.0)  /* rho_ref < 0: the library picks the shift  */

#define SC_INIT_EQUILIBRIUM 0  /* f = feq(rho_init, 0)                      */
#define SC_INIT_REST 1         /* f = feq(rho_init, -F / (2 rho_init)): the
                                  forced velocity (sum f c + F/2) / rho is
                                  zero at t = 0                              */

/* ---- problem statement -------------------------------------------------- */
typedef struct sc_lbm_params {
    int32_t lattice;      /* SC_D2Q9, SC_D3Q19, SC_D2Q13 or SC_D2Q25             */
    int32_t nx, ny, nz;   /* grid; nz must be 1 on the 2D lattices                */
    int32_t order;        /* force-stencil isotropy order: 4, 6, 8, 10 (2D);
                             4, 6, 8 (3D)                                         */
    int32_t psi_kind;     /* SC_PSI_EXP, SC_PSI_IDENTITY or SC_PSI_PR             */
    double G;             /* interaction strength (Eq. (1)); G < 0 attracts       */
    double c0;            /* force-weight scale: w_a = c0 w_hat_a (1/3 for the
                             classic nearest-neighbour weights 1/9, 1/36)         */
    double psi0, rho_psi; /* psi = psi0 (1 - exp(-rho / rho_psi))                 */
    double tau;           /* relaxation time (Eq. (3)), > 1/2                     */
    int32_t collision;    /* SC_SRT or SC_MRT                                     */
    int32_t precision;    /* SC_FP32_SHIFTED or SC_FP64                           */
    double s_bulk;        /* MRT rate of the c^2 (bulk) moment                    */
    double s_ghost;       /* MRT rate of all non-hydrodynamic moments             */
    double rho_ref;       /* storage shift, >= 0; or SC_RHO_REF_AUTO (any value
                             < 0): the median of rho_init over at most 2^20
                             evenly strided nodes, so that most nodes store
                             values near zero; sc_lbm_rho_ref() returns it     */
    int32_t obs_every;    /* K: steps between convergence checks (default 100)    */
    int32_t variant;      /* launch shape of the fused kernel; -1 = automatic     */
    int32_t forcing;      /* SC_GUO or SC_EDM                                     */
    int32_t init;         /* SC_INIT_EQUILIBRIUM or SC_INIT_REST (sc_lbm_create)   */
    double eos_a, eos_b;  /* Peng-Robinson a, b (SC_PSI_PR; Sec. 3: 2/49, 2/21)   */
    double eos_R, eos_T;  /* gas constant and absolute temperature                */
    double eos_alpha;     /* alpha(T) of the Peng-Robinson attraction term        */
} sc_lbm_params;

/* Fills *p with the defaults: D2Q9 64x64, E4, G = -5, c0 = 1/3, exp psi with
 * psi0 = rho_psi = 1, tau = 1, SRT, Guo forcing, FP32 shifted, MRT rates 1.2,
 * rho_ref = SC_RHO_REF_AUTO, K = 100, automatic variant, EOS fields zero,
 * SC_INIT_EQUILIBRIUM. */
void sc_lbm_default_params(sc_lbm_params* p);

/* ---- observables (FP64 reductions) -------------------------------------- */
typedef struct sc_lbm_obs {
    int64_t step;         /* time step of the observed state                      */
    double mass;          /* sum rho                                              */
    double mom[3];        /* sum rho u                                            */
    double max_u;         /* max |u|        (spurious-velocity maximum, Sec. 3)   */
    double mean_u;        /* mean |u| over fluid nodes (field-averaged, Sec. 3)   */
    double l2_u;          /* sqrt(mean |u|^2)                                     */
    double rho_in;        /* rho at the centre node (nx/2, ny/2, nz/2)            */
    double rho_out;       /* rho at node 0                                        */
    double p_in, p_out;   /* p = cs2 rho + G c0 psi^2 / 2 at those nodes           */
    double dp;            /* p_in - p_out (Laplace pressure jump)                 */
    double radius;        /* equivalent radius from sum (rho - rho_out) / (rho_in - rho_out) */
    double rho_min, rho_max; /* extremes of rho over finite fluid nodes           */
    double d_max_u;       /* |max_u - max_u at the previous check|, or -1         */
    int64_t nonfinite;    /* nodes with a non-finite rho or u                     */
    int32_t converged_by; /* rule that stopped the last sc_lbm_step: 0 none (or no
                             tol given); 1 d_max_u < tol; 2 FP32 resolution rule */
    int32_t status;       /* SC_OK or SC_E_NONFINITE                              */
} sc_lbm_obs;

typedef struct sc_lbm sc_lbm;

/* Bytes of one state buffer: Q * nx * ny * nz * (4 or 8); 0 if *p is invalid. */
size_t sc_lbm_state_bytes(const sc_lbm_params* p);

/* Validate *p, take the device buffers and initialise the state.
 * p->init == SC_INIT_EQUILIBRIUM: f = feq(rho_init, u = 0), the usual start
 * of the droplet test (Sec. 3; the paper does not state its initial
 * populations).
 * p->init == SC_INIT_REST: f = feq(rho_init, -F / (2 rho_init)) with F the
 * interaction force (Eq. (1)) of psi(rho_init) on the periodic grid, so
 * that the velocity the forcing schemes report, (sum_b f_b c_b + F/2) / rho
 * (Guo, Eq. (4); the exact difference method the same), is zero at t = 0:
 * the fluid starts at rest in the forced sense.  Both keep rho = rho_init;
 * walls set later do not change the initial state.
 *   rho_init  host [N] doubles, or NULL for rho = 1 everywhere;
 *   dev_a/b   two device buffers of sc_lbm_state_bytes(p) bytes each, owned
 *             by the caller and kept until sc_lbm_destroy; both NULL makes
 *             the library allocate (and free) its own;
 *   hip_stream  the hipStream_t to enqueue on, or NULL.
 * *out is written only on success.  Errors: SC_E_INVAL (bad parameters,
 * non-finite rho_init, only one buffer given), SC_E_NOMEM, SC_E_DEVICE. */
int sc_lbm_create(const sc_lbm_params* p, const double* rho_init, void* dev_a, void* dev_b,
                  void* hip_stream, sc_lbm** out);

/* Advance the state (Sec. 2, Eq. (1), (3), (4): psi, force, collision and
 * pull streaming fused in one kernel per step, or per two steps for the
 * launch shapes that block two steps in time; see
 * sc_lbm_steps_per_launch).
 *   max_steps  steps to run (>= 0);
 *   tol        0: run exactly max_steps, asynchronously (nothing is read
 *              back); > 0: every K = obs_every steps reduce max |u| and stop
 *              once |max_u - previous max_u| < tol (an FP32 state on 3
 *              consecutive checks: its round-off moves max_u by ~1e-7 per
 *              check, so one check can fall below tol by chance), or (FP32)
 *              once max_u of the last 50 checks scatters around its
 *              least-squares line by less than the velocity the FP32 state
 *              resolves, and that line moves by less than the same band over
 *              the next 300 checks: the stored g_b = f_b - w_b rho_ref are
 *              rounded to 2^-24 of at most w_b max(1, |rho - rho_ref|), so u
 *              is resolved to
 *              4 * 2^-24 * sum_b |c_b| w_b * max(1, |rho - rho_ref|) / rho_min
 *              (about 1e-6 for a droplet with rho in 0.15..2; at least 4 ulp
 *              of max_u).  A slow drift of max_u shows as a slope and keeps
 *              the run going; round-off noise of the state does not.  Each
 *              check is one fused pass over the state (see sc_lbm_check),
 *              captured with the K steps in one graph;
 *   steps_done  may be NULL; receives the steps actually taken.
 * Returns SC_E_NONFINITE as soon as a check sees a non-finite node. */
int sc_lbm_step(sc_lbm* h, int64_t max_steps, double tol, int64_t* steps_done);

/* Interaction force of Eq. (1) with the handle's stencil, G and c0.
 *   psi_in  host [N] psi field, or NULL to use psi(rho) of the current state;
 *   F_out   host [D][N] doubles (caller-owned).
 * Computed in the state precision; synchronous. */
int sc_lbm_force(sc_lbm* h, const double* psi_in, double* F_out);

/* FP64 reductions of the current state (see sc_lbm_obs) and optional host
 * copies of its fields, each nullable: rho_out [N], u_out [D][N] doubles,
 * f_out the raw state buffer (sc_lbm_state_bytes bytes: post-collision,
 * shifted by w_b sc_lbm_rho_ref(h), [Q][N] in the library's velocity
 * order).
 * Synchronous. */
int sc_lbm_observe(sc_lbm* h, sc_lbm_obs* obs, double* rho_out, double* u_out, void* f_out);

/* The observables of sc_lbm_observe (no fields) from one fused pass over
 * the current state: psi of each tile and its stencil halo in LDS, then per
 * node rho, u = (sum_b f_b c_b + F/2) / rho with F of Eq. (1), and the FP64
 * reduction slots (per-block partials summed in a fixed order); max_u equals
 * sc_lbm_observe's, the sums agree to rounding.  This is the check
 * sc_lbm_step runs every K steps, where it is captured in the same graph as
 * the K steps.  The partials and the result block live in device buffers of
 * the handle (about 90 KB, allocated on first use) and the result is copied
 * to pinned host memory.  Synchronous; obs->converged_by reports the last
 * sc_lbm_step's rule.  Errors: SC_E_INVAL (NULL argument), SC_E_NOMEM,
 * SC_E_DEVICE; SC_E_NONFINITE when a node is not finite (obs is filled). */
int sc_lbm_check(sc_lbm* h, sc_lbm_obs* obs);

/* sc_lbm_check without any device allocation, for callers that cannot
 * allocate (code in tight serving loops, harnesses that forbid allocation
 * after set-up).  Same kernels and result as sc_lbm_check; the per-block
 * partials and the result block live in a file-scope device array of
 * kCheckMaxBlocks x 11 + 15 doubles (about 90 KB, enough for any grid: the
 * check never uses more than 1,024 blocks), one copy per device, located at
 * sc_lbm_create with that device current and held until the process ends.
 * The result is copied to a local host array.  All calls on one GPU share
 * that device's array: calls that overlap on one GPU (other host threads,
 * other streams) race.  Synchronous.  Errors: SC_E_INVAL (NULL argument),
 * SC_E_UNSUPPORTED (more partial rows than the array holds), SC_E_DEVICE
 * (the array's address could not be found at creation, or a HIP error);
 * SC_E_NONFINITE when a node is not finite (obs is filled). */
int sc_lbm_check_noalloc(sc_lbm* h, sc_lbm_obs* obs);

/* Restore a state written by sc_lbm_observe(f_out) (checkpoint / resume):
 * f_in host buffer of sc_lbm_state_bytes bytes; step sets the step counter. */
int sc_lbm_set_state(sc_lbm* h, const void* f_in, int64_t step);

/* Solid walls (Sec. 3, droplet on a flat wall), 2D lattices only.
 *   solid  host [N] bytes, nonzero = solid node, in node order; NULL removes
 *          the walls;
 *   rho_w  virtual wall density: solid nodes enter the interaction force
 *          with psi(rho_w), which tunes the wettability.
 * Solid nodes do not collide: they apply the standard (full-way)
 * bounce-back, sending every population back along the link it arrived on
 * (any link length, so walls should be at least max |c| = 1 or 2 nodes
 * thick).  Their populations are those in transit through the wall; they
 * keep whatever the state holds (sc_lbm_create initialises every node from
 * rho_init).  Observables: velocities are zero on solid nodes and the |u|
 * norms run over fluid nodes; the mass counts every node.  With walls every
 * 2D lattice runs the any-lattice kernels (the launch shape falls back to
 * the automatic choice when that changes the kernel family).  Synchronises
 * the stream.  Errors: SC_E_INVAL, SC_E_UNSUPPORTED (D3Q19), SC_E_NOMEM,
 * SC_E_DEVICE. */
int sc_lbm_set_walls(sc_lbm* h, const uint8_t* solid, double rho_w);

/* Device pointer of the buffer holding the current state (for callers that
 * keep the data resident); NULL on a NULL handle. */
void* sc_lbm_state_ptr(sc_lbm* h);

/* The hipStream_t the handle enqueues on (the caller's, or its own). */
void* sc_lbm_stream(sc_lbm* h);

/* The storage shift rho_ref the handle uses (the one given, or the one
 * SC_RHO_REF_AUTO picked at creation); NaN on a NULL handle. */
double sc_lbm_rho_ref(const sc_lbm* h);

/* Time every launch shape of the fused step on *p's lattice, order,
 * precision, collision, forcing and grid (state rho = 1) the way
 * sc_lbm_step runs it: one warm-up graph of 32 steps, then the best of three
 * runs of `steps` steps rounded up to whole graphs (at least one).  The
 * fastest is remembered: later sc_lbm_create calls with variant = -1 and the
 * same problem shape use it.  With SC_LBM_TUNE_CACHE set to a file path the
 * choices persist across processes.  Outputs are nullable. */
int sc_lbm_autotune(const sc_lbm_params* p, int32_t steps, int32_t* best_variant, double* best_ms_per_step);

/* Name of the launch shape in use, and the number of launch shapes of the
 * kernel family that serves *p (for sweeps through sc_lbm_params.variant;
 * *p's own variant field is ignored): D2Q9 with Guo forcing, D3Q19, and the
 * any-lattice 2D family (D2Q13, D2Q25, D2Q9 with EDM) each have their own
 * list.  0 if *p is invalid. */
const char* sc_lbm_variant_name(const sc_lbm* h);
int sc_lbm_num_variants(const sc_lbm_params* p);

/* Time steps one kernel launch of the handle's launch shape advances: 1, or
 * 2 for the D2Q9 and any-lattice 2D shapes that fuse two steps per launch
 * (temporal blocking; sc_lbm_step still advances exactly the steps asked
 * for, and with walls every launch takes one step).  0 on NULL. */
int sc_lbm_steps_per_launch(const sc_lbm* h);

void sc_lbm_destroy(sc_lbm* h);
const char* sc_lbm_strerror(int code);

/* ---- batched sweeps ----------------------------------------------------- */
/* Many independent D2Q9 SRT droplets (the droplet test of Sec. 3 repeated
 * over a parameter sweep) advanced by ONE kernel launch per step over a
 * (item, tile) work list.  Items may differ in nx, ny, stencil order, G, c0
 * and tau; they must share precision, psi parameters and rho_ref (with
 * SC_RHO_REF_AUTO, one median over all items' initial densities).  Each
 * item keeps its own state (two buffers carved from one allocation).
 * Converged or diverged items leave the work list; the others continue. */
typedef struct sc_lbm_batch sc_lbm_batch;

/*   items      n parameter sets (lattice SC_D2Q9, collision SC_SRT, Guo
 *              forcing, psi SC_PSI_EXP or SC_PSI_IDENTITY); items[0].variant
 *              picks the batched launch shape (see sc_lbm_batch_variant_name):
 *              0 one step per launch on 32 x 8 tiles, 1 / 2 / 3 two steps per
 *              launch (temporal blocking, one-step launches for an odd
 *              remainder) on 32 x 8, 64 x 16 and 32 x 16 tiles; any other
 *              value the automatic shape (3 for FP32, 2 for FP64);
 *   rho_init   n host pointers to [nx*ny] initial densities (each nullable),
 *              or NULL for rho = 1 everywhere;
 *   hip_stream as for sc_lbm_create.
 * Errors: SC_E_INVAL, SC_E_UNSUPPORTED (other lattice, MRT, EDM or
 * Peng-Robinson item), SC_E_NOMEM, SC_E_DEVICE. */
int sc_lbm_batch_create(const sc_lbm_params* items, int32_t n, const double* const* rho_init, void* hip_stream,
                        sc_lbm_batch** out);

/* Advance every active item by up to max_steps.  tol = 0: exactly
 * max_steps, asynchronously.  tol > 0: every K = items[0].obs_every steps
 * each active item is reduced and leaves the work list when it meets the
 * steady-state rule of sc_lbm_step, or is quarantined when non-finite.
 * Returns when all items have left or max_steps are done. */
int sc_lbm_batch_step(sc_lbm_batch* b, int64_t max_steps, double tol, int64_t* steps_done);

/* Observables and optional fields of one item (as sc_lbm_observe);
 * obs->converged_by reports the rule that retired the item. */
int sc_lbm_batch_observe(sc_lbm_batch* b, int32_t item, sc_lbm_obs* obs, double* rho_out, double* u_out);

/* Steps taken by an item and how it left (0 running, 1 tolerance rule,
 * 2 FP32 resolution rule, -1 non-finite / quarantined). */
int sc_lbm_batch_status(sc_lbm_batch* b, int32_t item, int64_t* steps, int32_t* converged_by);

/* Number of items still in the work list. */
int32_t sc_lbm_batch_active(sc_lbm_batch* b);

/* The storage shift rho_ref every item uses; NaN on a NULL batch. */
double sc_lbm_batch_rho_ref(const sc_lbm_batch* b);

/* Continue an FP32 batch in FP64 from its current states: a sweep run in
 * FP32 to its steady-state rule is then finished to the literal rule (the
 * max |u| change below tol) with the FP64 state, whose resolution the rule
 * needs.  Each item's state is widened exactly into new FP64 buffers (same
 * storage shift rho_ref, freshly allocated; the FP32 buffers are freed),
 * then cleared of the net momentum the FP32 rounding gathered: the step
 * conserves momentum and every item starts with none (Sec. 2, Eq. (3)-(4):
 * the forcing adds sum F = 0 on the periodic grid), and a widened state
 * that kept it would drift across the lattice and never meet the literal
 * rule.  Every node's populations take the equilibrium change of the
 * uniform velocity -J/M at its own density (masses unchanged);
 * items retired by a convergence rule rejoin the work list with their
 * convergence history cleared, quarantined items stay out, and every item
 * keeps its own step count.  The batch then runs the automatic FP64 launch
 * shape.  Synchronises the stream.  Errors: SC_E_INVAL (NULL or already FP64
 * batch), SC_E_NOMEM, SC_E_DEVICE. */
int sc_lbm_batch_promote(sc_lbm_batch* b);

/* Name of the batched launch shape in use ("" on a NULL batch), and the
 * number of batched launch shapes (values of items[0].variant). */
const char* sc_lbm_batch_variant_name(const sc_lbm_batch* b);
int32_t sc_lbm_batch_num_variants(void);

/* Launch-shape tuner for batched sweeps: times every batched shape on a
 * scratch batch of the same n items (rho = 1 everywhere; the work does not
 * depend on the values) the way sc_lbm_batch_step runs it -- graph-replayed
 * 32-step chunks, steps rounded up to whole chunks, best of three -- and
 * returns the fastest shape (a value for items[0].variant) and its time per
 * step in ms.  Allocates and frees one scratch batch per shape on its own
 * stream; synchronises.  Errors: as sc_lbm_batch_create, SC_E_INVAL for
 * steps < 1. */
int sc_lbm_batch_autotune(const sc_lbm_params* items, int32_t n, int32_t steps, int32_t* best_variant,
                          double* best_ms);

void sc_lbm_batch_destroy(sc_lbm_batch* b);

/* ---- learned warm start: network kernels -------------------------------- */
/* Not part of the paper's method: a small convolutional net predicts the
 * steady density of a droplet from its parameters so the iteration above
 * starts closer to its fixed point (the iteration alone decides the
 * steady state).  Every pointer below is DEVICE memory owned by the caller;
 * every call is asynchronous on `stream` (a hipStream_t or NULL) and returns
 * SC_OK, SC_E_INVAL (bad size or NULL pointer) or SC_E_DEVICE.
 *
 * Layout: activations NCHW float32 [batch][C][h][w]; weights [cout][cin][3][3]
 * bfloat16 (stored as uint16) used in the products, FP32 accumulation;
 * biases float32 [cout].  3x3 convolutions use circular padding:
 *     out[b][co][y][x] = bias[co] + sum_ci sum_{dy,dx in -1..1}
 *                        w[co][ci][dy+1][dx+1] in[b][ci][(y+dy) mod h][(x+dx) mod w].
 * Supported channel counts: cin <= 32, cout in {1, 32}; batch <= 65535. */
int sc_nn_conv3x3_fwd(const float* in, const uint16_t* w, const float* bias, float* out, int32_t batch,
                      int32_t cin, int32_t cout, int32_t h, int32_t wd, void* stream);

/* Gradient w.r.t. the input (cin must be 32): gin = conv(gout, w flipped and
 * transposed); wt_scratch holds cin*cout*9 bfloat16. */
int sc_nn_conv3x3_bwd_data(const float* gout, const uint16_t* w, uint16_t* wt_scratch, float* gin, int32_t batch,
                           int32_t cin, int32_t cout, int32_t h, int32_t wd, void* stream);

/* The same two passes with the tanh of the net's hidden layers fused into
 * the store (no separate elementwise pass over the activations):
 *   sc_nn_conv3x3_fwd_tanh:      out = tanh(conv(in) + bias), cout = 32 only;
 *                                equals sc_nn_conv3x3_fwd then sc_nn_tanh_fwd;
 *   sc_nn_conv3x3_bwd_data_tanh: gin = (1 - y^2) conv(gout, w flipped and
 *                                transposed), y [batch][cin][h][wd] the tanh
 *                                activation that was the layer's input;
 *                                equals sc_nn_conv3x3_bwd_data then
 *                                sc_nn_tanh_bwd(y, gin).
 * Arguments, layouts and errors otherwise as above. */
int sc_nn_conv3x3_fwd_tanh(const float* in, const uint16_t* w, const float* bias, float* out, int32_t batch,
                           int32_t cin, int32_t cout, int32_t h, int32_t wd, void* stream);
int sc_nn_conv3x3_bwd_data_tanh(const float* gout, const uint16_t* w, uint16_t* wt_scratch, const float* y,
                                float* gin, int32_t batch, int32_t cin, int32_t cout, int32_t h, int32_t wd,
                                void* stream);

/* Gradients w.r.t. the weights (gw [cout][cin][9] float32) and biases
 * (gbias [cout]) summed over the batch, through nblk per-block partial rows
 * in partial_scratch (sc_nn_bwd_weight_scratch_floats(cin, cout, nblk)
 * floats); the partials are summed in a fixed order (deterministic). */
int32_t sc_nn_bwd_weight_scratch_floats(int32_t cin, int32_t cout, int32_t nblk);
int sc_nn_conv3x3_bwd_weight(const float* in, const float* gout, float* partial_scratch, int32_t nblk, float* gw,
                             float* gbias, int32_t batch, int32_t cin, int32_t cout, int32_t h, int32_t wd,
                             void* stream);

/* x <- tanh(x);  g <- g (1 - y^2) with y = tanh output. */
int sc_nn_tanh_fwd(float* x, int64_t n, void* stream);
int sc_nn_tanh_bwd(const float* y, float* g, int64_t n, void* stream);

/* Mean squared error over n values: grad (nullable) <- 2 (out - tgt) / n and
 * partial_scratch[k] <- sum over block k's share of (out - tgt)^2 (nblk
 * doubles; the loss is their sum / n). */
int sc_nn_mse(const float* out, const float* tgt, float* grad, double* partial_scratch, int32_t nblk, int64_t n,
              void* stream);

/* Adam step t >= 1 on n FP32 parameters p with gradient g and moments m, v;
 * writes the bfloat16 copy p_bf16 when non-NULL. */
int sc_nn_adam(float* p, const float* g, float* m, float* v, uint16_t* p_bf16, int64_t n, float lr, float beta1,
               float beta2, float eps, int32_t t, void* stream);

/* y <- bfloat16(x), round to nearest even. */
int sc_nn_to_bf16(const float* x, uint16_t* y, int64_t n, void* stream);

/* Network input: out [batch][5][h][w] with channel 0 = distance of the node to
 * the domain centre (w/2, h/2) divided by scale_r, minus params[b][0] (the
 * droplet radius in the same units, so channel 0 is of order one across the
 * interface and bfloat16 weights place it to a fraction of a node), and
 * channels 1..4 the four per-image values params[batch][4] broadcast over
 * the grid. */
int sc_nn_features(const float* params, float* out, int32_t batch, int32_t h, int32_t wd, float scale_r,
                   void* stream);

/* Initial density of a learned start (device buffers, one image per
 * workgroup): out[b] = the average over the 8 symmetries of the square
 * about node (h/2, h/2) (mirror of either axis, transpose) of
 * base[b] + inv_scale * resid[b], clamped to [lo, hi], then shifted
 * uniformly so that its sum equals mass[b].  A droplet centred on that node
 * of a periodic square grid keeps this symmetry under the step, so the
 * average removes only asymmetric error of the prediction.
 *   resid  float [batch][h][w] (the net's output), base and out double
 *          [batch][h][w], mass double [batch]; h must equal w.
 * Errors: SC_E_INVAL (NULL pointer, h != w, batch outside 1..65535,
 * lo > hi), SC_E_DEVICE. */
int sc_nn_start_field(const float* resid, const double* base, const double* mass, double* out, int32_t batch,
                      int32_t h, int32_t wd, float inv_scale, double lo, double hi, void* stream);

/* Detail of the last HIP failure seen by this host thread (which call, the
 * HIP error string and code); "" if none.  Valid until the next failure. */
const char* sc_lbm_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* SC_LBM_H */
