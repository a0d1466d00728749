/*
 * lbdem_oracle.c -- plain, slow, FP64 CPU reference of one coupled LBM-DEM
 * time step of Rettinger & Ruede, "A Coupled Lattice Boltzmann Method and
 * Discrete Element Method for Discrete Particle Simulations of Particulate
 * Flows" (arXiv 1711.00336).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. The GPU library shares no
 * code, header, table or helper with it; both follow the same written
 * conventions (cell-centred lattice, D3Q19 velocity ordering, PDF deviations
 * from the rest weights) that are restated here from the paper.
 *
 * Everything is in lattice units (Sec. 3.2.2, last paragraph): dx = dt = 1,
 * c_s^2 = 1/3, rho_f = 1. Each function names the passage it follows.
 * Where the paper is silent or garbled a documented reading is applied; the
 * readings are listed at the function that applies them.
 *
 * Parity status of each part:
 *   - LBM collide/stream, equilibrium, forcing, moments: pinned (Poiseuille
 *     closed form, moment identities, conservation).
 *   - Roma kernel, interpolation, spreading, volume fraction: pinned (moment
 *     conditions of the kernel, partition of unity, closed-form porosity).
 *   - Drag, lubrication, contact forces: pinned (closed forms, limits,
 *     restitution, rolling, antisymmetry).
 *   - Lattice curl and lift: pinned (closed-form curl of sinusoidal and
 *     wall-bounded linear fields; Saffman's lift in a linear shear).
 *   - Lattice gradient in grad P and in the convective part of Du_f/Dt:
 *     pinned (closed forms on sinusoidal and product fields, the wall ghost
 *     rules on linear fields).
 *   - Tenneti drag away from eps_p = 0: pinned (its dilute, close-packed and
 *     inertial limits, hand-evaluated values, the quadratic large-slip form
 *     that fixes the Reynolds number).
 *   - Per-cell relaxation time (Eilers, Smagorinsky): pinned (Einstein's
 *     dilute limit; Smagorinsky's nu_t = (C_s dx)^2 |S| on Chapman-Enskog
 *     non-equilibrium states; Poiseuille flow with the Eilers viscosity).
 *   - Du_f/Dt time discretisation, a_p lag, subcycle averaging of the fluid
 *     force, near-wall kernel renormalisation: parity unpinned against the
 *     paper (the paper does not fix them); checked by invariants only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* ---------------------------------------------------------------------------
 * D3Q19 lattice (Sec. 3.2.2, Eq. LBM_Equation; velocity set of Qian et al.).
 * The paper does not print the weights; the standard D3Q19 weights are
 * 1/3 (rest), 1/18 (6 axis links), 1/36 (12 face diagonals).
 * Ordering: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 face diagonals in
 * opposite pairs. Opposite of q (q>0) is q+1 for odd q, q-1 for even q.
 * ------------------------------------------------------------------------- */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double WQ(int q)
{
    if (q == 0) return 1.0 / 3.0;
    if (q <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int OPP(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }

/* ---------------------------------------------------------------------------
 * Parameters and state
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t n[3];
    int32_t periodic[3];
    double tau;      /* BGK relaxation time of the pure fluid (tau_e = tau without Eilers and LES) */
    double rho_f;    /* fluid density used in the closures */
    double g[3];     /* gravitational acceleration, acting on the particles */
    double fb[3];    /* fluid body-force density f_b */
    double e_n, mu_c, T_c, h_c, h_min;
    int32_t lub_stab, use_lub, use_am;
    int32_t n_int, n_dem;
    double c_am;
    int32_t use_lift;  /* shear-induced lift (Table 1) on/off */
    int32_t use_eilers, use_les;  /* per-cell tau_e: Eilers viscosity, Smagorinsky LES */
    int32_t lub_contact;  /* 1: lubrication also while spheres overlap (gap clamped); 0: open gap only */
} orc_params;

typedef struct {
    double *df;      /* [19][Nc]  f_q - w_q, post-streaming */
    double *uprev;   /* [3][Nc]   fluid-phase velocity of the previous step */
    int64_t step;
    int64_t np;
    double *x, *u, *w, *a;  /* [np][3]: position, velocity, angular velocity, du_p/dt */
    double *d, *rho_p;      /* [np] */
} orc_state;

/* optional outputs; any pointer may be NULL */
typedef struct {
    double *f_acc;   /* [3][Nc] subcycle-averaged force density used by the LBM */
    double *eps_f;   /* [Nc] fluid fraction at the LBM collision */
    double *dudt;    /* [3][Nc] Du_f/Dt */
    double *gradp;   /* [3][Nc] grad P */
    double *rho;     /* [Nc] density of the post-stream state at step start */
    double *j;       /* [3][Nc] momentum sum_q c_q f_q at step start */
    double *F_am, *F_d, *F_pr, *F_const; /* [np][3], last subcycle */
    double impulse_pr[3];  /* (1/n_int) sum_k sum_p F_pr */
    double impulse_gb[3];  /* (1/n_int) sum_k sum_p (rho_p - rho_f) V_p g */
    double impulse_fb[3];  /* (1/n_int) sum_k sum_x eps_f f_b */
    double min_eps_f;
    int32_t status;        /* 0 ok, 3 unstable */
    double *F_l;           /* [np][3] lift, last subcycle (zero with lift off) */
    double *curl;          /* [3][Nc] curl of u_f at the last subcycle's start (lift on) */
} orc_aux;

static int64_t NC(const orc_params *p) { return (int64_t)p->n[0] * p->n[1] * p->n[2]; }
static int64_t CIDX(const orc_params *p, int i, int j, int k)
{
    return (int64_t)i + (int64_t)p->n[0] * ((int64_t)j + (int64_t)p->n[1] * k);
}
static int wrapi(int i, int n) { i %= n; return i < 0 ? i + n : i; }

static double mu0(const orc_params *p)
{
    /* Eq. visc_tau with tau_e = tau: mu/rho_f = (tau - 1/2) c_s^2 */
    return p->rho_f * (p->tau - 0.5) / 3.0;
}

/* ---------------------------------------------------------------------------
 * Interpolation / distribution kernel (Sec. 3.1.2, Eq. filter_def and
 * Eq. interpolation; Sec. 3.2.1, Eq. distribution_filter with D = I).
 * The missing parenthesis of the first branch is closed after the root.
 * Reading: r is applied per axis and the 3-D weight is the product
 * phi(r_x) phi(r_y) phi(r_z), Roma et al.'s definition; the support is the
 * 3x3x3 block of cells around the particle. (A radial reading would not
 * satisfy the volume conservation of Eq. fluid_volume_fraction.)
 * ------------------------------------------------------------------------- */
double orc_roma(double r)
{
    r = fabs(r);
    if (r < 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
    if (r < 1.5) return (5.0 - 3.0 * r - sqrt(1.0 - 3.0 * (1.0 - r) * (1.0 - r))) / 6.0;
    return 0.0;
}

/* Per-axis stencil of a particle at coordinate xp: cells floor(xp)-1 ..
 * floor(xp)+1. Periodic axes wrap. Walled axes (reading: the paper is silent
 * on kernels that cross a wall) drop cells outside [0, n) and renormalise the
 * remaining weights to sum 1, so volume and force are conserved.
 * Returns the number of cells written. */
int orc_axis_stencil(double xp, int n, int periodic, int32_t *idx, double *wt)
{
    int b = (int)floor(xp);
    int m = 0;
    double s = 0.0;
    for (int o = -1; o <= 1; ++o) {
        int i = b + o;
        double w = orc_roma((double)i + 0.5 - xp);
        if (periodic) {
            idx[m] = wrapi(i, n);
            wt[m] = w;
            ++m;
        } else if (i >= 0 && i < n) {
            idx[m] = i;
            wt[m] = w;
            s += w;
            ++m;
        }
    }
    if (!periodic) {
        for (int t = 0; t < m; ++t) wt[t] /= s;
    }
    return m;
}

typedef struct {
    int m;
    int64_t cell[27];
    double w[27];
} stencil27;

static void particle_stencil(const orc_params *p, const double *xp, stencil27 *st)
{
    int32_t ix[3][3];
    double wx[3][3];
    int mx[3];
    for (int a = 0; a < 3; ++a) mx[a] = orc_axis_stencil(xp[a], p->n[a], p->periodic[a], ix[a], wx[a]);
    st->m = 0;
    for (int c = 0; c < mx[2]; ++c)
        for (int b = 0; b < mx[1]; ++b)
            for (int a = 0; a < mx[0]; ++a) {
                st->cell[st->m] = CIDX(p, ix[0][a], ix[1][b], ix[2][c]);
                st->w[st->m] = wx[0][a] * wx[1][b] * wx[2][c];
                st->m++;
            }
}

/* phi_|p = sum_x I(x, x_p) phi(x)   (Eq. interpolation); field is [ncomp][Nc] */
static void interp(const orc_params *p, const stencil27 *st, const double *field, int ncomp, double *out)
{
    int64_t nc = NC(p);
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int t = 0; t < st->m; ++t) s += st->w[t] * field[c * nc + st->cell[t]];
        out[c] = s;
    }
}

/* field(x) += scale * D(x, x_p) * val  (Eq. distribution_filter); dx^3 = 1 */
static void spread(const orc_params *p, const stencil27 *st, double *field, int ncomp,
                   const double *val, double scale)
{
    int64_t nc = NC(p);
    for (int c = 0; c < ncomp; ++c)
        for (int t = 0; t < st->m; ++t) field[c * nc + st->cell[t]] += scale * st->w[t] * val[c];
}

double orc_interp_scalar(const orc_params *p, const double *field, const double *xp)
{
    stencil27 st;
    double v;
    particle_stencil(p, xp, &st);
    interp(p, &st, field, 1, &v);
    return v;
}

void orc_spread_scalar(const orc_params *p, double *field, const double *xp, double val)
{
    stencil27 st;
    particle_stencil(p, xp, &st);
    spread(p, &st, field, 1, &val, 1.0);
}

/* Eq. fluid_volume_fraction: eps_f(x) = 1 - sum_i D(x, x_p,i) V_p,i / dx^3 */
static double sphere_volume(double d) { return M_PI * d * d * d / 6.0; }

void orc_eps_field(const orc_params *p, int64_t np, const double *x, const double *d, double *eps_f)
{
    int64_t nc = NC(p);
    double *solid = calloc((size_t)nc, sizeof(double));
    for (int64_t i = 0; i < np; ++i) {
        stencil27 st;
        double v = sphere_volume(d[i]);
        particle_stencil(p, x + 3 * i, &st);
        spread(p, &st, solid, 1, &v, 1.0);
    }
    for (int64_t c = 0; c < nc; ++c) eps_f[c] = 1.0 - solid[c];
    free(solid);
}

/* ---------------------------------------------------------------------------
 * GNS lattice Boltzmann pieces (Sec. 3.2.2).
 * PDFs are carried as deviations df_q = f_q - w_q from the rest state
 * (rho = 1, u = 0). This is an exact change of variables: rho = 1 + sum df,
 * sum_q c_q f_q = sum_q c_q df_q because sum_q w_q c_q = 0, and the BGK
 * update is affine in f so it maps to the same update of df with
 * f^eq - w_q in place of f^eq. It keeps the small velocity moments free of
 * the O(1) rest weights.
 * ------------------------------------------------------------------------- */

/* moments of the PDFs (Eq. MacVel, first part): drho = rho - 1, j = sum c f */
void orc_moments(const double *dfq /* [19] */, double *drho, double j[3])
{
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int q = 0; q < Q; ++q) {
        r += dfq[q];
        jx += CV[q][0] * dfq[q];
        jy += CV[q][1] * dfq[q];
        jz += CV[q][2] * dfq[q];
    }
    *drho = r;
    j[0] = jx; j[1] = jy; j[2] = jz;
}

/* Eq. LBM_EQ minus the rest weight:
 * f_q^eq - w_q = w_q (rho - 1) + w_q rho ( c.u/c_s^2 + (c.u)^2/(2 eps c_s^4) - u.u/(2 eps c_s^2) ) */
void orc_feq_dev(double drho, const double u[3], double eps, double out[19])
{
    double rho = 1.0 + drho;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < Q; ++q) {
        double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
        out[q] = WQ(q) * drho + WQ(q) * rho * (3.0 * cu + 4.5 * cu * cu / eps - 1.5 * uu / eps);
    }
}

/* Eq. Forcing: F_q = w_q (1 - 1/(2 tau)) [ c/c_s^2 - u/(eps c_s^2) + (c.u) c/(eps c_s^4) ] . f */
void orc_guo(const double u[3], double eps, const double f[3], double tau, double out[19])
{
    double pre = 1.0 - 0.5 / tau;
    for (int q = 0; q < Q; ++q) {
        double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            double v = 3.0 * CV[q][a] - 3.0 * u[a] / eps + 9.0 * cu * CV[q][a] / eps;
            s += v * f[a];
        }
        out[q] = WQ(q) * pre * s;
    }
}

/* Per-cell relaxation time tau_e = tau_* + tau_t (Eq. tau_e; Alg. 1, the
 * two steps before the GNS-LBM step), from the cell's solid fraction eps_p,
 * density rho and PDF deviations df with their equilibrium feq:
 *  - Eilers (Eq. visc_eilers, reading of the garbled denominator as
 *    1 - eps_p/eps_cp, Eilers' form): mu_* = mu_0 (1 + 0.5 [mu] eps_p /
 *    (1 - eps_p/eps_cp))^2, [mu] = 2.5, eps_cp = 0.64, and with Eq.
 *    visc_tau_* tau_* = 1/2 + (tau - 1/2) mu_* / mu_0;
 *  - Smagorinsky (Eqs. visc_turb, tau_t): nu_t = tau_t c_s^2 = (C_s dx)^2 S,
 *    S = Qbar/(2 rho c_s^2 tau_e), Qbar = sqrt(2 sum Q_ab Q_ab),
 *    Q_ab = sum_q c_qa c_qb (f_q - f_q^eq), C_s = 0.1, dx = 1. With
 *    tau_e = tau_* + tau_t this is tau_t^2 + tau_* tau_t = C_s^2 Qbar/(2 rho c_s^4),
 *    solved for its positive root. (The printed closed form carries 2 sqrt 2
 *    where this root carries 2; the two agree when its Qbar is read as
 *    sqrt(sum Q_ab Q_ab), without the factor 2 under the root: the reading
 *    keeps the defining relation.) rho is the cell's density. */
double orc_tau_e(const orc_params *p, double eps_p, double rho, const double df[19], const double feq[19])
{
    double ts = p->tau;
    if (p->use_eilers) {
        const double b = 1.0 + 0.5 * 2.5 * eps_p / (1.0 - eps_p / 0.64);
        ts = 0.5 + (p->tau - 0.5) * b * b;
    }
    if (!p->use_les) return ts;
    double Qm[3][3] = {{0}};
    for (int q = 0; q < Q; ++q) {
        const double neq = df[q] - feq[q];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Qm[a][b] += CV[q][a] * CV[q][b] * neq;
    }
    double qq = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) qq += Qm[a][b] * Qm[a][b];
    const double Qbar = sqrt(2.0 * qq);
    const double cs = 0.1, cs4 = 1.0 / 9.0;
    const double rhs = cs * cs * Qbar / (2.0 * rho * cs4);
    const double tt = 0.5 * (sqrt(ts * ts + 4.0 * rhs) - ts);
    return ts + tt;
}

/* One GNS-LBM update (Eq. LBM_Equation): collide every cell with its own
 * eps_f and force density f_acc, then stream to x + c_q. The velocity in the
 * equilibrium and the forcing is Eq. MacVel, u = (j + f/2)/rho.
 * Boundaries: periodic axes wrap; on walled axes a link that would leave the
 * domain through the wall plane is reflected in place into the opposite
 * direction of the same cell (half-way bounce-back, no-slip at the plane
 * midway between the last cell centre and its ghost). */
void orc_lbm_collide_stream(const orc_params *p, const double *df_in, double *df_out,
                            const double *eps_f, const double *f_acc)
{
    int64_t nc = NC(p);
    const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int jj = 0; jj < ny; ++jj)
            for (int i = 0; i < nx; ++i) {
                int64_t c = CIDX(p, i, jj, k);
                double f[Q], feq[Q], F[Q], j[3], u[3], drho, fx[3];
                for (int q = 0; q < Q; ++q) f[q] = df_in[q * nc + c];
                orc_moments(f, &drho, j);
                double rho = 1.0 + drho;
                for (int a = 0; a < 3; ++a) {
                    fx[a] = f_acc ? f_acc[a * nc + c] : 0.0;
                    u[a] = (j[a] + 0.5 * fx[a]) / rho;
                }
                double eps = eps_f ? eps_f[c] : 1.0;
                orc_feq_dev(drho, u, eps, feq);
                const double tau = orc_tau_e(p, 1.0 - eps, rho, f, feq);
                orc_guo(u, eps, fx, tau, F);
                int pos[3] = {i, jj, k};
                for (int q = 0; q < Q; ++q) {
                    double post = f[q] + (feq[q] - f[q]) / tau + F[q];
                    int t[3], wall = 0;
                    for (int a = 0; a < 3; ++a) {
                        t[a] = pos[a] + CV[q][a];
                        if (t[a] < 0 || t[a] >= p->n[a]) {
                            if (p->periodic[a]) t[a] = wrapi(t[a], p->n[a]);
                            else wall = 1;
                        }
                    }
                    if (wall) df_out[OPP(q) * nc + c] = post;
                    else df_out[q * nc + CIDX(p, t[0], t[1], t[2])] = post;
                }
            }
}

/* ---------------------------------------------------------------------------
 * Lattice differential operators (Sec. 3.2.3, gradient of a scalar):
 *   grad phi(x) ~ (1/c_s^2) sum_q w_q c_q phi(x + c_q)
 * Reading for neighbours beyond a wall (the paper is silent): the ghost
 * value is the value of the cell mirrored back into the domain; a scalar
 * keeps its value (zero normal gradient), a velocity component flips sign
 * once per mirrored axis (no-slip at the half-way wall plane).
 * ------------------------------------------------------------------------- */
static int64_t ghost_cell(const orc_params *p, int i, int j, int k, int q, double *sign)
{
    int t[3] = {i + CV[q][0], j + CV[q][1], k + CV[q][2]};
    *sign = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (t[a] < 0 || t[a] >= p->n[a]) {
            if (p->periodic[a]) t[a] = wrapi(t[a], p->n[a]);
            else {
                t[a] = t[a] < 0 ? 0 : p->n[a] - 1;
                *sign = -*sign;
            }
        }
    }
    return CIDX(p, t[0], t[1], t[2]);
}

static void cross(const double a[3], const double b[3], double c[3]);
static double dot(const double a[3], const double b[3]);

/* Lattice curl (Sec. 3.2.3, rotation of a vector field):
 *   curl psi(x) ~ (1/c_s^2) sum_q w_q c_q x psi(x + c_q)
 * applied to a velocity field with the ghost rule above. u, out: [3][Nc]. */
void orc_curl_field(const orc_params *p, const double *u, double *out)
{
    const int64_t nc = NC(p);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->n[2]; ++k)
        for (int jj = 0; jj < p->n[1]; ++jj)
            for (int i = 0; i < p->n[0]; ++i) {
                const int64_t c = CIDX(p, i, jj, k);
                double s[3] = {0.0, 0.0, 0.0};
                for (int q = 0; q < Q; ++q) {
                    double sg, cq[3], v[3], cv[3];
                    int64_t nb = ghost_cell(p, i, jj, k, q, &sg);
                    for (int a = 0; a < 3; ++a) {
                        cq[a] = CV[q][a];
                        v[a] = sg * u[a * nc + nb];
                    }
                    cross(cq, v, cv);
                    for (int a = 0; a < 3; ++a) s[a] += WQ(q) * cv[a];
                }
                for (int a = 0; a < 3; ++a) out[a * nc + c] = 3.0 * s[a];
            }
}

/* ---------------------------------------------------------------------------
 * Drag (Sec. 3.1.2, Table 1; Tenneti et al. correlation as printed):
 *   F_d = 3 pi d mu0 (1 - eps_p) C_d(Re, eps_p) (u_f|p - u_p)
 *   C_d = (1 - eps_p) ( C_d0/(1 - eps_p)^3 + A + B ),  C_d0 = 1 + 0.15 Re^0.687
 *   A = 5.81 eps_p/(1 - eps_p)^3 + 0.48 eps_p^(1/3)/(1 - eps_p)^4
 *   B = eps_p^3 Re (0.95 + 0.61 eps_p^3/(1 - eps_p)^2)
 *   Re = (1 - eps_p) rho_f d |u_p - u_f|p| / mu0
 * Taken literally, including both (1 - eps_p) factors.
 * orc_drag_factor returns (1 - eps_p) C_d, so F_d = 3 pi d mu0 * factor * w.
 * ------------------------------------------------------------------------- */
double orc_drag_factor(double Re, double ep)
{
    double e1 = 1.0 - ep;
    double cd0 = 1.0 + 0.15 * (Re > 0.0 ? pow(Re, 0.687) : 0.0);
    double A = 5.81 * ep / (e1 * e1 * e1) + 0.48 * (ep > 0.0 ? cbrt(ep) : 0.0) / (e1 * e1 * e1 * e1);
    double B = ep * ep * ep * Re * (0.95 + 0.61 * ep * ep * ep / (e1 * e1));
    double cd = e1 * (cd0 / (e1 * e1 * e1) + A + B);
    return e1 * cd;
}

void orc_drag(double d, double mu, double rho_f, double ep, const double w[3], double F[3])
{
    double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double Re = (1.0 - ep) * rho_f * d * wn / mu;
    double fac = 3.0 * M_PI * d * mu * orc_drag_factor(Re, ep);
    for (int a = 0; a < 3; ++a) F[a] = fac * w[a];
}

/* Shear-induced lift (Table 1, after Saffman):
 *   F_l = 1.61 d^2 sqrt(mu0 rho_f / |omega|) (w x omega)
 * with w = u_f|p - u_p and omega = (curl u_f)|p. Reading: F_l = 0 where
 * omega = 0, the limit of the formula (its magnitude scales with sqrt|omega|). */
void orc_lift(double d, double mu, double rho_f, const double w[3], const double om[3], double F[3])
{
    const double on = sqrt(dot(om, om));
    if (on == 0.0) {
        F[0] = F[1] = F[2] = 0.0;
        return;
    }
    double c[3];
    cross(w, om, c);
    const double s = 1.61 * d * d * sqrt(mu * rho_f / on);
    for (int a = 0; a < 3; ++a) F[a] = s * c[a];
}

/* ---------------------------------------------------------------------------
 * DEM (Sec. 3.1.1) and lubrication (Sec. 3.1.3).
 * ------------------------------------------------------------------------- */

/* Eq. damping_to_stiffness and Eq. collision_time solved for k_n and xi_n
 * given T_c, e_n and the pair's reduced mass m_ij:
 *   k_n = m_ij (pi^2 + ln^2 e_n) / T_c^2,   xi_n = -2 ln(e_n) m_ij / T_c. */
void orc_collision_params(double mij, double e_n, double T_c, double *kn, double *xi)
{
    double L = log(e_n);
    *kn = mij * (M_PI * M_PI + L * L) / (T_c * T_c);
    *xi = -2.0 * L * mij / T_c;
}

/* Lubrication coefficients (Sec. 3.1.3, Ball & Melrose), for a gap h that is
 * already clamped and a mean diameter dm. */
void orc_lub_coeffs(double h, double dm, double mu, double *asq, double *ash)
{
    double L = log(dm / (2.0 * h));
    *asq = 1.5 * M_PI * mu * dm * (dm / (4.0 * h) + (18.0 / 40.0) * L + (9.0 / 84.0) * (h / dm) * L);
    *ash = 0.5 * M_PI * mu * dm * L * (dm + h) * (dm + h) / 4.0;
}

typedef struct {
    double r, m, I;  /* radius, mass, moment of inertia */
    const double *x, *u, *w;
    double d;
} pinfo;

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Contact of particle i with a partner: n points from i to the partner,
 * dist is the centre distance (pair) or the centre-to-plane distance (wall,
 * then r_j = 0 in the overlap and the partner velocity/spin terms vanish).
 *   delta = (d_i + d_j)/2 - |x_j - x_i|,
 *   u_r = u_i - u_j + (d_i/2 w_i + d_j/2 w_j) x n,
 *   F^n = -k_n delta n - xi_n u_r^n,
 *   F^t = -min(mu_c |F^n|, xi_t |u_r^t|) t,  t = u_r^t/|u_r^t|, only if |u_r^t| > 0,
 *   xi_t = xi_n.
 * Torque reading: the printed torque (d_i/2) F^t x n has the opposite sign of
 * the moment of F^t applied at the contact point x_i + (d_i/2) n, which is
 * (d_i/2) n x F^t; with the printed sign friction would spin the sphere up
 * against its slip. The moment n x F^t is used. */
static void contact(const orc_params *p, double delta, const double n[3], const double ur[3], double mij,
                    double ri, double F[3], double T[3])
{
    double kn, xi;
    orc_collision_params(mij, p->e_n, p->T_c, &kn, &xi);
    double urn_s = dot(ur, n);
    double urn[3], urt[3], Fn[3];
    for (int a = 0; a < 3; ++a) {
        urn[a] = urn_s * n[a];
        urt[a] = ur[a] - urn[a];
        Fn[a] = -kn * delta * n[a] - xi * urn[a];
    }
    double urt_n = sqrt(dot(urt, urt));
    double Ft[3] = {0.0, 0.0, 0.0};
    if (urt_n > 0.0) {
        double fn_n = sqrt(dot(Fn, Fn));
        double mag = fmin(p->mu_c * fn_n, xi * urt_n);
        for (int a = 0; a < 3; ++a) Ft[a] = -mag * urt[a] / urt_n;
    }
    double tq[3];
    cross(n, Ft, tq);
    for (int a = 0; a < 3; ++a) {
        F[a] += Fn[a] + Ft[a];
        T[a] += ri * tq[a];
    }
}

/* Eq. lubrication_force for sphere i; only if h < h_c; h := max(h, h_min).
 * Reading (explicit stability): the gap is also floored at
 * h_stab = 3 pi mu dm^2 dt_DEM / (8 r m_ij) with r = 1/4, where the leading
 * term of a_sq makes a_sq dt_DEM / m_ij = r. A sphere with k partners at
 * the floor relaxes up to (k + 1)/2 times faster than one pair, and with
 * the lagged added mass the explicit update stays stable only below
 * 2 - 2 C_am rho_f / rho_p; r = 1/4 covers a full shell of twelve partners.
 * (With r = 1 three near-touching partners already diverge: the dilute
 * 128^3 packing does so in a few steps.) It only acts when lub_stab is set.
 * Reading for overlapping spheres (h <= 0): the text clamps the gap at
 * h_min and applies the force (lub_contact = 1, the default); the collision
 * results of Sec. 5 (a rebound near e_n at large Stokes numbers, Table 3)
 * need the force on the open gap only (lub_contact = 0), as the clamped
 * force overdamps the contact spring at those Stokes numbers. */
static void lubrication(const orc_params *p, double h, double dm, double mij, const double n[3],
                        const double upr[3], double dt_dem, double F[3])
{
    if (!(h < p->h_c)) return;
    if (!p->lub_contact && !(h > 0.0)) return;
    double mu = mu0(p);
    double he = fmax(h, p->h_min);
    if (p->lub_stab) he = fmax(he, 3.0 * M_PI * mu * dm * dm * dt_dem / (8.0 * 0.25 * mij));
    double asq, ash;
    orc_lub_coeffs(he, dm, mu, &asq, &ash);
    double un = dot(upr, n);
    double s = 2.0 / (he + dm);
    for (int a = 0; a < 3; ++a) F[a] += -asq * un * n[a] - ash * s * s * (upr[a] - un * n[a]);
}

/* force/torque on particle i from particle j; dx = x_j - x_i (minimum image) */
static void pair_interaction(const orc_params *p, const pinfo *pi, const pinfo *pj, const double dx[3],
                             double dt_dem, double F[3], double T[3])
{
    double dist2 = dot(dx, dx);
    double reach = pi->r + pj->r + (p->use_lub ? fmax(p->h_c, 0.0) : 0.0);
    if (dist2 >= reach * reach) return;
    double dist = sqrt(dist2);
    double n[3] = {dx[0] / dist, dx[1] / dist, dx[2] / dist};
    double delta = pi->r + pj->r - dist;
    double mij = pi->m * pj->m / (pi->m + pj->m);
    if (delta > 0.0) {
        double s[3], ur[3];
        for (int a = 0; a < 3; ++a) s[a] = pi->r * pi->w[a] + pj->r * pj->w[a];
        cross(s, n, ur);
        for (int a = 0; a < 3; ++a) ur[a] += pi->u[a] - pj->u[a];
        contact(p, delta, n, ur, mij, pi->r, F, T);
    }
    if (p->use_lub) {
        double dm = 2.0 * pi->d * pj->d / (pi->d + pj->d);
        double upr[3] = {pi->u[0] - pj->u[0], pi->u[1] - pj->u[1], pi->u[2] - pj->u[2]};
        lubrication(p, -delta, dm, mij, n, upr, dt_dem, F);
    }
}

/* sphere-wall: the wall is a plane at coordinate 0 or n[a] of a walled axis;
 * m_ij = m_i; for lubrication <d> = 2 d_i (d_j -> infinity), u_pr = u_i. */
static void wall_interaction(const orc_params *p, const pinfo *pi, double dt_dem, double F[3], double T[3])
{
    for (int a = 0; a < 3; ++a) {
        if (p->periodic[a]) continue;
        for (int side = 0; side < 2; ++side) {
            double dist = side == 0 ? pi->x[a] : (double)p->n[a] - pi->x[a];
            double n[3] = {0.0, 0.0, 0.0};
            n[a] = side == 0 ? -1.0 : 1.0;
            double delta = pi->r - dist;
            if (delta > 0.0) {
                double s[3], ur[3];
                for (int b = 0; b < 3; ++b) s[b] = pi->r * pi->w[b];
                cross(s, n, ur);
                for (int b = 0; b < 3; ++b) ur[b] += pi->u[b];
                contact(p, delta, n, ur, pi->m, pi->r, F, T);
            }
            if (p->use_lub) lubrication(p, -delta, 2.0 * pi->d, pi->m, n, pi->u, dt_dem, F);
        }
    }
}

/* exported for the closed-form tests: force and torque on i from j */
void orc_pair_force(const orc_params *p, const double *xi, const double *ui, const double *wi, double di,
                    double rhoi, const double *xj, const double *uj, const double *wj, double dj, double rhoj,
                    double dt_dem, double F[3], double T[3])
{
    pinfo a = {0.5 * di, rhoi * sphere_volume(di), 0.0, xi, ui, wi, di};
    pinfo b = {0.5 * dj, rhoj * sphere_volume(dj), 0.0, xj, uj, wj, dj};
    double dx[3];
    for (int k = 0; k < 3; ++k) {
        dx[k] = xj[k] - xi[k];
        if (p->periodic[k]) dx[k] -= p->n[k] * nearbyint(dx[k] / p->n[k]);
        F[k] = 0.0;
        T[k] = 0.0;
    }
    pair_interaction(p, &a, &b, dx, dt_dem, F, T);
}

void orc_wall_force(const orc_params *p, const double *xi, const double *ui, const double *wi, double di,
                    double rhoi, double dt_dem, double F[3], double T[3])
{
    pinfo a = {0.5 * di, rhoi * sphere_volume(di), 0.0, xi, ui, wi, di};
    for (int k = 0; k < 3; ++k) F[k] = T[k] = 0.0;
    wall_interaction(p, &a, dt_dem, F, T);
}

/* ---------------------------------------------------------------------------
 * Collision/lubrication forces on all particles (Eq. forces_collision,
 * Eq. torques_collision, Eq. lubrication_force): a plain sum over all
 * partners j != i in index order. For many particles the candidate partners
 * come from a uniform cell list (cells at least as wide as the interaction
 * reach), sorted by index so that the sum runs in the same order as the
 * all-pairs loop.
 * ------------------------------------------------------------------------- */
typedef struct {
    int use;
    int nb[3];
    double cs[3];
    int64_t *head, *next;
} celllist;

static int64_t cl_threshold = 4096;

/* particle count above which partners come from the cell list (tests lower it) */
void orc_set_celllist_threshold(int64_t n) { cl_threshold = n; }

static void cl_build(const orc_params *p, int64_t np, const double *x, double reach, celllist *cl)
{
    cl->use = np > cl_threshold;
    if (!cl->use) return;
    int64_t tot = 1;
    for (int a = 0; a < 3; ++a) {
        cl->nb[a] = (int)floor(p->n[a] / reach);
        if (cl->nb[a] < 1) cl->nb[a] = 1;
        cl->cs[a] = (double)p->n[a] / cl->nb[a];
        tot *= cl->nb[a];
    }
    cl->head = malloc(sizeof(int64_t) * (size_t)tot);
    cl->next = malloc(sizeof(int64_t) * (size_t)np);
    for (int64_t c = 0; c < tot; ++c) cl->head[c] = -1;
    for (int64_t i = np - 1; i >= 0; --i) {
        int b[3];
        for (int a = 0; a < 3; ++a) {
            b[a] = (int)floor(x[3 * i + a] / cl->cs[a]);
            if (b[a] < 0) b[a] = 0;
            if (b[a] >= cl->nb[a]) b[a] = cl->nb[a] - 1;
        }
        int64_t c = b[0] + (int64_t)cl->nb[0] * (b[1] + (int64_t)cl->nb[1] * b[2]);
        cl->next[i] = cl->head[c];
        cl->head[c] = i;
    }
}

static void cl_free(celllist *cl)
{
    if (cl->use) {
        free(cl->head);
        free(cl->next);
    }
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : x > y;
}

/* partners of particle i in ascending index order (all j != i, or cell-list candidates) */
static int64_t partners(const orc_params *p, const celllist *cl, int64_t np, const double *x, int64_t i,
                        int64_t **buf, int64_t *cap)
{
    int64_t m = 0;
    if (!cl->use) {
        if (*cap < np) {
            *cap = np;
            *buf = realloc(*buf, sizeof(int64_t) * (size_t)np);
        }
        for (int64_t j = 0; j < np; ++j)
            if (j != i) (*buf)[m++] = j;
        return m;
    }
    int b[3];
    for (int a = 0; a < 3; ++a) {
        b[a] = (int)floor(x[3 * i + a] / cl->cs[a]);
        if (b[a] < 0) b[a] = 0;
        if (b[a] >= cl->nb[a]) b[a] = cl->nb[a] - 1;
    }
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dxx = -1; dxx <= 1; ++dxx) {
                int t[3] = {b[0] + dxx, b[1] + dy, b[2] + dz}, ok = 1;
                for (int a = 0; a < 3; ++a) {
                    if (t[a] < 0 || t[a] >= cl->nb[a]) {
                        if (p->periodic[a]) t[a] = wrapi(t[a], cl->nb[a]);
                        else ok = 0;
                    }
                }
                if (!ok) continue;
                int64_t c = t[0] + (int64_t)cl->nb[0] * (t[1] + (int64_t)cl->nb[1] * t[2]);
                for (int64_t j = cl->head[c]; j >= 0; j = cl->next[j]) {
                    if (j == i) continue;
                    if (m >= *cap) {
                        *cap = *cap * 2 + 64;
                        *buf = realloc(*buf, sizeof(int64_t) * (size_t)*cap);
                    }
                    (*buf)[m++] = j;
                }
            }
    qsort(*buf, (size_t)m, sizeof(int64_t), cmp_i64);
    /* a periodic axis with fewer than three cells visits a cell twice */
    int64_t k = 0;
    for (int64_t t = 0; t < m; ++t)
        if (k == 0 || (*buf)[k - 1] != (*buf)[t]) (*buf)[k++] = (*buf)[t];
    return k;
}

/* F, T: [np][3] outputs = collision + lubrication (+ walls) from the state x,u,w */
void orc_dem_forces(const orc_params *p, int64_t np, const double *x, const double *u, const double *w,
                    const double *d, const double *rho_p, double dt_dem, double *F, double *T)
{
    double dmax = 0.0;
    for (int64_t i = 0; i < np; ++i) dmax = fmax(dmax, d[i]);
    double reach = dmax + (p->use_lub ? fmax(p->h_c, 0.0) : 0.0);
    celllist cl;
    cl_build(p, np, x, reach, &cl);
#pragma omp parallel
    {
        int64_t *buf = NULL, cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < np; ++i) {
            pinfo pi = {0.5 * d[i], rho_p[i] * sphere_volume(d[i]), 0.0, x + 3 * i, u + 3 * i, w + 3 * i, d[i]};
            double f[3] = {0.0, 0.0, 0.0}, t[3] = {0.0, 0.0, 0.0};
            int64_t m = partners(p, &cl, np, x, i, &buf, &cap);
            for (int64_t k = 0; k < m; ++k) {
                int64_t j = buf[k];
                pinfo pj = {0.5 * d[j], rho_p[j] * sphere_volume(d[j]), 0.0, x + 3 * j, u + 3 * j, w + 3 * j, d[j]};
                double dx[3];
                for (int a = 0; a < 3; ++a) {
                    dx[a] = x[3 * j + a] - x[3 * i + a];
                    if (p->periodic[a]) dx[a] -= p->n[a] * nearbyint(dx[a] / p->n[a]);
                }
                pair_interaction(p, &pi, &pj, dx, dt_dem, f, t);
            }
            wall_interaction(p, &pi, dt_dem, f, t);
            for (int a = 0; a < 3; ++a) {
                F[3 * i + a] = f[a];
                T[3 * i + a] = t[a];
            }
        }
        free(buf);
    }
    cl_free(&cl);
}

/* ---------------------------------------------------------------------------
 * Diagnostics (Sec. 4.1, mean relative settling velocity; conservation)
 * ------------------------------------------------------------------------- */
typedef struct {
    double mass_dev;      /* sum_x (rho - 1) */
    double mom_fluid[3];  /* sum_x sum_q c_q f_q */
    double mom_part[3];   /* sum_p m_p u_p */
    double u_ps;          /* mean_p u_p,z - mean_x u_f,z */
    double mean_eps_f;
    double min_eps_f;
    double max_u;
} orc_diag;

void orc_diagnostics(const orc_params *p, const orc_state *s, orc_diag *out)
{
    int64_t nc = NC(p), np = s->np;
    double *eps = malloc(sizeof(double) * (size_t)nc);
    orc_eps_field(p, np, s->x, s->d, eps);
    double mass = 0.0, mf[3] = {0, 0, 0}, se = 0.0, mine = 1e300, maxu = 0.0, sufz = 0.0;
    for (int64_t c = 0; c < nc; ++c) {
        double f[Q], drho, j[3];
        for (int q = 0; q < Q; ++q) f[q] = s->df[q * nc + c];
        orc_moments(f, &drho, j);
        double rho = 1.0 + drho;
        mass += drho;
        double ub[3];
        for (int a = 0; a < 3; ++a) {
            mf[a] += j[a];
            /* volume-averaged velocity with the body force only (Eq. MacVel) */
            ub[a] = (j[a] + 0.5 * eps[c] * p->fb[a]) / rho;
        }
        double un = sqrt(dot(ub, ub));
        if (un > maxu) maxu = un;
        sufz += ub[2] / eps[c];  /* u_f = u_bar / eps_f */
        se += eps[c];
        if (eps[c] < mine) mine = eps[c];
    }
    double mp[3] = {0, 0, 0}, supz = 0.0;
    for (int64_t i = 0; i < np; ++i) {
        double m = s->rho_p[i] * sphere_volume(s->d[i]);
        for (int a = 0; a < 3; ++a) mp[a] += m * s->u[3 * i + a];
        supz += s->u[3 * i + 2];
    }
    out->mass_dev = mass;
    for (int a = 0; a < 3; ++a) {
        out->mom_fluid[a] = mf[a];
        out->mom_part[a] = mp[a];
    }
    out->u_ps = (np > 0 ? supz / (double)np : 0.0) - sufz / (double)nc;
    out->mean_eps_f = se / (double)nc;
    out->min_eps_f = mine;
    out->max_u = maxu;
    free(eps);
}

/* ---------------------------------------------------------------------------
 * One coupled time step, Alg. 1 (Sec. 3.3), in the paper's order:
 *
 *   S1  Du_f/Dt from the post-stream state (not re-evaluated in subcycles,
 *       Sec. 3.2.3 stability measures).
 *   S2  n_int interaction subcycles, each:
 *       (a) f_ext := eps_f f_b                   (external body force)
 *       (b) u_f and, with lift on, curl u_f (grad P depends on rho only
 *           and is evaluated once per step)
 *       (c) F_l (lift on) and F_am per particle, distributed to f_ext
 *       (d) u_f once more, now including the spread forces of (c)
 *       (e) F_pr, F_d per particle, F_d distributed; F_g (+ buoyancy)
 *       (f) accumulate f_ext / n_int for the LBM step
 *       (g) n_DEM DEM substeps with the fluid forces frozen
 *       (h) du_p/dt over the subcycle, for the next added-mass evaluation
 *       (i) eps_f at the new particle positions
 *   S3  GNS-LBM collide + stream with eps_f and the averaged force density.
 *
 * Readings (the paper does not fix these; parity unpinned against it):
 *  - Du_f/Dt = (u_f^n - u_f^{n-1})/dt + (u_f^n . grad) u_f^n, where u_f^n is
 *    the fluid-phase velocity of the post-stream state with f_ext = eps_f f_b
 *    and the gradient is the lattice operator; at the first step the time
 *    derivative part is zero.
 *  - du_p/dt in F_am is the velocity change over the previous interaction
 *    subcycle divided by its length (zero at start).
 *  - f_ext is rebuilt at every subcycle; the LBM uses the mean of the
 *    subcycles' f_ext, which keeps the momentum exchange between the phases
 *    exact.
 *  - Gravity acts on the particles only; buoyancy -rho_f V g is added to
 *    them (Sec. 3.1.2, pressure force paragraph); rho_f is the constant
 *    closure density.
 *  - Time integration: semi-implicit Euler u += dt F/m, w += dt T/I,
 *    x += dt u, all forces from the substep's initial state.
 *  - T_c <= 0 selects T_c = 20 dt_DEM.
 * ------------------------------------------------------------------------- */
int orc_step(const orc_params *pin, orc_state *s, orc_aux *aux)
{
    orc_params P = *pin;
    const orc_params *p = &P;
    const int64_t nc = NC(p), np = s->np;
    const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
    const double dt_int = 1.0 / p->n_int;
    const double dt_dem = dt_int / p->n_dem;
    if (P.T_c <= 0.0) P.T_c = 20.0 * dt_dem;
    const double mu = mu0(p);
    int status = 0;

    double *rho = malloc(sizeof(double) * (size_t)nc);
    double *drho = malloc(sizeof(double) * (size_t)nc);
    double *j = malloc(sizeof(double) * 3 * (size_t)nc);
    double *eps = malloc(sizeof(double) * (size_t)nc);
    double *un = malloc(sizeof(double) * 3 * (size_t)nc);
    double *dudt = malloc(sizeof(double) * 3 * (size_t)nc);
    double *gradp = malloc(sizeof(double) * 3 * (size_t)nc);
    double *fext = malloc(sizeof(double) * 3 * (size_t)nc);
    double *facc = calloc(3 * (size_t)nc, sizeof(double));
    double *uf = malloc(sizeof(double) * 3 * (size_t)nc);
    double *epsp = malloc(sizeof(double) * (size_t)nc);
    double *uf0 = malloc(sizeof(double) * 3 * (size_t)nc);
    double *curl = calloc(3 * (size_t)nc, sizeof(double));
    double *Fl = calloc(3 * (size_t)(np + 1), sizeof(double));
    double *Fam = calloc(3 * (size_t)(np + 1), sizeof(double));
    double *Fd = calloc(3 * (size_t)(np + 1), sizeof(double));
    double *Fpr = calloc(3 * (size_t)(np + 1), sizeof(double));
    double *Fc = calloc(3 * (size_t)(np + 1), sizeof(double));
    double *Fdem = calloc(3 * (size_t)(np + 1), sizeof(double));
    double *Tdem = calloc(3 * (size_t)(np + 1), sizeof(double));
    double *ustart = calloc(3 * (size_t)(np + 1), sizeof(double));
    stencil27 *st = malloc(sizeof(stencil27) * (size_t)(np + 1));
    double imp_pr[3] = {0, 0, 0}, imp_gb[3] = {0, 0, 0}, imp_fb[3] = {0, 0, 0};

    /* S0: moments of the current post-stream PDFs (Eq. MacVel) */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double f[Q], jj[3], dr;
        for (int q = 0; q < Q; ++q) f[q] = s->df[q * nc + c];
        orc_moments(f, &dr, jj);
        drho[c] = dr;
        rho[c] = 1.0 + dr;
        for (int a = 0; a < 3; ++a) j[a * nc + c] = jj[a];
    }
    orc_eps_field(p, np, s->x, s->d, eps);

    /* S1: Du_f/Dt, stored per cell (Alg. 1; Table 1 added mass). u_f is the
     * fluid-phase velocity u_bar/eps_f (Sec. 3.2.3), u_bar from Eq. MacVel
     * with f_ext = eps_f f_b. */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        for (int a = 0; a < 3; ++a)
            un[a * nc + c] = (j[a * nc + c] + 0.5 * eps[c] * p->fb[a]) / (rho[c] * eps[c]);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int jj = 0; jj < ny; ++jj)
            for (int i = 0; i < nx; ++i) {
                int64_t c = CIDX(p, i, jj, k);
                /* lattice gradient G[a][b] = d u_b / d x_a */
                double G[3][3] = {{0}}, gp[3] = {0, 0, 0};
                for (int q = 0; q < Q; ++q) {
                    double sg;
                    int64_t nb = ghost_cell(p, i, jj, k, q, &sg);
                    for (int a = 0; a < 3; ++a) {
                        for (int b = 0; b < 3; ++b) G[a][b] += WQ(q) * CV[q][a] * (sg * un[b * nc + nb]);
                        /* grad P with P = eps_f p = c_s^2 rho (Eq. MacVel, pressure);
                         * (1/c_s^2) sum_q w_q c_q P(x+c_q) = sum_q w_q c_q (rho - 1)(x+c_q)
                         * because sum_q w_q c_q = 0 */
                        gp[a] += WQ(q) * CV[q][a] * drho[nb];
                    }
                }
                for (int b = 0; b < 3; ++b) {
                    double conv = 0.0;
                    for (int a = 0; a < 3; ++a) conv += un[a * nc + c] * (3.0 * G[a][b]);
                    double dtu = s->step > 0 ? (un[b * nc + c] - s->uprev[b * nc + c]) : 0.0;
                    dudt[b * nc + c] = dtu + conv;
                    gradp[b * nc + c] = gp[b];
                }
            }
    /* keep u_f^n for the next step's time derivative */
    memcpy(s->uprev, un, sizeof(double) * 3 * (size_t)nc);

    /* S2: interaction subcycles */
    for (int sc = 0; sc < p->n_int; ++sc) {
        /* (a) f_ext = eps_f f_b */
        for (int64_t c = 0; c < nc; ++c)
            for (int a = 0; a < 3; ++a) fext[a * nc + c] = eps[c] * p->fb[a];
        for (int a = 0; a < 3; ++a) {
            double se = 0.0;
            for (int64_t c = 0; c < nc; ++c) se += eps[c];
            imp_fb[a] += se * p->fb[a] * dt_int;
        }
        for (int64_t i = 0; i < np; ++i) particle_stencil(p, s->x + 3 * i, &st[i]);

        /* (b) u_f = (j + f_ext/2) / (rho eps_f) at the subcycle start and its
         *     lattice curl (Alg. 1, first step of the subcycle loop) */
        if (p->use_lift) {
            for (int64_t c = 0; c < nc; ++c)
                for (int a = 0; a < 3; ++a)
                    uf0[a * nc + c] = (j[a * nc + c] + 0.5 * fext[a * nc + c]) / (rho[c] * eps[c]);
            orc_curl_field(p, uf0, curl);
        }

        /* (c) lift (Table 1) from u_f and curl u_f of (b), and added mass,
         *     F_am = C_am rho_f V (Du_f/Dt|p - du_p/dt); their sum is
         *     distributed with Eq. forces_pf (minus sign: reaction on the fluid) */
        for (int64_t i = 0; i < np; ++i) {
            double V = sphere_volume(s->d[i]);
            double Du[3], F1[3];
            interp(p, &st[i], dudt, 3, Du);
            for (int a = 0; a < 3; ++a)
                Fam[3 * i + a] = p->use_am ? p->c_am * p->rho_f * V * (Du[a] - s->a[3 * i + a]) : 0.0;
            if (p->use_lift) {
                double om[3], ufp[3], w[3];
                interp(p, &st[i], curl, 3, om);
                interp(p, &st[i], uf0, 3, ufp);
                for (int a = 0; a < 3; ++a) w[a] = ufp[a] - s->u[3 * i + a];
                orc_lift(s->d[i], mu, p->rho_f, w, om, Fl + 3 * i);
            }
            for (int a = 0; a < 3; ++a) F1[a] = Fam[3 * i + a] + Fl[3 * i + a];
            spread(p, &st[i], fext, 3, F1, -1.0);
        }

        /* (d) u_f = (j + f_ext/2) / (rho eps_f), f_ext now holding the spread forces */
        for (int64_t c = 0; c < nc; ++c) {
            for (int a = 0; a < 3; ++a) uf[a * nc + c] = (j[a * nc + c] + 0.5 * fext[a * nc + c]) / (rho[c] * eps[c]);
            epsp[c] = 1.0 - eps[c];
        }

        /* (e) pressure gradient force, drag, gravity + buoyancy */
        for (int64_t i = 0; i < np; ++i) {
            double V = sphere_volume(s->d[i]);
            double ufp[3], gpp[3], ep, w[3];
            interp(p, &st[i], uf, 3, ufp);
            interp(p, &st[i], gradp, 3, gpp);
            interp(p, &st[i], epsp, 1, &ep);
            for (int a = 0; a < 3; ++a) {
                Fpr[3 * i + a] = -V * gpp[a];
                w[a] = ufp[a] - s->u[3 * i + a];
            }
            orc_drag(s->d[i], mu, p->rho_f, ep, w, Fd + 3 * i);
            spread(p, &st[i], fext, 3, Fd + 3 * i, -1.0);
            for (int a = 0; a < 3; ++a) {
                double fgb = (s->rho_p[i] - p->rho_f) * V * p->g[a];
                Fc[3 * i + a] = Fd[3 * i + a] + Fpr[3 * i + a] + Fam[3 * i + a] + Fl[3 * i + a] + fgb;
                imp_pr[a] += Fpr[3 * i + a] * dt_int;
                imp_gb[a] += fgb * dt_int;
            }
        }

        /* (f) subcycle-averaged force density for the LBM step */
        for (int64_t c = 0; c < 3 * nc; ++c) facc[c] += fext[c] * dt_int;

        /* (g) DEM substeps with F_fp + F_g frozen (Sec. 3.3) */
        memcpy(ustart, s->u, sizeof(double) * 3 * (size_t)np);
        for (int sub = 0; sub < p->n_dem; ++sub) {
            orc_dem_forces(p, np, s->x, s->u, s->w, s->d, s->rho_p, dt_dem, Fdem, Tdem);
            for (int64_t i = 0; i < np; ++i) {
                double V = sphere_volume(s->d[i]);
                double m = s->rho_p[i] * V;
                double I = m * s->d[i] * s->d[i] / 10.0;
                for (int a = 0; a < 3; ++a) {
                    s->u[3 * i + a] += dt_dem * (Fc[3 * i + a] + Fdem[3 * i + a]) / m;
                    s->w[3 * i + a] += dt_dem * Tdem[3 * i + a] / I;
                    s->x[3 * i + a] += dt_dem * s->u[3 * i + a];
                    if (p->periodic[a]) {
                        /* periodic wrap into [0, L); a tiny negative coordinate
                         * whose shifted value rounds to L is mapped to 0 */
                        double L = (double)p->n[a];
                        if (s->x[3 * i + a] >= L) s->x[3 * i + a] -= L;
                        else if (s->x[3 * i + a] < 0.0) {
                            s->x[3 * i + a] += L;
                            if (s->x[3 * i + a] >= L) s->x[3 * i + a] = 0.0;
                        }
                    } else if (!(s->x[3 * i + a] > 0.0 && s->x[3 * i + a] < (double)p->n[a])) {
                        status = 3;
                    }
                }
            }
        }
        /* (h) du_p/dt over the subcycle */
        for (int64_t i = 0; i < 3 * np; ++i) s->a[i] = (s->u[i] - ustart[i]) / dt_int;

        /* (i) eps_f from the new positions */
        orc_eps_field(p, np, s->x, s->d, eps);
    }

    double mine = 1e300;
    for (int64_t c = 0; c < nc; ++c) {
        if (!(eps[c] > 0.0) || !isfinite(eps[c])) status = 3;
        if (eps[c] < mine) mine = eps[c];
    }

    /* S3: GNS-LBM step. Reading for the failure checks (the paper states no
     * limits): besides non-finite values, a cell velocity
     * u_bar = (j + f_acc/2)/rho of magnitude above 0.1 is flagged, beyond
     * the low-Mach range in which the second-order equilibrium holds. */
    for (int64_t c = 0; c < nc; ++c) {
        double uu = 0.0;
        for (int a = 0; a < 3; ++a) {
            double ua = (j[a * nc + c] + 0.5 * facc[a * nc + c]) / rho[c];
            uu += ua * ua;
        }
        if (!(uu <= 0.01)) status = 3;
    }
    double *dfn = malloc(sizeof(double) * Q * (size_t)nc);
    orc_lbm_collide_stream(p, s->df, dfn, eps, facc);
    for (int64_t c = 0; c < Q * nc; ++c)
        if (!isfinite(dfn[c])) status = 3;
    memcpy(s->df, dfn, sizeof(double) * Q * (size_t)nc);
    free(dfn);
    for (int64_t i = 0; i < 3 * np; ++i)
        if (!isfinite(s->x[i]) || !isfinite(s->u[i])) status = 3;
    s->step += 1;

    if (aux) {
        if (aux->f_acc) memcpy(aux->f_acc, facc, sizeof(double) * 3 * (size_t)nc);
        if (aux->eps_f) memcpy(aux->eps_f, eps, sizeof(double) * (size_t)nc);
        if (aux->dudt) memcpy(aux->dudt, dudt, sizeof(double) * 3 * (size_t)nc);
        if (aux->gradp) memcpy(aux->gradp, gradp, sizeof(double) * 3 * (size_t)nc);
        if (aux->rho) memcpy(aux->rho, rho, sizeof(double) * (size_t)nc);
        if (aux->j) memcpy(aux->j, j, sizeof(double) * 3 * (size_t)nc);
        if (aux->F_am) memcpy(aux->F_am, Fam, sizeof(double) * 3 * (size_t)np);
        if (aux->F_d) memcpy(aux->F_d, Fd, sizeof(double) * 3 * (size_t)np);
        if (aux->F_pr) memcpy(aux->F_pr, Fpr, sizeof(double) * 3 * (size_t)np);
        if (aux->F_const) memcpy(aux->F_const, Fc, sizeof(double) * 3 * (size_t)np);
        if (aux->F_l) memcpy(aux->F_l, Fl, sizeof(double) * 3 * (size_t)np);
        if (aux->curl) memcpy(aux->curl, curl, sizeof(double) * 3 * (size_t)nc);
        for (int a = 0; a < 3; ++a) {
            aux->impulse_pr[a] = imp_pr[a];
            aux->impulse_gb[a] = imp_gb[a];
            aux->impulse_fb[a] = imp_fb[a];
        }
        aux->min_eps_f = mine;
        aux->status = status;
    }

    free(rho); free(drho); free(j); free(eps); free(un); free(dudt); free(gradp);
    free(fext); free(facc); free(uf); free(epsp); free(Fam); free(Fd); free(Fpr);
    free(Fc); free(Fdem); free(Tdem); free(ustart); free(st); free(uf0); free(curl); free(Fl);
    return status;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
