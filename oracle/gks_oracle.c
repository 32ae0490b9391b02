/*
 * gks_oracle.c -- plain, slow FP64 CPU oracle of the turbulent gas-kinetic scheme
 * (M. Righi, "A gas-kinetic scheme for the simulation of compressible turbulent
 * flows", arXiv:1302.2132, 2013): per-interface BGK flux with a k-omega turbulent
 * relaxation time, followed by the finite-volume update.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code, header,
 * table or helper with the HIP library; the two meet only through the seeded
 * input generators.
 *
 * How it computes (deliberately the long way):
 *  - Every velocity-space integral is evaluated generically: the integrand is
 *    expanded into monomials u^a v^b w^c (xi^2)^q and each monomial's moment is
 *    the product of one-dimensional Gaussian moments (full range, u>0 or u<0).
 *  - Every expansion coefficient (a, A, a-bar, A-bar) is found by assembling the
 *    moment matrix <psi_m psi_n>_g monomial by monomial and solving it by
 *    Gaussian elimination with partial pivoting.
 *  - The time-integrated distribution of the Kogan solution is kept as a list of
 *    terms (weight, Maxwellian, half space, polynomial); flux, its u-less twin G
 *    and the heat flux are integrals of that list against u*psi, psi and the
 *    peculiar-velocity heat-flux polynomial.
 *
 * Readings of the paper (each also listed in the design notes):
 *  - Maxwellian normalisation (lambda/pi)^(b/2), b = D + K = 2/(gamma-1) total
 *    degrees of freedom, K = b - D internal ones (Eq. maxwellian and the sentence
 *    after it).
 *  - The left state feeds u>0 and the right state u<0 in the interface state
 *    (Eq. intermediatestate, Heaviside labels read as h_l = H(u), h_r = 1-H(u)).
 *  - Equilibrium expansion g = g0 (1 + abar x + Abar t) (Eq. eqlgform read with +Abar t,
 *    consistent with the (t - tau + tau e^{-t/tau}) Abar term of Eq. resultingf);
 *    the left slope/time terms of Eq. resultingf carry h_l, a_l, A_l.
 *  - abar_l, abar_r from (W0 - Wbar_i)/(x_{i+1/2}-x_i) and (Wbar_{i+1}-W0)/(x_{i+1}-x_{i+1/2}).
 *  - Abar from the compatibility condition integrated over [0, dt].
 *  - The flux is the exact time integral of Eq. resultingf (Eq. fluxesf); the compact
 *    alpha/beta form of Eq. resultingf4 is not used for the flux.
 *  - tau = mu/p0 + tau_a (Eq. taua) + (k/omega)/(T sqrt(1+eta^2)) (Eq. tautchenadjusted)
 *    with T = p0/rho0, eta = S/(C_mu omega), interface state W0.
 *  - Prandtl correction: F_E += (1/Pr - 1) q, q the time-integrated heat flux of the
 *    interface distribution in the frame of U0.
 *  - k-omega transport (og_run_kw; the turbulence-model equations that the implementation
 *    section solves beside the flow, with the Wilcox 2006 k-omega model the paper names):
 *    conservative rho k,
 *    rho omega; convection with the GKS time-integrated mass flux, upwind by its sign;
 *    face diffusion with mu + sigma* rho k/omega and mu + sigma rho k/omega (face means of
 *    the two cells); production P from the paper's turbulent viscosity
 *    mu_t = rho k/(omega sqrt(1+eta^2)); cross-diffusion sigma_d (rho/omega) grad k.grad omega
 *    where that product is positive; the sinks beta* omega rho k and beta omega rho omega
 *    point-implicit in the step; a ghost cell's k, omega and, in the face diffusion,
 *    density take their interior image's values.
 *  - Reconstruction (the paper names second- and third-order TVD/MUSCL and fifth-order
 *    WENO, with minmod on the variables and their gradients): the gradients are always
 *    the minmod of the one-sided slopes; the face values come from them, from the limited
 *    kappa = 1/3 slopes, or from Jiang and Shu's WENO5 applied to the conservative
 *    variables in index space (uniform-grid coefficients on stretched meshes too), which
 *    needs three ghost layers and at least three cells per axis.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_OK 0
#define OG_ERR_ARG 1
#define OG_ERR_NONPHYSICAL 2

#define OG_MAXT 256   /* monomials per polynomial (largest product: heat-flux polynomial x (u a.psi), 160 terms in 3D) */
#define OG_NU 12      /* u powers kept */
#define OG_NT 9       /* tangential powers kept */

enum { OG_PERIODIC = 0, OG_WALL = 1, OG_DIRICHLET = 2, OG_PROFILE = 3, OG_OUTFLOW = 4 };
enum { R_ALL = 0, R_POS = 1, R_NEG = 2 };

/* ------------------------------------------------------------------------ */
/* Gas and Maxwellian parameters                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dim;           /* 2 or 3 */
    double b;          /* total degrees of freedom 2/(gamma-1) */
    double K;          /* internal degrees of freedom b - dim */
    double gamma, prandtl, mu, c_a, c_mu;
    int eps_mode;      /* 0: rarefaction eps = tau/dt; 1: eps = tau/tau_hat (see og_face) */
    int multi_d;       /* 1: the distributions are expanded along the tangential axes too */
} og_gas;

typedef struct {       /* face-local frame: U[0] is the face-normal velocity */
    double rho, U[3], lam;
} og_maxw;

typedef struct {
    double u[3][OG_NU];   /* <u^n>: all u, u>0, u<0 (rho-normalised) */
    double v[OG_NT];      /* <v^n> full range */
    double w[OG_NT];      /* <w^n> full range (3D) */
    double xi[3];         /* <(xi^2)^q> */
} og_mom;

/* ------------------------------------------------------------------------ */
/* Polynomials in (u, v, w, xi^2)                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    double c[OG_MAXT];
    signed char e[OG_MAXT][4];
} og_poly;

static void p_term(og_poly* p, double c, int a, int b, int cc, int q)
{
    if (p->n >= OG_MAXT) { fprintf(stderr, "gks_oracle: polynomial overflow\n"); abort(); }
    p->c[p->n] = c;
    p->e[p->n][0] = (signed char)a; p->e[p->n][1] = (signed char)b;
    p->e[p->n][2] = (signed char)cc; p->e[p->n][3] = (signed char)q;
    p->n++;
}

static void p_const(og_poly* p, double c) { p->n = 0; p_term(p, c, 0, 0, 0, 0); }

/* psi_m in the face-local frame: 1, u, v, [w], (u^2+v^2+[w^2]+xi^2)/2 */
static void p_psi(int dim, int m, og_poly* p)
{
    p->n = 0;
    if (m == 0) { p_term(p, 1.0, 0, 0, 0, 0); return; }
    if (m <= dim) {
        int a = m - 1;
        p_term(p, 1.0, a == 0, a == 1, a == 2, 0);
        return;
    }
    p_term(p, 0.5, 2, 0, 0, 0);
    p_term(p, 0.5, 0, 2, 0, 0);
    if (dim == 3) p_term(p, 0.5, 0, 0, 2, 0);
    p_term(p, 0.5, 0, 0, 0, 1);
}

/* a . psi */
static void p_lin(int dim, const double* a, og_poly* p)
{
    og_poly t;
    p->n = 0;
    for (int m = 0; m < dim + 2; ++m) {
        p_psi(dim, m, &t);
        for (int i = 0; i < t.n; ++i)
            p_term(p, a[m] * t.c[i], t.e[i][0], t.e[i][1], t.e[i][2], t.e[i][3]);
    }
}

static void p_mul(const og_poly* a, const og_poly* b, og_poly* out)
{
    out->n = 0;
    for (int i = 0; i < a->n; ++i)
        for (int j = 0; j < b->n; ++j)
            p_term(out, a->c[i] * b->c[j], a->e[i][0] + b->e[j][0], a->e[i][1] + b->e[j][1],
                   a->e[i][2] + b->e[j][2], a->e[i][3] + b->e[j][3]);
}

static void p_upow(og_poly* p, int k)
{
    for (int i = 0; i < p->n; ++i) p->e[i][0] = (signed char)(p->e[i][0] + k);
}

/* multiply by the tangential velocity t (0: v, 1: w) */
static void p_tpow(og_poly* p, int t)
{
    for (int i = 0; i < p->n; ++i) p->e[i][1 + t] = (signed char)(p->e[i][1 + t] + 1);
}

/* <p>_g over the u-range `range` (tangential and internal variables over all values) */
static double p_expect(const og_poly* p, const og_mom* M, int range)
{
    double s = 0.0;
    for (int i = 0; i < p->n; ++i) {
        int a = p->e[i][0], b = p->e[i][1], c = p->e[i][2], q = p->e[i][3];
        if (a >= OG_NU || b >= OG_NT || c >= OG_NT || q > 2) {
            fprintf(stderr, "gks_oracle: moment order out of table\n"); abort();
        }
        s += p->c[i] * M->u[range][a] * M->v[b] * M->w[c] * M->xi[q];
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Moments of a Maxwellian                                                  */
/* ------------------------------------------------------------------------ */
/* One-dimensional Gaussian moments with mean U and variance 1/(2 lambda):
 *   <u^{n+1}> = U <u^n> + n/(2 lambda) <u^{n-1}>            (all u)
 * and for the half lines the same recurrence after the first two terms,
 *   <u^0>_{>0} = erfc(-sqrt(lambda) U)/2,  <u^1>_{>0} = U <u^0>_{>0} + e^{-lambda U^2}/(2 sqrt(pi lambda)),
 *   <u^0>_{<0} = erfc( sqrt(lambda) U)/2,  <u^1>_{<0} = U <u^0>_{<0} - e^{-lambda U^2}/(2 sqrt(pi lambda)),
 * (integration by parts of the Gaussian; the boundary term at u = 0 appears only for n = 0).
 * Internal variable: K independent Gaussian components, <xi^2> = K/(2 lambda),
 * <xi^4> = K(K+2)/(4 lambda^2). */
static void og_moments(const og_gas* gas, const og_maxw* g, og_mom* M)
{
    const double lam = g->lam, U = g->U[0];
    const double h = 1.0 / (2.0 * lam);
    const double sl = sqrt(lam);
    const double tail = exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
    M->u[R_ALL][0] = 1.0;
    M->u[R_ALL][1] = U;
    M->u[R_POS][0] = 0.5 * erfc(-sl * U);
    M->u[R_POS][1] = U * M->u[R_POS][0] + tail;
    M->u[R_NEG][0] = 0.5 * erfc(sl * U);
    M->u[R_NEG][1] = U * M->u[R_NEG][0] - tail;
    for (int r = 0; r < 3; ++r)
        for (int n = 1; n + 1 < OG_NU; ++n)
            M->u[r][n + 1] = U * M->u[r][n] + n * h * M->u[r][n - 1];
    const double V = g->U[1], Wt = g->U[2];
    M->v[0] = 1.0; M->v[1] = V;
    M->w[0] = 1.0; M->w[1] = (gas->dim == 3) ? Wt : 0.0;
    for (int n = 1; n + 1 < OG_NT; ++n) {
        M->v[n + 1] = V * M->v[n] + n * h * M->v[n - 1];
        M->w[n + 1] = (gas->dim == 3) ? Wt * M->w[n] + n * h * M->w[n - 1] : 0.0;
    }
    M->xi[0] = 1.0;
    M->xi[1] = gas->K * h;
    M->xi[2] = gas->K * (gas->K + 2.0) * h * h;
}

/* Conservative (face-local) -> Maxwellian parameters.  p = (2/b)(rho E - rho|U|^2/2),
 * lambda = rho/(2p). */
static int og_prim(const og_gas* gas, const double* W, og_maxw* g)
{
    const int dim = gas->dim;
    const double rho = W[0];
    if (!(rho > 0.0) || !isfinite(rho)) return OG_ERR_NONPHYSICAL;
    double ke = 0.0;
    g->U[0] = g->U[1] = g->U[2] = 0.0;
    for (int d = 0; d < dim; ++d) { g->U[d] = W[1 + d] / rho; ke += g->U[d] * W[1 + d]; }
    const double p = (2.0 / gas->b) * (W[dim + 1] - 0.5 * ke);
    if (!(p > 0.0) || !isfinite(p)) return OG_ERR_NONPHYSICAL;
    g->rho = rho;
    g->lam = rho / (2.0 * p);
    return OG_OK;
}

/* Solve  sum_n <psi_m psi_n>_g x_n = r_m  (Gaussian elimination, partial pivoting). */
static int og_solve_moment_system(const og_gas* gas, const og_mom* M, const double* r, double* x)
{
    const int nv = gas->dim + 2;
    double A[5][6];
    og_poly pm, pn, prod;
    for (int m = 0; m < nv; ++m) {
        p_psi(gas->dim, m, &pm);
        for (int n = 0; n < nv; ++n) {
            p_psi(gas->dim, n, &pn);
            p_mul(&pm, &pn, &prod);
            A[m][n] = p_expect(&prod, M, R_ALL);
        }
        A[m][nv] = r[m];
    }
    for (int col = 0; col < nv; ++col) {
        int piv = col;
        for (int row = col + 1; row < nv; ++row)
            if (fabs(A[row][col]) > fabs(A[piv][col])) piv = row;
        if (A[piv][col] == 0.0) return OG_ERR_NONPHYSICAL;
        if (piv != col)
            for (int j = 0; j <= nv; ++j) { double t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
        for (int row = col + 1; row < nv; ++row) {
            double f = A[row][col] / A[col][col];
            for (int j = col; j <= nv; ++j) A[row][j] -= f * A[col][j];
        }
    }
    for (int row = nv - 1; row >= 0; --row) {
        double s = A[row][nv];
        for (int j = row + 1; j < nv; ++j) s -= A[row][j] * x[j];
        x[row] = s / A[row][row];
    }
    return OG_OK;
}

/* ------------------------------------------------------------------------ */
/* Time weights of the Kogan solution                                       */
/* ------------------------------------------------------------------------ */
/* Integrating Eq. resultingf over [0, dt] term by term (E = e^{-dt/tau}):
 *   g0 term          (1 - e^{-t/tau})                 -> gam0 = dt - tau (1-E)
 *   u abar g0 term   (-tau + tau e^{-t/tau} + t e^{-t/tau}) -> gam1 = 2 tau^2 (1-E) - tau dt (1+E)
 *   Abar g0 term     (t - tau + tau e^{-t/tau})       -> gam2 = dt^2/2 - tau dt + tau^2 (1-E)
 *   g_l, g_r term    e^{-t/tau}                       -> gam3 = tau (1-E)
 *   u a g_{l,r} term -(t + tau) e^{-t/tau}            -> gam4 = -(2 tau^2 (1-E) - tau dt E)
 *   A g_{l,r} term   -tau e^{-t/tau}                  -> gam5 = -tau^2 (1-E)
 * The time-integrated compatibility condition divides by tau*gam0; the ratios
 * c1 = gam1/(tau gam0), c4 = gam4/(tau gam0), c5 = gam5/(tau gam0) depend on x = dt/tau only.
 * For x < 1/2 the cancelling combinations are summed as Taylor series in x. */
typedef struct { double g[6]; double c1, c4, c5; } og_tw;

static void og_kogan_weights(double tau, double dt, og_tw* k)
{
    if (tau <= 0.0) {   /* collisionless limit is not this; tau = 0 is the Euler limit f = g */
        k->g[0] = dt; k->g[1] = 0.0; k->g[2] = 0.5 * dt * dt;
        k->g[3] = 0.0; k->g[4] = 0.0; k->g[5] = 0.0;
        k->c1 = -1.0; k->c4 = 0.0; k->c5 = 0.0;
        return;
    }
    const double x = dt / tau;
    double s, g0, g1, g2, g4;
    if (x < 0.5) {
        /* s  = sum_{n>=1} (-1)^{n+1} x^n/n!
           g0 = x - s             = sum_{n>=2} (-1)^n x^n/n!
           g1 = 2s - x(1+e^{-x})  = sum_{n>=3} (-1)^n (n-2) x^n/n!
           g2 = x^2/2 - x + s     = sum_{n>=3} (-1)^{n+1} x^n/n!
           g4 = 2s - x e^{-x}     = x + g1 */
        double term = 1.0;   /* x^n/n! */
        s = g0 = g1 = g2 = 0.0;
        for (int n = 1; n <= 40; ++n) {
            term *= x / n;
            double sg = (n % 2) ? 1.0 : -1.0;   /* (-1)^{n+1} */
            s += sg * term;
            if (n >= 2) g0 -= sg * term;
            if (n >= 3) { g1 -= sg * (n - 2) * term; g2 += sg * term; }
            if (term < 1e-300) break;
        }
        g4 = x + g1;
    } else {
        const double E = exp(-x);
        s = 1.0 - E;
        g0 = x - s;
        g1 = 2.0 * s - x * (1.0 + E);
        g2 = 0.5 * x * x - x + s;
        g4 = 2.0 * s - x * E;
    }
    k->g[0] = tau * g0;
    k->g[1] = tau * tau * g1;
    k->g[2] = tau * tau * g2;
    k->g[3] = tau * s;
    k->g[4] = -tau * tau * g4;
    k->g[5] = -tau * tau * s;
    k->c1 = g1 / g0;
    k->c4 = -g4 / g0;
    k->c5 = -s / g0;
}

/* Time weights with the rarefaction measured against a resolved time scale tau_hat
 * (Eqs. tautautilde, rarefactionkepsilon, epsilonkomega).  Eq. resultingf, regrouped as in
 * Eq. resultingf2 but with the slope terms written out exactly, reads
 *   f = f_c (1 + Abar t) + e^{-t/tau} (f_u - f_c) + t e^{-t/tau} u (abar g0 - a g_{l,r}),
 *   f_c = g0 (1 - tau (abar u + Abar)),  f_u = g_{l,r} (1 - tau (a u + A)),
 * and its time average depends on eps = tau/dt only through the averages of e^{-t/tau} and
 * t e^{-t/tau}.  The tau_hat mode evaluates those with eps = tau/tau_hat, i.e. with the
 * decay time tau_e = dt tau/tau_hat in the exponentials, while f_c and f_u keep the
 * physical tau.  With I0 = int_0^dt e^{-t/tau_e} dt and I1 = int_0^dt t e^{-t/tau_e} dt:
 *   gam0 = dt - I0,  gam1 = -tau gam0 + I1,  gam2 = dt^2/2 - tau gam0,
 *   gam3 = I0,       gam4 = -tau I0 - I1,    gam5 = -tau I0,
 * and the integrated compatibility condition keeps its form (gam0 + gam3 = dt), its
 * coefficients being c_j = gam_j/(tau gam0) (1/2 dt^2 - gam2 = tau gam0).  tau_e = tau
 * reproduces og_kogan_weights; tau_e = 0 is the hydrodynamic limit f = f_c (1 + Abar t)
 * (Eq. hydroturbolimit). */
static void og_time_weights(double tau, double tau_e, double dt, og_tw* k)
{
    if (tau <= 0.0) {
        og_kogan_weights(tau, dt, k);
        return;
    }
    double I0, I1, gam0;
    if (tau_e <= 0.0) {
        I0 = 0.0; I1 = 0.0; gam0 = dt;
    } else {
        const double x = dt / tau_e;
        double s, g0, h;   /* s = 1 - e^{-x}, g0 = x - s, h = s - x e^{-x} */
        if (x < 0.5) {
            double term = 1.0;
            s = g0 = h = 0.0;
            for (int n = 1; n <= 40; ++n) {
                term *= x / n;
                double sg = (n % 2) ? 1.0 : -1.0;   /* (-1)^{n+1} */
                s += sg * term;
                if (n >= 2) { g0 -= sg * term; h -= sg * (n - 1) * term; }
                if (term < 1e-300) break;
            }
        } else {
            const double E = exp(-x);
            s = 1.0 - E;
            g0 = x - s;
            h = s - x * E;
        }
        I0 = tau_e * s;
        I1 = tau_e * tau_e * h;
        gam0 = tau_e * g0;
    }
    k->g[0] = gam0;
    k->g[1] = -tau * gam0 + I1;
    k->g[2] = 0.5 * dt * dt - tau * gam0;
    k->g[3] = I0;
    k->g[4] = -tau * I0 - I1;
    k->g[5] = -tau * I0;
    k->c1 = k->g[1] / (tau * gam0);
    k->c4 = k->g[4] / (tau * gam0);
    k->c5 = k->g[5] / (tau * gam0);
}

/* ------------------------------------------------------------------------ */
/* Relaxation time                                                          */
/* ------------------------------------------------------------------------ */
/* tau = mu/p0 + C_a |p_r - p_l|/|p_r + p_l| dt + (k/omega) / (T sqrt(1 + eta^2)),
 * T = p0/rho0, eta = S/(C_mu omega)   (Eqs. relaxation time, taua, tautchenadjusted). */
static double og_tau(const og_gas* gas, double rho0, double p0, double pl, double pr,
                     double kf, double wf, double Sf, double dt)
{
    double tau = gas->mu / p0;
    tau += gas->c_a * fabs(pr - pl) / fabs(pr + pl) * dt;
    const double eta = Sf / (gas->c_mu * wf);
    tau += (kf / wf) / ((p0 / rho0) * sqrt(1.0 + eta * eta));
    return tau;
}

/* ------------------------------------------------------------------------ */
/* One interface, face-local frame                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    double w;         /* weight (density times a time weight) */
    int which;        /* 0: g0, 1: g_l, 2: g_r */
    int range;
    og_poly poly;
} og_term;

/* info layout (doubles): W0[5] a_l[5] a_r[5] A_l[5] A_r[5] abar_l[5] abar_r[5] Abar[5]
 *                        tau gam[6] c1 c4 c5 eps_hat   -> 51 values */
#define OG_INFO_LEN 51

/* <u^k v_t psi_m (b.psi)>_g over the u-range `range` (v_t the tangential velocity t) */
static double og_tan_moment(int dim, const double* b, int t, int m, const og_mom* M, int range, int k)
{
    og_poly pb, pm, prod;
    p_lin(dim, b, &pb);
    p_psi(dim, m, &pm);
    p_mul(&pm, &pb, &prod);
    p_tpow(&prod, t);
    p_upow(&prod, k);
    return p_expect(&prod, M, range);
}

/* tsl, tsr: tangential gradients of the conservative variables of the two cells,
 * [(dim - 1) x 5] in the face-local frame (tangential axis t, component m at t*5 + m), used
 * when gas->multi_d; NULL otherwise. */
static int og_face(const og_gas* gas, const double* Wl, const double* Wr,
                   const double* sl, const double* sr, const double* tsl, const double* tsr,
                   const double* Wi, const double* Wi1,
                   double dxl, double dxr, double kf, double wf, double Sf, double dt,
                   double* F, double* G, double* qout, double* info)
{
    const int dim = gas->dim, nv = dim + 2;
    og_maxw gl, gr, g0;
    og_mom Ml, Mr, M0;
    int st;
    if ((st = og_prim(gas, Wl, &gl)) || (st = og_prim(gas, Wr, &gr))) return st;
    og_moments(gas, &gl, &Ml);
    og_moments(gas, &gr, &Mr);

    /* interface state: left Maxwellian over u>0, right over u<0 (Eq. intermediatestate) */
    double W0[5] = {0, 0, 0, 0, 0};
    og_poly pm, pa, prod, tmp;
    for (int m = 0; m < nv; ++m) {
        p_psi(dim, m, &pm);
        W0[m] = gl.rho * p_expect(&pm, &Ml, R_POS) + gr.rho * p_expect(&pm, &Mr, R_NEG);
    }
    if ((st = og_prim(gas, W0, &g0))) return st;
    og_moments(gas, &g0, &M0);

    /* spatial slopes of the initial distribution: <psi (a.psi)>_g = dW/dx / rho (Eq. initialf0) */
    double a_l[5], a_r[5], A_l[5], A_r[5], ab_l[5], ab_r[5], Ab[5], r[5] = {0, 0, 0, 0, 0};
    for (int m = 0; m < nv; ++m) r[m] = sl[m] / gl.rho;
    if ((st = og_solve_moment_system(gas, &Ml, r, a_l))) return st;
    for (int m = 0; m < nv; ++m) r[m] = sr[m] / gr.rho;
    if ((st = og_solve_moment_system(gas, &Mr, r, a_r))) return st;

    /* multi-dimensional expansion (the alternative the implementation section mentions):
       tangential slopes b of each side from its tangential gradients, and of the interface
       state from the mean of the two, <psi (b.psi)>_g = dW/dy / rho per tangential axis */
    const int ntan = (gas->multi_d && tsl && tsr) ? dim - 1 : 0;
    double b_l[2][5], b_r[2][5], b_0[2][5];
    for (int t = 0; t < ntan; ++t) {
        for (int m = 0; m < nv; ++m) r[m] = tsl[t * 5 + m] / gl.rho;
        if ((st = og_solve_moment_system(gas, &Ml, r, b_l[t]))) return st;
        for (int m = 0; m < nv; ++m) r[m] = tsr[t * 5 + m] / gr.rho;
        if ((st = og_solve_moment_system(gas, &Mr, r, b_r[t]))) return st;
        for (int m = 0; m < nv; ++m) r[m] = 0.5 * (tsl[t * 5 + m] + tsr[t * 5 + m]) / g0.rho;
        if ((st = og_solve_moment_system(gas, &M0, r, b_0[t]))) return st;
    }

    /* time slopes from the compatibility condition at t = 0: <psi (a u + A)>_g = 0 */
    /* (with the expansion: <psi (a u + b.v_t + A)>_g = 0) */
    p_lin(dim, a_l, &pa);
    for (int m = 0; m < nv; ++m) {
        p_psi(dim, m, &pm); p_mul(&pm, &pa, &prod); p_upow(&prod, 1);
        r[m] = -p_expect(&prod, &Ml, R_ALL);
        for (int t = 0; t < ntan; ++t) r[m] -= og_tan_moment(dim, b_l[t], t, m, &Ml, R_ALL, 0);
    }
    if ((st = og_solve_moment_system(gas, &Ml, r, A_l))) return st;
    p_lin(dim, a_r, &pa);
    for (int m = 0; m < nv; ++m) {
        p_psi(dim, m, &pm); p_mul(&pm, &pa, &prod); p_upow(&prod, 1);
        r[m] = -p_expect(&prod, &Mr, R_ALL);
        for (int t = 0; t < ntan; ++t) r[m] -= og_tan_moment(dim, b_r[t], t, m, &Mr, R_ALL, 0);
    }
    if ((st = og_solve_moment_system(gas, &Mr, r, A_r))) return st;

    /* equilibrium slopes from the one-sided differences through W0 (Eq. eqlgform) */
    for (int m = 0; m < nv; ++m) r[m] = (W0[m] - Wi[m]) / (g0.rho * dxl);
    if ((st = og_solve_moment_system(gas, &M0, r, ab_l))) return st;
    for (int m = 0; m < nv; ++m) r[m] = (Wi1[m] - W0[m]) / (g0.rho * dxr);
    if ((st = og_solve_moment_system(gas, &M0, r, ab_r))) return st;

    /* relaxation time and time weights */
    const double p0 = g0.rho / (2.0 * g0.lam);
    const double pl = gl.rho / (2.0 * gl.lam), pr = gr.rho / (2.0 * gr.lam);
    const double tau = og_tau(gas, g0.rho, p0, pl, pr, kf, wf, Sf, dt);
    /* degree of rarefaction against the resolved time scale tau_hat = rho/|D rho| (Eqs.
       tautilde, epsilonkomega), D rho the material derivative at the interface along the
       normal: with the mean of the two one-sided gradients through W0 (those of the
       equilibrium slopes), D rho = d_t rho + U0 d_x rho = U0 d_x rho - d_x (rho U) by mass
       conservation.  eps_hat = tau/tau_hat. */
    double drho = 0.0;
    {
        const double grho = 0.5 * ((W0[0] - Wi[0]) / dxl + (Wi1[0] - W0[0]) / dxr);
        const double gmom = 0.5 * ((W0[1] - Wi[1]) / dxl + (Wi1[1] - W0[1]) / dxr);
        drho = g0.U[0] * grho - gmom;
    }
    const double eps_hat = tau * fabs(drho) / g0.rho;
    og_tw kw;
    if (gas->eps_mode) og_time_weights(tau, dt * eps_hat, dt, &kw);
    else og_kogan_weights(tau, dt, &kw);

    /* Abar from the compatibility condition integrated over [0, dt]:
       int_0^dt int (g - f) psi = 0 ; the W0 terms cancel because gam0 + gam3 = dt, leaving
       rho0 <psi (Abar.psi)>_g0 = c1 rho0 (<u psi abar_l.psi>_{g0,>0} + <u psi abar_r.psi>_{g0,<0})
                                + c4 (rho_l <u psi a_l.psi>_{gl,>0} + rho_r <u psi a_r.psi>_{gr,<0})
                                + c5 (rho_l <psi A_l.psi>_{gl,>0} + rho_r <psi A_r.psi>_{gr,<0}) */
    {
        og_poly q_abl, q_abr, q_al, q_ar, q_Al, q_Ar;
        p_lin(dim, ab_l, &q_abl); p_lin(dim, ab_r, &q_abr);
        p_lin(dim, a_l, &q_al);   p_lin(dim, a_r, &q_ar);
        p_lin(dim, A_l, &q_Al);   p_lin(dim, A_r, &q_Ar);
        for (int m = 0; m < nv; ++m) {
            double x1, x4, x5;
            p_psi(dim, m, &pm);
            p_mul(&pm, &q_abl, &prod); p_upow(&prod, 1); x1 = p_expect(&prod, &M0, R_POS);
            p_mul(&pm, &q_abr, &prod); p_upow(&prod, 1); x1 += p_expect(&prod, &M0, R_NEG);
            p_mul(&pm, &q_al, &prod); p_upow(&prod, 1); x4 = gl.rho * p_expect(&prod, &Ml, R_POS);
            p_mul(&pm, &q_ar, &prod); p_upow(&prod, 1); x4 += gr.rho * p_expect(&prod, &Mr, R_NEG);
            p_mul(&pm, &q_Al, &prod); x5 = gl.rho * p_expect(&prod, &Ml, R_POS);
            p_mul(&pm, &q_Ar, &prod); x5 += gr.rho * p_expect(&prod, &Mr, R_NEG);
            for (int t = 0; t < ntan; ++t) {      /* the tangential slopes enter like the normal ones */
                x1 += og_tan_moment(dim, b_0[t], t, m, &M0, R_ALL, 0);
                x4 += gl.rho * og_tan_moment(dim, b_l[t], t, m, &Ml, R_POS, 0);
                x4 += gr.rho * og_tan_moment(dim, b_r[t], t, m, &Mr, R_NEG, 0);
            }
            r[m] = (kw.c1 * g0.rho * x1 + kw.c4 * x4 + kw.c5 * x5) / g0.rho;
        }
        if ((st = og_solve_moment_system(gas, &M0, r, Ab))) return st;
    }

    /* time-integrated distribution at the interface, term by term (Eq. resultingf) */
    static __thread og_term terms[16];
    int nt = 0;
#define ADD_TERM(W_, WH_, R_, POLYSET_) do { terms[nt].w = (W_); terms[nt].which = (WH_); \
        terms[nt].range = (R_); POLYSET_; ++nt; } while (0)
    ADD_TERM(g0.rho * kw.g[0], 0, R_ALL, p_const(&terms[nt].poly, 1.0));
    ADD_TERM(g0.rho * kw.g[1], 0, R_POS, (p_lin(dim, ab_l, &terms[nt].poly), p_upow(&terms[nt].poly, 1)));
    ADD_TERM(g0.rho * kw.g[1], 0, R_NEG, (p_lin(dim, ab_r, &terms[nt].poly), p_upow(&terms[nt].poly, 1)));
    ADD_TERM(g0.rho * kw.g[2], 0, R_ALL, p_lin(dim, Ab, &terms[nt].poly));
    ADD_TERM(gl.rho * kw.g[3], 1, R_POS, p_const(&terms[nt].poly, 1.0));
    ADD_TERM(gl.rho * kw.g[4], 1, R_POS, (p_lin(dim, a_l, &terms[nt].poly), p_upow(&terms[nt].poly, 1)));
    ADD_TERM(gl.rho * kw.g[5], 1, R_POS, p_lin(dim, A_l, &terms[nt].poly));
    ADD_TERM(gr.rho * kw.g[3], 2, R_NEG, p_const(&terms[nt].poly, 1.0));
    ADD_TERM(gr.rho * kw.g[4], 2, R_NEG, (p_lin(dim, a_r, &terms[nt].poly), p_upow(&terms[nt].poly, 1)));
    ADD_TERM(gr.rho * kw.g[5], 2, R_NEG, p_lin(dim, A_r, &terms[nt].poly));
    for (int t = 0; t < ntan; ++t) {   /* tangential slopes: as the normal ones, v_t in place of u */
        ADD_TERM(g0.rho * kw.g[1], 0, R_ALL, (p_lin(dim, b_0[t], &terms[nt].poly), p_tpow(&terms[nt].poly, t)));
        ADD_TERM(gl.rho * kw.g[4], 1, R_POS, (p_lin(dim, b_l[t], &terms[nt].poly), p_tpow(&terms[nt].poly, t)));
        ADD_TERM(gr.rho * kw.g[4], 2, R_NEG, (p_lin(dim, b_r[t], &terms[nt].poly), p_tpow(&terms[nt].poly, t)));
    }
#undef ADD_TERM
    const og_mom* Ms[3] = {&M0, &Ml, &Mr};

    /* flux F = int int u psi f (Eq. fluxesf) and G = int int psi f */
    for (int m = 0; m < nv; ++m) {
        double fsum = 0.0, gsum = 0.0;
        p_psi(dim, m, &pm);
        for (int t = 0; t < nt; ++t) {
            p_mul(&terms[t].poly, &pm, &prod);
            gsum += terms[t].w * p_expect(&prod, Ms[terms[t].which], terms[t].range);
            p_upow(&prod, 1);
            fsum += terms[t].w * p_expect(&prod, Ms[terms[t].which], terms[t].range);
        }
        F[m] = fsum;
        if (G) G[m] = gsum;
    }

    /* heat flux in the frame of U0: q = int int (u - U0) (|u - U0|^2 + xi^2)/2 f */
    {
        og_poly lin1, quad, P;
        lin1.n = 0; p_term(&lin1, 1.0, 1, 0, 0, 0); p_term(&lin1, -g0.U[0], 0, 0, 0, 0);
        quad.n = 0;
        p_term(&quad, 0.5, 2, 0, 0, 0); p_term(&quad, -g0.U[0], 1, 0, 0, 0); p_term(&quad, 0.5 * g0.U[0] * g0.U[0], 0, 0, 0, 0);
        p_term(&quad, 0.5, 0, 2, 0, 0); p_term(&quad, -g0.U[1], 0, 1, 0, 0); p_term(&quad, 0.5 * g0.U[1] * g0.U[1], 0, 0, 0, 0);
        if (dim == 3) {
            p_term(&quad, 0.5, 0, 0, 2, 0); p_term(&quad, -g0.U[2], 0, 0, 1, 0);
            p_term(&quad, 0.5 * g0.U[2] * g0.U[2], 0, 0, 0, 0);
        }
        p_term(&quad, 0.5, 0, 0, 0, 1);
        p_mul(&lin1, &quad, &P);
        double q = 0.0;
        for (int t = 0; t < nt; ++t) {
            p_mul(&terms[t].poly, &P, &tmp);
            q += terms[t].w * p_expect(&tmp, Ms[terms[t].which], terms[t].range);
        }
        if (qout) *qout = q;
        F[nv - 1] += (1.0 / gas->prandtl - 1.0) * q;
    }

    if (info) {
        const double* vecs[8] = {W0, a_l, a_r, A_l, A_r, ab_l, ab_r, Ab};
        for (int v = 0; v < 8; ++v)
            for (int m = 0; m < 5; ++m) info[5 * v + m] = (m < nv) ? vecs[v][m] : 0.0;
        info[40] = tau;
        for (int i = 0; i < 6; ++i) info[41 + i] = kw.g[i];
        info[47] = kw.c1; info[48] = kw.c4; info[49] = kw.c5;
        info[50] = eps_hat;
    }
    return OG_OK;
}

/* ------------------------------------------------------------------------ */
/* Grid, ghost cells, strain rate                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dim;
    long n[3];
    const double* xf[3];
    int bc[3][2];
    const double* bc_data[3][2];
    double gamma, prandtl, mu, c_a, c_mu, cfl, t_end;
    int eps_mode;      /* 0: eps = tau/dt; 1: eps = tau/tau_hat */
    int recon;         /* 0: second-order MUSCL (minmod); 1: third-order MUSCL (limited kappa = 1/3);
                          2: fifth-order WENO face values (minmod gradients) */
    int multi_d;       /* 1: multi-dimensional expansion (tangential slopes) */
} og_case;

typedef struct {
    const og_case* c;
    og_gas gas;
    int nv;
    long n[3], g[3], e[3];    /* interior cells, ghost width of the state, extended size per axis */
    long next;                /* extended cell count */
    double* xfe[3];           /* extended face coordinates, index i + 2 (i from -2 .. n+2) */
    double* xc[3];            /* extended centres, index i + 2 (two ghost layers) */
    double* dx[3];            /* extended widths, index i + 2 */
} og_grid;

static long gidx(const og_grid* gr, long i, long j, long k)
{
    return ((k + gr->g[2]) * gr->e[1] + (j + gr->g[1])) * gr->e[0] + (i + gr->g[0]);
}

static int og_grid_init(og_grid* gr, const og_case* c)
{
    memset(gr, 0, sizeof(*gr));
    gr->c = c;
    if (c->dim != 2 && c->dim != 3) return OG_ERR_ARG;
    if (!(c->gamma > 1.0)) return OG_ERR_ARG;
    gr->gas.dim = c->dim;
    gr->gas.b = 2.0 / (c->gamma - 1.0);
    gr->gas.K = gr->gas.b - c->dim;
    if (gr->gas.K < 0.0) return OG_ERR_ARG;
    gr->gas.gamma = c->gamma; gr->gas.prandtl = c->prandtl; gr->gas.mu = c->mu;
    gr->gas.c_a = c->c_a; gr->gas.c_mu = c->c_mu;
    if (c->eps_mode != 0 && c->eps_mode != 1) return OG_ERR_ARG;
    if (c->recon < 0 || c->recon > 2) return OG_ERR_ARG;
    if (c->multi_d != 0 && c->multi_d != 1) return OG_ERR_ARG;
    gr->gas.multi_d = c->multi_d;
    gr->gas.eps_mode = c->eps_mode;
    gr->nv = c->dim + 2;
    gr->next = 1;
    for (int d = 0; d < 3; ++d) {
        gr->n[d] = (d < c->dim) ? c->n[d] : 1;
        if (gr->n[d] < 1) return OG_ERR_ARG;
        /* the fifth-order stencil reaches a third cell beyond the boundary */
        gr->g[d] = (d < c->dim) ? (c->recon == 2 ? 3 : 2) : 0;
        if (d < c->dim && c->recon == 2 && gr->n[d] < 3) return OG_ERR_ARG;
        gr->e[d] = gr->n[d] + 2 * gr->g[d];
        gr->next *= gr->e[d];
    }
    for (int d = 0; d < c->dim; ++d) {
        long n = gr->n[d];
        if (n < 2) return OG_ERR_ARG;
        gr->xfe[d] = (double*)malloc(sizeof(double) * (n + 5));
        gr->xc[d] = (double*)malloc(sizeof(double) * (n + 4));
        gr->dx[d] = (double*)malloc(sizeof(double) * (n + 4));
        const double* xf = c->xf[d];
        for (long i = 0; i <= n; ++i) gr->xfe[d][i + 2] = xf[i];
        for (long m = 1; m <= 2; ++m) {
            if (c->bc[d][0] == OG_PERIODIC) gr->xfe[d][2 - m] = xf[0] - (xf[n] - xf[n - m]);
            else gr->xfe[d][2 - m] = 2.0 * xf[0] - xf[m];
            if (c->bc[d][1] == OG_PERIODIC) gr->xfe[d][n + 2 + m] = xf[n] + (xf[m] - xf[0]);
            else gr->xfe[d][n + 2 + m] = 2.0 * xf[n] - xf[n - m];
        }
        for (long i = 0; i < n + 4; ++i) {
            gr->xc[d][i] = 0.5 * (gr->xfe[d][i] + gr->xfe[d][i + 1]);
            gr->dx[d][i] = gr->xfe[d][i + 1] - gr->xfe[d][i];
            if (!(gr->dx[d][i] > 0.0)) return OG_ERR_ARG;
        }
        if ((c->bc[d][0] == OG_PERIODIC) != (c->bc[d][1] == OG_PERIODIC)) return OG_ERR_ARG;
    }
    return OG_OK;
}

static void og_grid_free(og_grid* gr)
{
    for (int d = 0; d < 3; ++d) { free(gr->xfe[d]); free(gr->xc[d]); free(gr->dx[d]); }
}

/* image of a (possibly ghost) index along one axis */
static long og_image(int bc, long i, long n, int side)
{
    if (side == 0) {
        if (bc == OG_PERIODIC) return i + n;
        if (bc == OG_WALL) return -1 - i;
        return 0;
    }
    if (bc == OG_PERIODIC) return i - n;
    if (bc == OG_WALL) return 2 * n - 1 - i;
    return n - 1;
}

static long og_clamp(long i, long n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

/* Fill the two ghost layers of W, axis by axis (x, then y over all x, then z over all x, y).
 * periodic: wrap; wall: mirror with momentum negated (no-slip, adiabatic); outflow: copy the
 * boundary cell; dirichlet: fixed state; profile: fixed state per boundary cell. */
static void og_fill_W(const og_grid* gr, const double* W, double* We)
{
    const og_case* c = gr->c;
    const int nv = gr->nv, dim = c->dim;
    const long N = gr->n[0] * gr->n[1] * gr->n[2];
    for (long k = 0; k < gr->n[2]; ++k)
        for (long j = 0; j < gr->n[1]; ++j)
            for (long i = 0; i < gr->n[0]; ++i) {
                long s = (k * gr->n[1] + j) * gr->n[0] + i;
                for (int m = 0; m < nv; ++m) We[m * gr->next + gidx(gr, i, j, k)] = W[m * N + s];
            }
    for (int d = 0; d < dim; ++d) {
        long lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            if (a < d) { lo[a] = -gr->g[a]; hi[a] = gr->n[a] + gr->g[a]; }
            else { lo[a] = 0; hi[a] = gr->n[a]; }
        }
        lo[d] = -gr->g[d]; hi[d] = gr->n[d] + gr->g[d];
        for (long k = lo[2]; k < hi[2]; ++k)
            for (long j = lo[1]; j < hi[1]; ++j)
                for (long i = lo[0]; i < hi[0]; ++i) {
                    long idx[3] = {i, j, k};
                    long id = idx[d];
                    if (id >= 0 && id < gr->n[d]) continue;
                    int side = id < 0 ? 0 : 1;
                    int bc = c->bc[d][side];
                    long src[3] = {i, j, k};
                    src[d] = og_image(bc, id, gr->n[d], side);
                    long gi = gidx(gr, i, j, k), si = gidx(gr, src[0], src[1], src[2]);
                    if (bc == OG_DIRICHLET) {
                        for (int m = 0; m < nv; ++m) We[m * gr->next + gi] = c->bc_data[d][side][m];
                    } else if (bc == OG_PROFILE) {
                        /* tangential cell index: remaining axes in increasing order */
                        long t = 0, stride = 1, ntan = 1;
                        for (int a = 0; a < dim; ++a) if (a != d) ntan *= gr->n[a];
                        for (int a = 0; a < dim; ++a) {
                            if (a == d) continue;
                            t += og_clamp(idx[a], gr->n[a]) * stride;
                            stride *= gr->n[a];
                        }
                        for (int m = 0; m < nv; ++m)
                            We[m * gr->next + gi] = c->bc_data[d][side][m * ntan + t];
                    } else {
                        for (int m = 0; m < nv; ++m) {
                            double v = We[m * gr->next + si];
                            if (bc == OG_WALL && m >= 1 && m <= dim) v = -v;
                            We[m * gr->next + gi] = v;
                        }
                    }
                }
    }
}

/* interior image of an extended cell (per-axis image for every ghost coordinate) */
static long og_image_cell(const og_grid* gr, long i, long j, long k)
{
    long idx[3] = {i, j, k};
    for (int d = 0; d < gr->c->dim; ++d) {
        if (idx[d] < 0) idx[d] = og_image(gr->c->bc[d][0], idx[d], gr->n[d], 0);
        else if (idx[d] >= gr->n[d]) idx[d] = og_image(gr->c->bc[d][1], idx[d], gr->n[d], 1);
        if (idx[d] < 0 || idx[d] >= gr->n[d]) idx[d] = og_clamp(idx[d], gr->n[d]);
    }
    return (idx[2] * gr->n[1] + idx[1]) * gr->n[0] + idx[0];
}

/* Strain-rate magnitude S = sqrt(2 S_ab S_ab), S_ab = (dU_a/dx_b + dU_b/dx_a)/2, with
 * central differences of the cell-averaged velocity over the neighbouring centres. */
/* Velocity gradient grad[a][b] = dU_a/dx_b of interior cell (i, j, k) by central
 * differences over the neighbouring centres (ghost-filled state We). */
static void og_velocity_gradient(const og_grid* gr, const double* We, long i, long j, long k,
                                 double grad[3][3])
{
    const int dim = gr->c->dim;
    long c0[3] = {i, j, k};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) grad[a][b] = 0.0;
    for (int b = 0; b < dim; ++b) {       /* derivative direction */
        long cp[3] = {i, j, k}, cm[3] = {i, j, k};
        cp[b] += 1; cm[b] -= 1;
        long ip = gidx(gr, cp[0], cp[1], cp[2]), im = gidx(gr, cm[0], cm[1], cm[2]);
        double h = gr->xc[b][c0[b] + 1 + 2] - gr->xc[b][c0[b] - 1 + 2];
        for (int a = 0; a < dim; ++a) {   /* velocity component */
            double up = We[(1 + a) * gr->next + ip] / We[ip];
            double um = We[(1 + a) * gr->next + im] / We[im];
            grad[a][b] = (up - um) / h;
        }
    }
}

/* S^2 = 2 S_ab S_ab with S_ab the symmetric part of the velocity gradient. */
static double og_strain_sq(int dim, const double grad[3][3])
{
    double ss = 0.0;
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
            double sab = 0.5 * (grad[a][b] + grad[b][a]);
            ss += sab * sab;
        }
    return 2.0 * ss;
}

static void og_strain(const og_grid* gr, const double* We, double* S)
{
    const long N = gr->n[0] * gr->n[1] * gr->n[2];
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        long i = s % gr->n[0], j = (s / gr->n[0]) % gr->n[1], k = s / (gr->n[0] * gr->n[1]);
        double grad[3][3];
        og_velocity_gradient(gr, We, i, j, k, grad);
        S[s] = sqrt(og_strain_sq(gr->c->dim, grad));
    }
}

static double og_minmod(double p, double q)
{
    if (p * q <= 0.0) return 0.0;
    return (p > 0.0 ? 1.0 : -1.0) * fmin(fabs(p), fabs(q));
}

/* Limited kappa-scheme (van Leer's MUSCL family) with kappa = 1/3, the third-order member:
 * the slope towards the face of a cell whose one-sided slopes are `away` (across the far
 * face) and `toward` (across this face) is
 *   (1 - kappa)/2 minmod(away, b toward) + (1 + kappa)/2 minmod(toward, b away),
 * b = (3 - kappa)/(1 - kappa) = 4.  On a uniform grid the face value W_i + slope dx/2 is
 * exact for the cell averages of a quadratic where neither limiter acts, and it stays
 * between the averages of the two cells sharing the face (no new extremum). */
static double og_muscl3(double away, double toward)
{
    const double kappa = 1.0 / 3.0, b = (3.0 - kappa) / (1.0 - kappa);
    return 0.5 * (1.0 - kappa) * og_minmod(away, b * toward) + 0.5 * (1.0 + kappa) * og_minmod(toward, b * away);
}

/* Fifth-order WENO value (Jiang and Shu's weighted ENO, 1996) at the face between cells
 * c and d of five consecutive cell averages a, b, c, d, e, the upwind side being a..c:
 * the three third-order candidates of the stencils {a,b,c}, {b,c,d}, {c,d,e}, each the
 * face value of the parabola with those cell averages, weighted by
 *   alpha_k = d_k / (eps + beta_k)^2,  (d_0, d_1, d_2) = (1/10, 6/10, 3/10),  eps = 1e-6,
 * beta_k the smoothness indicator of candidate k: the sum over its first and second
 * derivatives of dx^(2l-1) times the integral of the squared l-th derivative over cell c.
 * With all beta_k equal the weights are the linear ones, which combine the candidates
 * into the fifth-order upwind interpolation.  Index space: the cell widths do not enter. */
static double og_weno5(double a, double b, double c, double d, double e)
{
    const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    const double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    const double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
    const double s0 = a - 2.0 * b + c, t0 = a - 4.0 * b + 3.0 * c;
    const double s1 = b - 2.0 * c + d, t1 = b - d;
    const double s2 = c - 2.0 * d + e, t2 = 3.0 * c - 4.0 * d + e;
    const double beta0 = 13.0 / 12.0 * s0 * s0 + 0.25 * t0 * t0;
    const double beta1 = 13.0 / 12.0 * s1 * s1 + 0.25 * t1 * t1;
    const double beta2 = 13.0 / 12.0 * s2 * s2 + 0.25 * t2 * t2;
    const double eps = 1e-6;
    const double al0 = 0.1 / ((eps + beta0) * (eps + beta0));
    const double al1 = 0.6 / ((eps + beta1) * (eps + beta1));
    const double al2 = 0.3 / ((eps + beta2) * (eps + beta2));
    return (al0 * q0 + al1 * q1 + al2 * q2) / (al0 + al1 + al2);
}

/* One component along a face normal: cell values w[0..3] (cells i-1, i, i+1, i+2) with
 * centres xc[0..3], face at xf between cells i and i+1; for recon 2 also w[-1] and w[4]
 * (cells i-2, i+3).  Gradients sl, sr: minmod of the one-sided slopes on centre
 * distances (every scheme); face values wl, wr from those (recon 0), from the limited
 * kappa = 1/3 slopes (recon 1), or the fifth-order WENO values of cells i-2 .. i+2 and,
 * mirrored, i+3 .. i-1 (recon 2). */
static void og_reconstruct(int recon, const double* w, const double* xc, double xf, double* wl, double* wr,
                           double* sl, double* sr)
{
    const double d0 = (w[1] - w[0]) / (xc[1] - xc[0]);
    const double d1 = (w[2] - w[1]) / (xc[2] - xc[1]);
    const double d2 = (w[3] - w[2]) / (xc[3] - xc[2]);
    *sl = og_minmod(d0, d1);
    *sr = og_minmod(d1, d2);
    if (recon == 2) {
        *wl = og_weno5(w[-1], w[0], w[1], w[2], w[3]);
        *wr = og_weno5(w[4], w[3], w[2], w[1], w[0]);
    } else if (recon == 1) {
        *wl = w[1] + og_muscl3(d0, d1) * (xf - xc[1]);
        *wr = w[2] - og_muscl3(d2, d1) * (xc[2] - xf);
    } else {
        *wl = w[1] + *sl * (xf - xc[1]);
        *wr = w[2] - *sr * (xc[2] - xf);
    }
}

/* local rate  sum_d (|U_d| + c)/dx_d + 2 nu_eff sum_d 1/dx_d^2,
 * nu_eff = (mu + rho k/omega)/rho * max(4/3, gamma/Pr);  dt = CFL / max rate */
static int og_max_rate(const og_grid* gr, const double* W, const double* kk, const double* om,
                       double* rate_out)
{
    const og_case* c = gr->c;
    const int dim = c->dim, nv = gr->nv;
    const long N = gr->n[0] * gr->n[1] * gr->n[2];
    const double fac = fmax(4.0 / 3.0, c->gamma / c->prandtl);
    double mx = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : mx) reduction(| : bad)
    for (long s = 0; s < N; ++s) {
        long idx[3] = {s % gr->n[0], (s / gr->n[0]) % gr->n[1], s / (gr->n[0] * gr->n[1])};
        double w[5];
        for (int m = 0; m < nv; ++m) w[m] = W[m * N + s];
        og_maxw g;
        if (og_prim(&gr->gas, w, &g)) { bad = 1; continue; }
        double p = g.rho / (2.0 * g.lam);
        double cs = sqrt(c->gamma * p / g.rho);
        double nu = (c->mu + g.rho * kk[s] / om[s]) / g.rho * fac;
        double r = 0.0, r2 = 0.0;
        for (int d = 0; d < dim; ++d) {
            double h = gr->dx[d][idx[d] + 2];
            r += (fabs(g.U[d]) + cs) / h;
            r2 += 1.0 / (h * h);
        }
        r += 2.0 * nu * r2;
        if (r > mx) mx = r;
    }
    *rate_out = mx;
    return bad ? OG_ERR_NONPHYSICAL : OG_OK;
}

/* Flux through one face.  axis d; (fi, fj, fk) are face coordinates (the face lies on the low
 * side of cell (fi, fj, fk) along d).  Fout in global component order.  diag_out (or NULL):
 * the face's eps_hat = tau/tau_hat and its relaxation time tau. */
static int og_face_at(const og_grid* gr, const double* We, const double* kk, const double* om,
                      const double* S, int d, long fi, long fj, long fk, double dt, double* Fout,
                      double* diag_out)
{
    const int dim = gr->c->dim, nv = gr->nv;
    long base[3] = {fi, fj, fk};
    /* cells base-3 .. base+2 along d (the outer two for the fifth-order stencil only) */
    double Wx[6][5];
    double xcs[4];
    const int wide = gr->c->recon == 2;
    for (int o = -1; o < 5; ++o) {
        if (!wide && (o < 0 || o > 3)) continue;
        long cc[3] = {base[0], base[1], base[2]};
        cc[d] += o - 2;
        long gi = gidx(gr, cc[0], cc[1], cc[2]);
        for (int m = 0; m < nv; ++m) Wx[o + 1][m] = We[m * gr->next + gi];
        if (o >= 0 && o <= 3) xcs[o] = gr->xc[d][cc[d] + 2];
    }
    double (*Wc)[5] = Wx + 1;                        /* Wc[o]: cell base-2+o */
    const double xface = gr->xfe[d][base[d] + 2];
    /* minmod slopes of the conservative variables on centre-to-centre distances; the face
       values from them (second order) or from the limited kappa = 1/3 combination of the
       two one-sided slopes (third-order MUSCL) */
    double sL[5], sR[5], WL[5], WR[5];
    for (int m = 0; m < nv; ++m) {
        double w[6] = {0.0, Wc[0][m], Wc[1][m], Wc[2][m], Wc[3][m], 0.0};
        if (wide) { w[0] = Wx[0][m]; w[5] = Wx[5][m]; }
        og_reconstruct(gr->c->recon, w + 1, xcs, xface, &WL[m], &WR[m], &sL[m], &sR[m]);
    }
    /* rotate to the face-local frame: normal first, then remaining axes in order */
    int perm[3];
    perm[0] = d;
    for (int a = 0, t = 1; a < dim; ++a) if (a != d) perm[t++] = a;
    double lWL[5], lWR[5], lsL[5], lsR[5], lWi[5], lWi1[5];
    for (int m = 0; m < nv; ++m) {
        int src = (m >= 1 && m <= dim) ? 1 + perm[m - 1] : m;
        lWL[m] = WL[src]; lWR[m] = WR[src]; lsL[m] = sL[src]; lsR[m] = sR[src];
        lWi[m] = Wc[1][src]; lWi1[m] = Wc[2][src];
    }
    long cl[3] = {fi, fj, fk}, cr[3] = {fi, fj, fk};
    cl[d] -= 1;
    /* tangential gradients of the two cells (multi-dimensional expansion): minmod of the
       one-sided differences along each tangential axis on centre distances, from the
       ghost-filled state (a cell beyond the boundary along the normal takes its ghost
       neighbours, corners filled axis by axis as everywhere) */
    double tsl[10] = {0}, tsr[10] = {0};
    if (gr->gas.multi_d) {
        for (int t = 1; t < dim; ++t) {
            const int a = perm[t];
            for (int side = 0; side < 2; ++side) {
                const long* c = side ? cr : cl;
                double* out = side ? tsr : tsl;
                long cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
                cp[a] += 1; cm[a] -= 1;
                const long i0 = gidx(gr, c[0], c[1], c[2]);
                const long ip = gidx(gr, cp[0], cp[1], cp[2]), im = gidx(gr, cm[0], cm[1], cm[2]);
                const double hp = gr->xc[a][c[a] + 1 + 2] - gr->xc[a][c[a] + 2];
                const double hm = gr->xc[a][c[a] + 2] - gr->xc[a][c[a] - 1 + 2];
                for (int m = 0; m < nv; ++m) {
                    const int src = (m >= 1 && m <= dim) ? 1 + perm[m - 1] : m;
                    const double dp = (We[src * gr->next + ip] - We[src * gr->next + i0]) / hp;
                    const double dm = (We[src * gr->next + i0] - We[src * gr->next + im]) / hm;
                    out[(t - 1) * 5 + m] = og_minmod(dm, dp);
                }
            }
        }
    }
    long il = og_image_cell(gr, cl[0], cl[1], cl[2]), ir = og_image_cell(gr, cr[0], cr[1], cr[2]);
    double kf = 0.5 * (kk[il] + kk[ir]);
    double wf = 0.5 * (om[il] + om[ir]);
    double Sf = 0.5 * (S[il] + S[ir]);
    double F[5], info[OG_INFO_LEN];
    int st = og_face(&gr->gas, lWL, lWR, lsL, lsR, tsl, tsr, lWi, lWi1, xface - xcs[1], xcs[2] - xface,
                     kf, wf, Sf, dt, F, NULL, NULL, diag_out ? info : NULL);
    if (st) return st;
    if (diag_out) {
        diag_out[0] = info[50];
        diag_out[1] = info[40];
    }
    for (int m = 0; m < nv; ++m) {
        int dst = (m >= 1 && m <= dim) ? 1 + perm[m - 1] : m;
        Fout[dst] = F[m];
    }
    return OG_OK;
}

/* Net time-integrated flux out of cell idx per unit volume, component m of the face
 * arrays F[d] (component-major, fn[d] faces along each axis). */
static double og_flux_out(const og_grid* gr, double* const F[3], const long fn[3][3], int m, const long idx[3])
{
    double acc = 0.0;
    for (int d = 0; d < gr->c->dim; ++d) {
        long nf = fn[d][0] * fn[d][1] * fn[d][2];
        long lo = (idx[2] * fn[d][1] + idx[1]) * fn[d][0] + idx[0];
        long hi = lo + (d == 0 ? 1 : (d == 1 ? fn[d][0] : fn[d][0] * fn[d][1]));
        acc += (F[d][m * nf + hi] - F[d][m * nf + lo]) / gr->dx[d][idx[d] + 2];
    }
    return acc;
}

/* Conservative update of the flow variables of every cell: Wn = W - flux out. */
static void og_update(const og_grid* gr, const double* W, double* const F[3], const long fn[3][3], double* Wn)
{
    const long N = gr->n[0] * gr->n[1] * gr->n[2];
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        long idx[3] = {s % gr->n[0], (s / gr->n[0]) % gr->n[1], s / (gr->n[0] * gr->n[1])};
        for (int m = 0; m < gr->nv; ++m) Wn[m * N + s] = W[m * N + s] - og_flux_out(gr, F, fn, m, idx);
    }
}

/* One explicit step W -> Wn with step dt.  All faces, then the conservative update. */
static int og_step(const og_grid* gr, const double* W, const double* kk, const double* om,
                   double dt, double* Wn, double* We, double* S)
{
    const int dim = gr->c->dim, nv = gr->nv;
    og_fill_W(gr, W, We);
    og_strain(gr, We, S);
    double* F[3] = {NULL, NULL, NULL};
    long fn[3][3];
    int bad = 0;
    for (int d = 0; d < dim; ++d) {
        for (int a = 0; a < 3; ++a) fn[d][a] = gr->n[a] + (a == d ? 1 : 0);
        long nf = fn[d][0] * fn[d][1] * fn[d][2];
        F[d] = (double*)malloc(sizeof(double) * nv * nf);
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
        for (long f = 0; f < nf; ++f) {
            long fi = f % fn[d][0], fj = (f / fn[d][0]) % fn[d][1], fk = f / (fn[d][0] * fn[d][1]);
            double Fl[5];
            if (og_face_at(gr, We, kk, om, S, d, fi, fj, fk, dt, Fl, NULL)) { bad = 1; continue; }
            for (int m = 0; m < nv; ++m) F[d][m * nf + f] = Fl[m];
        }
    }
    if (!bad) og_update(gr, W, F, fn, Wn);
    for (int d = 0; d < dim; ++d) free(F[d]);
    return bad ? OG_ERR_NONPHYSICAL : OG_OK;
}

static int og_check_fields(const og_grid* gr, const double* W, const double* kk, const double* om)
{
    const long N = gr->n[0] * gr->n[1] * gr->n[2];
    for (long s = 0; s < N; ++s) {
        double w[5];
        og_maxw g;
        for (int m = 0; m < gr->nv; ++m) w[m] = W[m * N + s];
        if (og_prim(&gr->gas, w, &g)) return OG_ERR_NONPHYSICAL;
        if (!(kk[s] >= 0.0) || !isfinite(kk[s]) || !(om[s] > 0.0) || !isfinite(om[s])) return OG_ERR_ARG;
    }
    return OG_OK;
}

/* ------------------------------------------------------------------------ */
/* k-omega transport                                                         */
/* ------------------------------------------------------------------------ */
/* constants of the Wilcox (2006) k-omega model */
#define KW_ALPHA (13.0 / 25.0)
#define KW_BETA 0.0708
#define KW_BETA_STAR 0.09
#define KW_SIGMA 0.5
#define KW_SIGMA_STAR 0.6
#define KW_SIGMA_DO 0.125

/* value of a cell field at a (possibly ghost) cell: its interior image's value */
static double og_kw_at(const og_grid* gr, const double* f, const long* c)
{
    return f[og_image_cell(gr, c[0], c[1], c[2])];
}

/* Explicit sources of one interior cell s at the state We (ghost-filled) and fields k, om:
 *   Qk = P,  Qw = alpha (omega/k) P + sigma_d (rho/omega) grad k . grad omega,
 *   P = mu_t (S^2 - 2/3 div^2) - 2/3 rho k div,  mu_t = rho k/(omega sqrt(1+eta^2)),
 *   S^2 = 2 S_ab S_ab,  eta = S/(C_mu omega),  sigma_d = sigma_do where grad k.grad omega > 0.
 * alpha (omega/k) P is written as alpha rho ((S^2 - 2/3 div^2)/sqrt(1+eta^2) - 2/3 omega div),
 * which is the same quantity without the division by k.  Central differences over the
 * neighbouring centres, as for the strain rate. */
static void og_kw_source_cell(const og_grid* gr, const double* We, const double* kk, const double* om,
                              long s, double* Qk, double* Qw)
{
    const int dim = gr->c->dim;
    long i = s % gr->n[0], j = (s / gr->n[0]) % gr->n[1], k = s / (gr->n[0] * gr->n[1]);
    long c0[3] = {i, j, k};
    double grad[3][3], gk[3] = {0}, gw[3] = {0};
    og_velocity_gradient(gr, We, i, j, k, grad);
    for (int b = 0; b < dim; ++b) {
        long cp[3] = {i, j, k}, cm[3] = {i, j, k};
        cp[b] += 1; cm[b] -= 1;
        double h = gr->xc[b][c0[b] + 1 + 2] - gr->xc[b][c0[b] - 1 + 2];
        gk[b] = (og_kw_at(gr, kk, cp) - og_kw_at(gr, kk, cm)) / h;
        gw[b] = (og_kw_at(gr, om, cp) - og_kw_at(gr, om, cm)) / h;
    }
    const double s2 = og_strain_sq(dim, grad);
    double div = 0.0, cross = 0.0;
    for (int a = 0; a < dim; ++a) {
        div += grad[a][a];
        cross += gk[a] * gw[a];
    }
    const double rho = We[gidx(gr, i, j, k)];
    const double kc = kk[s], wc = om[s];
    const double eta = sqrt(s2) / (gr->c->c_mu * wc);
    const double root = sqrt(1.0 + eta * eta);
    const double mut = rho * kc / (wc * root);
    const double shear = s2 - 2.0 / 3.0 * div * div;
    *Qk = mut * shear - 2.0 / 3.0 * rho * kc * div;
    *Qw = KW_ALPHA * rho * (shear / root - 2.0 / 3.0 * wc * div);
    if (cross > 0.0) *Qw += KW_SIGMA_DO * rho / wc * cross;
}

/* Time-integrated fluxes of rho k and rho omega through one face (axis d, face coordinates
 * as in og_face_at), given the face's time-integrated mass flux Frho.  W: interior state;
 * a ghost cell's density, k and omega (so its eddy viscosity) are its interior image's. */
static void og_kw_face(const og_grid* gr, const double* W, const double* kk, const double* om, int d,
                       long fi, long fj, long fk, double Frho, double dt, double* Fk, double* Fw)
{
    long cl[3] = {fi, fj, fk}, cr[3] = {fi, fj, fk};
    cl[d] -= 1;
    const double kl = og_kw_at(gr, kk, cl), kr = og_kw_at(gr, kk, cr);
    const double wl = og_kw_at(gr, om, cl), wr = og_kw_at(gr, om, cr);
    const double rl = og_kw_at(gr, W, cl), rr = og_kw_at(gr, W, cr);
    const double nut = 0.5 * (rl * kl / wl + rr * kr / wr);
    const double dn = gr->xc[d][cr[d] + 2] - gr->xc[d][cl[d] + 2];
    const double mu = gr->c->mu;
    *Fk = Frho * (Frho >= 0.0 ? kl : kr) - dt * (mu + KW_SIGMA_STAR * nut) * (kr - kl) / dn;
    *Fw = Frho * (Frho >= 0.0 ? wl : wr) - dt * (mu + KW_SIGMA * nut) * (wr - wl) / dn;
}

/* One explicit step of the flow and of rho k, rho omega (rk, rw: conservative, in/out via
 * rkn, rwn).  kk, om are rk/rho, rw/rho of the current state. */
static int og_step_kw(const og_grid* gr, const double* W, const double* kk, const double* om,
                      const double* rk, const double* rw, double dt, double* Wn, double* rkn, double* rwn,
                      double* We, double* S)
{
    const int dim = gr->c->dim, nv = gr->nv;
    const long N = gr->n[0] * gr->n[1] * gr->n[2];
    og_fill_W(gr, W, We);
    og_strain(gr, We, S);
    double* F[3] = {NULL, NULL, NULL};
    double* Fk[3] = {NULL, NULL, NULL};
    double* Fw[3] = {NULL, NULL, NULL};
    long fn[3][3];
    int bad = 0;
    for (int d = 0; d < dim; ++d) {
        for (int a = 0; a < 3; ++a) fn[d][a] = gr->n[a] + (a == d ? 1 : 0);
        long nf = fn[d][0] * fn[d][1] * fn[d][2];
        F[d] = (double*)malloc(sizeof(double) * nv * nf);
        Fk[d] = (double*)malloc(sizeof(double) * nf);
        Fw[d] = (double*)malloc(sizeof(double) * nf);
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
        for (long f = 0; f < nf; ++f) {
            long fi = f % fn[d][0], fj = (f / fn[d][0]) % fn[d][1], fk = f / (fn[d][0] * fn[d][1]);
            double Fl[5];
            if (og_face_at(gr, We, kk, om, S, d, fi, fj, fk, dt, Fl, NULL)) { bad = 1; continue; }
            for (int m = 0; m < nv; ++m) F[d][m * nf + f] = Fl[m];
            og_kw_face(gr, W, kk, om, d, fi, fj, fk, Fl[0], dt, &Fk[d][f], &Fw[d][f]);
        }
    }
    if (!bad) {
        og_update(gr, W, F, fn, Wn);
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (long s = 0; s < N; ++s) {
            long idx[3] = {s % gr->n[0], (s / gr->n[0]) % gr->n[1], s / (gr->n[0] * gr->n[1])};
            double ak = rk[s] - og_flux_out(gr, Fk, fn, 0, idx);
            double aw = rw[s] - og_flux_out(gr, Fw, fn, 0, idx);
            double Qk, Qw;
            og_kw_source_cell(gr, We, kk, om, s, &Qk, &Qw);
            rkn[s] = (ak + dt * Qk) / (1.0 + dt * KW_BETA_STAR * om[s]);
            rwn[s] = (aw + dt * Qw) / (1.0 + dt * KW_BETA * om[s]);
            if (!(rkn[s] >= 0.0) || !(rwn[s] > 0.0) || !isfinite(rkn[s]) || !isfinite(rwn[s])) bad = 1;
        }
    }
    for (int d = 0; d < dim; ++d) { free(F[d]); free(Fk[d]); free(Fw[d]); }
    return bad ? OG_ERR_NONPHYSICAL : OG_OK;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (ctypes)                                           */
/* ------------------------------------------------------------------------ */
static void og_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Run nsteps explicit steps in place.  t_io: time in/out.  Returns the residual of the last
 * step, the last dt and the steps taken.  Steps stop once t reaches t_end (t_end > 0). */
int og_run(const og_case* c, double* W, const double* kk, const double* om, int nsteps,
           int nthreads, double* res, double* dt_last, double* t_io, long* steps_done)
{
    og_grid gr;
    int st = og_grid_init(&gr, c);
    if (st) { og_grid_free(&gr); return st; }
    og_threads(nthreads);
    const long N = gr.n[0] * gr.n[1] * gr.n[2];
    const int nv = gr.nv;
    if ((st = og_check_fields(&gr, W, kk, om))) { og_grid_free(&gr); return st; }
    double* We = (double*)malloc(sizeof(double) * nv * gr.next);
    double* S = (double*)malloc(sizeof(double) * N);
    double* Wn = (double*)malloc(sizeof(double) * nv * N);
    double t = t_io ? *t_io : 0.0;
    long done = 0;
    for (int step = 0; step < nsteps; ++step) {
        if (c->t_end > 0.0 && t >= c->t_end) break;
        double rate;
        if ((st = og_max_rate(&gr, W, kk, om, &rate))) break;
        double dt = c->cfl / rate, tn = t + dt;
        if (c->t_end > 0.0 && tn >= c->t_end) { dt = c->t_end - t; tn = c->t_end; }
        if ((st = og_step(&gr, W, kk, om, dt, Wn, We, S))) break;
        for (int m = 0; m < nv; ++m) {
            double acc = 0.0;
            for (long s = 0; s < N; ++s) {
                double r = (Wn[m * N + s] - W[m * N + s]) / dt;
                acc += r * r;
            }
            if (res) res[m] = sqrt(acc / (double)N);
        }
        memcpy(W, Wn, sizeof(double) * nv * N);
        if (dt_last) *dt_last = dt;
        t = tn;
        ++done;
        if ((st = og_check_fields(&gr, W, kk, om))) break;
    }
    if (t_io) *t_io = t;
    if (steps_done) *steps_done = done;
    free(We); free(S); free(Wn);
    og_grid_free(&gr);
    return st;
}

/* og_run with k and omega transported (in/out) instead of frozen.  The residual covers the
 * flow variables. */
int og_run_kw(const og_case* c, double* W, double* kk, double* om, int nsteps, int nthreads,
              double* res, double* dt_last, double* t_io, long* steps_done)
{
    og_grid gr;
    int st = og_grid_init(&gr, c);
    if (st) { og_grid_free(&gr); return st; }
    og_threads(nthreads);
    const long N = gr.n[0] * gr.n[1] * gr.n[2];
    const int nv = gr.nv;
    if ((st = og_check_fields(&gr, W, kk, om))) { og_grid_free(&gr); return st; }
    double* We = (double*)malloc(sizeof(double) * nv * gr.next);
    double* S = (double*)malloc(sizeof(double) * N);
    double* Wn = (double*)malloc(sizeof(double) * nv * N);
    double* rk = (double*)malloc(sizeof(double) * N);
    double* rw = (double*)malloc(sizeof(double) * N);
    double* rkn = (double*)malloc(sizeof(double) * N);
    double* rwn = (double*)malloc(sizeof(double) * N);
    for (long s = 0; s < N; ++s) { rk[s] = W[s] * kk[s]; rw[s] = W[s] * om[s]; }
    double t = t_io ? *t_io : 0.0;
    long done = 0;
    for (int step = 0; step < nsteps; ++step) {
        if (c->t_end > 0.0 && t >= c->t_end) break;
        double rate;
        if ((st = og_max_rate(&gr, W, kk, om, &rate))) break;
        double dt = c->cfl / rate, tn = t + dt;
        if (c->t_end > 0.0 && tn >= c->t_end) { dt = c->t_end - t; tn = c->t_end; }
        if ((st = og_step_kw(&gr, W, kk, om, rk, rw, dt, Wn, rkn, rwn, We, S))) break;
        for (int m = 0; m < nv; ++m) {
            double acc = 0.0;
            for (long s = 0; s < N; ++s) {
                double r = (Wn[m * N + s] - W[m * N + s]) / dt;
                acc += r * r;
            }
            if (res) res[m] = sqrt(acc / (double)N);
        }
        memcpy(W, Wn, sizeof(double) * nv * N);
        memcpy(rk, rkn, sizeof(double) * N);
        memcpy(rw, rwn, sizeof(double) * N);
        for (long s = 0; s < N; ++s) { kk[s] = rk[s] / W[s]; om[s] = rw[s] / W[s]; }
        if (dt_last) *dt_last = dt;
        t = tn;
        ++done;
        if ((st = og_check_fields(&gr, W, kk, om))) break;
    }
    if (t_io) *t_io = t;
    if (steps_done) *steps_done = done;
    free(We); free(S); free(Wn); free(rk); free(rw); free(rkn); free(rwn);
    og_grid_free(&gr);
    return st;
}

/* Explicit k-omega sources Qk, Qw of every interior cell at state W and fields k, omega. */
int og_kw_sources(const og_case* c, const double* W, const double* kk, const double* om, double* Qk, double* Qw)
{
    og_grid gr;
    int st = og_grid_init(&gr, c);
    if (!st) {
        const long N = gr.n[0] * gr.n[1] * gr.n[2];
        double* We = (double*)malloc(sizeof(double) * gr.nv * gr.next);
        og_fill_W(&gr, W, We);
        for (long s = 0; s < N; ++s) og_kw_source_cell(&gr, We, kk, om, s, &Qk[s], &Qw[s]);
        free(We);
    }
    og_grid_free(&gr);
    return st;
}

/* CFL time step of a state (before any end-time clipping). */
int og_dt(const og_case* c, const double* W, const double* kk, const double* om, double* dt)
{
    og_grid gr;
    int st = og_grid_init(&gr, c);
    if (!st) {
        double rate;
        st = og_max_rate(&gr, W, kk, om, &rate);
        if (!st) *dt = c->cfl / rate;
    }
    og_grid_free(&gr);
    return st;
}

/* Strain-rate magnitude of every interior cell. */
int og_strain_field(const og_case* c, const double* W, double* S)
{
    og_grid gr;
    int st = og_grid_init(&gr, c);
    if (!st) {
        double* We = (double*)malloc(sizeof(double) * gr.nv * gr.next);
        og_fill_W(&gr, W, We);
        og_strain(&gr, We, S);
        free(We);
    }
    og_grid_free(&gr);
    return st;
}

/* Ghost-extended copy of W (nv x extended cells), for inspection. */
int og_ghost_fill(const og_case* c, const double* W, double* We)
{
    og_grid gr;
    int st = og_grid_init(&gr, c);
    if (!st) og_fill_W(&gr, W, We);
    og_grid_free(&gr);
    return st;
}

/* New values of selected cells after one step of size dt from W (the rest of the grid is
 * only read).  out: ncells x nv, cell-major. */
int og_step_cells(const og_case* c, const double* W, const double* kk, const double* om, double dt,
                  const long* cells, long ncells, int nthreads, double* out)
{
    og_grid gr;
    int st = og_grid_init(&gr, c);
    if (st) { og_grid_free(&gr); return st; }
    og_threads(nthreads);
    const long N = gr.n[0] * gr.n[1] * gr.n[2];
    const int nv = gr.nv, dim = c->dim;
    double* We = (double*)malloc(sizeof(double) * nv * gr.next);
    double* S = (double*)malloc(sizeof(double) * N);
    og_fill_W(&gr, W, We);
    og_strain(&gr, We, S);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (long q = 0; q < ncells; ++q) {
        long s = cells[q];
        long idx[3] = {s % gr.n[0], (s / gr.n[0]) % gr.n[1], s / (gr.n[0] * gr.n[1])};
        double acc[5];
        for (int m = 0; m < nv; ++m) acc[m] = W[m * N + s];
        for (int d = 0; d < dim; ++d) {
            double Flo[5], Fhi[5];
            long hi[3] = {idx[0], idx[1], idx[2]};
            hi[d] += 1;
            if (og_face_at(&gr, We, kk, om, S, d, idx[0], idx[1], idx[2], dt, Flo, NULL) ||
                og_face_at(&gr, We, kk, om, S, d, hi[0], hi[1], hi[2], dt, Fhi, NULL)) { bad = 1; continue; }
            for (int m = 0; m < nv; ++m) acc[m] -= (Fhi[m] - Flo[m]) / gr.dx[d][idx[d] + 2];
        }
        for (int m = 0; m < nv; ++m) out[q * nv + m] = acc[m];
    }
    free(We); free(S);
    og_grid_free(&gr);
    return bad ? OG_ERR_NONPHYSICAL : OG_OK;
}

/* Single interface in the face-local frame.  params: gamma, prandtl, mu, c_a, c_mu, eps_mode.
 * tsl, tsr: tangential gradients [(dim - 1) x 5] (multi-dimensional expansion) or NULL.
 * F, G: nv values; q: heat flux; info: OG_INFO_LEN values (see og_face). */
int og_face_flux(int dim, const double* params, const double* Wl, const double* Wr,
                 const double* sl, const double* sr, const double* tsl, const double* tsr,
                 const double* Wi, const double* Wi1,
                 double dxl, double dxr, double kf, double wf, double Sf, double dt,
                 double* F, double* G, double* q, double* info)
{
    og_gas gas;
    if (dim != 2 && dim != 3) return OG_ERR_ARG;
    gas.dim = dim; gas.gamma = params[0]; gas.prandtl = params[1]; gas.mu = params[2];
    gas.c_a = params[3]; gas.c_mu = params[4]; gas.eps_mode = params[5] != 0.0;
    gas.multi_d = tsl && tsr;
    gas.b = 2.0 / (gas.gamma - 1.0); gas.K = gas.b - dim;
    return og_face(&gas, Wl, Wr, sl, sr, tsl, tsr, Wi, Wi1, dxl, dxr, kf, wf, Sf, dt, F, G, q, info);
}

/* Moments <u^n> (n < OG_NU) of one Maxwellian for the three u ranges; out: 3*OG_NU values. */
int og_moments_u(double U, double lam, double* out)
{
    og_gas gas; og_maxw g; og_mom M;
    memset(&gas, 0, sizeof(gas)); gas.dim = 2; gas.K = 0.0;
    g.rho = 1.0; g.U[0] = U; g.U[1] = g.U[2] = 0.0; g.lam = lam;
    og_moments(&gas, &g, &M);
    for (int r = 0; r < 3; ++r)
        for (int n = 0; n < OG_NU; ++n) out[r * OG_NU + n] = M.u[r][n];
    return OG_OK;
}

/* gam0..gam5, c1, c4, c5 for (tau, dt). */
int og_kogan(double tau, double dt, double* out)
{
    og_tw k;
    og_kogan_weights(tau, dt, &k);
    for (int i = 0; i < 6; ++i) out[i] = k.g[i];
    out[6] = k.c1; out[7] = k.c4; out[8] = k.c5;
    return OG_OK;
}

/* Reconstruction of one component at one face (og_reconstruct): out = wl, wr, sl, sr.
 * w holds cells i-1 .. i+2 (recon 0, 1) or i-2 .. i+3 (recon 2); xc the centres of cells
 * i-1 .. i+2. */
int og_recon(int recon, const double* w, const double* xc, double xf, double* out)
{
    if (recon < 0 || recon > 2) return OG_ERR_ARG;
    og_reconstruct(recon, recon == 2 ? w + 1 : w, xc, xf, &out[0], &out[1], &out[2], &out[3]);
    return OG_OK;
}

/* Fifth-order WENO face value of five cell averages (og_weno5). */
double og_weno5_value(const double* v) { return og_weno5(v[0], v[1], v[2], v[3], v[4]); }

/* gam0..gam5, c1, c4, c5 with the exponential decay time tau_e (og_time_weights). */
int og_kogan_e(double tau, double tau_e, double dt, double* out)
{
    og_tw k;
    og_time_weights(tau, tau_e, dt, &k);
    for (int i = 0; i < 6; ++i) out[i] = k.g[i];
    out[6] = k.c1; out[7] = k.c4; out[8] = k.c5;
    return OG_OK;
}

/* Degree of rarefaction eps_hat = tau/tau_hat of every face at state W, with the CFL step
 * of W, reduced to each cell as the largest over its 2 dim faces. */
/* A per-cell diagnostic of the face fluxes at the state's CFL step (which = 0: eps_hat =
 * tau/tau_hat, the rarefaction measure of Eqs. tautautilde and epsilonkomega; which = 1: the
 * relaxation time tau of Eqs. relaxation time, taua and tautchenadjusted): the largest over
 * the cell's faces. */
static int og_face_diag_field(const og_case* c, const double* W, const double* kk, const double* om, int which,
                              double* out)
{
    og_grid gr;
    int st = og_grid_init(&gr, c);
    if (st) { og_grid_free(&gr); return st; }
    const int dim = c->dim;
    const long N = gr.n[0] * gr.n[1] * gr.n[2];
    double rate;
    if ((st = og_max_rate(&gr, W, kk, om, &rate))) { og_grid_free(&gr); return st; }
    const double dt = c->cfl / rate;
    double* We = (double*)malloc(sizeof(double) * gr.nv * gr.next);
    double* S = (double*)malloc(sizeof(double) * N);
    og_fill_W(&gr, W, We);
    og_strain(&gr, We, S);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long s = 0; s < N; ++s) {
        long idx[3] = {s % gr.n[0], (s / gr.n[0]) % gr.n[1], s / (gr.n[0] * gr.n[1])};
        double mx = 0.0, F[5];
        for (int d = 0; d < dim; ++d)
            for (int side = 0; side < 2; ++side) {
                long f[3] = {idx[0], idx[1], idx[2]};
                f[d] += side;
                double diag[2];
                if (og_face_at(&gr, We, kk, om, S, d, f[0], f[1], f[2], dt, F, diag)) { bad = 1; continue; }
                if (diag[which] > mx) mx = diag[which];
            }
        out[s] = mx;
    }
    free(We); free(S);
    og_grid_free(&gr);
    return bad ? OG_ERR_NONPHYSICAL : OG_OK;
}

/* eps_hat = tau/tau_hat of every face at the state's CFL step, the largest per cell. */
int og_eps_field(const og_case* c, const double* W, const double* kk, const double* om, double* out)
{
    return og_face_diag_field(c, W, kk, om, 0, out);
}

/* The relaxation time tau of every face at the state's CFL step, the largest per cell. */
int og_tau_field(const og_case* c, const double* W, const double* kk, const double* om, double* out)
{
    return og_face_diag_field(c, W, kk, om, 1, out);
}

/* Solve <psi_m psi_n>_g x = r for a Maxwellian given by (rho, U[3], lam); face-local frame. */
int og_moment_solve(int dim, double gamma, const double* rhoUlam, const double* r, double* x)
{
    og_gas gas; og_maxw g; og_mom M;
    memset(&gas, 0, sizeof(gas));
    gas.dim = dim; gas.gamma = gamma; gas.b = 2.0 / (gamma - 1.0); gas.K = gas.b - dim;
    g.rho = rhoUlam[0]; g.U[0] = rhoUlam[1]; g.U[1] = rhoUlam[2]; g.U[2] = rhoUlam[3]; g.lam = rhoUlam[4];
    og_moments(&gas, &g, &M);
    return og_solve_moment_system(&gas, &M, r, x);
}

/* tau for explicit face quantities. */
double og_tau_value(double mu, double c_a, double c_mu, double rho0, double p0, double pl,
                    double pr, double kf, double wf, double Sf, double dt)
{
    og_gas gas;
    memset(&gas, 0, sizeof(gas));
    gas.mu = mu; gas.c_a = c_a; gas.c_mu = c_mu;
    return og_tau(&gas, rho0, p0, pl, pr, kf, wf, Sf, dt);
}

int og_info_len(void) { return OG_INFO_LEN; }
int og_nu(void) { return OG_NU; }
