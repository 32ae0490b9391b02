// gks_flux.hpp -- closed-form per-interface flux of the turbulent gas-kinetic scheme.
//
// One face, face-local frame (index 1 of a state vector is the normal momentum).  The
// scheme is Xu's BGK-NS flux as used by Righi (arXiv:1302.2132): the Kogan integral
// solution of the BGK model (Eq. integralbgk) with a Chapman-Enskog initial distribution
// on each side (Eq. initialf0), an equilibrium state built from the two half-space
// Maxwellians (Eq. intermediatestate) with its own linear expansion in space and time
// (Eq. eqlgform), integrated exactly over the time step (Eqs. resultingf, fluxesf), with
// tau = mu/p + tau_a + k-omega part (Eqs. relaxation time, taua, tautchenadjusted) and the
// Prandtl-number correction of the heat flux.
//
// How this differs from a literal evaluation:
//  * moments factorise into a u-moment sequence (full line or half line) times
//    tangential/internal moments; every <u^k psi (a.psi)> used here is a closed form in
//    five u-moments (tmom), so no moment table over (u, v, w, xi) is ever built;
//  * every moment-matrix system M(g) a = r is solved in closed form (solve);
//  * the time-integrated compatibility condition makes int int psi f = dt W0 +
//    dt^2/2 rho0 <psi Abar.psi>, so the u-less moments needed by the heat-flux
//    correction come for free from the right-hand side of the Abar system.
//
// Scalar type R is double (FP64 form) or float (FP32-flux form); reconstruction and
// primitive recovery arrive in double.  The code is plain templated arithmetic so that
// the library can also run it on the host with an operation-counting number type.
#pragma once

#ifndef GKS_HD
#define GKS_HD __host__ __device__
#endif

#include <type_traits>

#include "erfc_poly.hpp"

namespace gks {

GKS_HD inline double g_exp(double x) { return exp(x); }
GKS_HD inline float g_exp(float x) { return expf(x); }
GKS_HD inline double g_abs(double x) { return fabs(x); }
GKS_HD inline float g_abs(float x) { return fabsf(x); }
GKS_HD inline double g_min(double x, double y) { return fmin(x, y); }
GKS_HD inline float g_min(float x, float y) { return fminf(x, y); }
GKS_HD inline double g_copysign(double x, double s) { return copysign(x, s); }
GKS_HD inline float g_copysign(float x, float s) { return copysignf(x, s); }

// Reciprocal and reciprocal square root from the hardware estimates (v_rcp, v_rsq) refined
// by Newton-Raphson steps, r <- r + r (1 - x r) and y <- y + (y/2)(1 - x y^2), each of
// which squares the relative error of the estimate: two steps in FP64, one in FP32, leave
// about one ulp for the positive, normal, finite arguments of the flux (a non-physical
// state that reaches them is rejected by its own checks).  Host builds (operation
// counting, tests) use the plain operations.
GKS_HD inline double g_rcp(double x)
{
#ifdef __HIP_DEVICE_COMPILE__
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}
GKS_HD inline float g_rcp(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
#else
    return 1.0f / x;
#endif
}
GKS_HD inline double g_rsqrt(double x)
{
#ifdef __HIP_DEVICE_COMPILE__
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
#else
    return 1.0 / sqrt(x);
#endif
}
GKS_HD inline float g_rsqrt(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    const float y = __builtin_amdgcn_rsqf(x);
    return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);
#else
    return 1.0f / sqrtf(x);
#endif
}

template <typename R> GKS_HD inline R rconst(double v) { return R(v); }

// erfc(ax) for ax >= 0, given e = exp(-ax^2) (which the half-line moments need anyway):
// erfc(ax) = e g(ax) / (1 + 2 ax), with g(x) = (1 + 2x) exp(x^2) erfc(x) a polynomial in
// y = (ax - K)/(ax + K) (the truncated Chebyshev series of erfc_poly.hpp in the power
// basis), summed by Horner's rule.  One reciprocal serves both the map and 1/(1 + 2 ax).
template <typename R> struct ErfcPoly;
template <> struct ErfcPoly<double> {
    static constexpr int N = ERFC_N64;
    GKS_HD static constexpr double a(int k) { return ERFC_A64[k]; }
};
template <> struct ErfcPoly<float> {
    static constexpr int N = ERFC_N32;
    GKS_HD static constexpr float a(int k) { return ERFC_A32[k]; }
};

template <typename R>
GKS_HD inline R erfc_e(R ax, R e)
{
    const R K = R(ERFC_K);
    const R p = ax + K, q = R(1) + R(2) * ax;
    const R r = g_rcp(p * q);
    const R y = (ax - K) * q * r;          // (ax - K)/(ax + K)
    const R iq = p * r;                    // 1/(1 + 2 ax)
    R g = R(ErfcPoly<R>::a(ErfcPoly<R>::N - 1));
#pragma unroll
    for (int k = ErfcPoly<R>::N - 2; k >= 0; --k) g = g * y + R(ErfcPoly<R>::a(k));
    return e * g * iq;
}

// Maxwellian in the face-local frame together with the derived quantities every moment
// needs.  h = 1/(2 lambda) is the variance of each velocity component; bt = b - 1 is the
// number of quadratic degrees of freedom besides the normal velocity.
template <typename R, int D>
struct Mx {
    R rho, U[D], lam, h;
    R vt2;   // |tangential velocity|^2
    R q;     // <v^2 + w^2 + xi^2> = vt2 + bt h
};

template <typename R, int D>
GKS_HD inline void mx_set(Mx<R, D>& g, R rho, const R* U, R lam, R h, R bt)
{
    g.rho = rho;
    g.lam = lam;
    g.h = h;
    R v2 = R(0);
    for (int d = 0; d < D; ++d) g.U[d] = U[d];
    for (int d = 1; d < D; ++d) v2 = v2 + U[d] * U[d];
    g.vt2 = v2;
    g.q = v2 + bt * h;
}

// u-moment recurrence  m_{n+1} = U m_n + n h m_{n-1}  (Gaussian, integration by parts),
// filled from the first two entries up to index `last`.
template <typename R>
GKS_HD inline void urec(R* m, R U, R h, int last)
{
    for (int n = 1; n < last; ++n) m[n + 1] = U * m[n] + R(n) * h * m[n - 1];
}

// T = <u^k psi (a.psi)> from u-moments mk[0..4] = <u^k> .. <u^{k+4}> (full or half line),
// tangential velocities and xi over all values.  With c0 = a_0 + a_t.V_t + a_E q/2 and
// P_j = c0 <u^{k+j}> + a_u <u^{k+j+1}> + a_E/2 <u^{k+j+2}>:
//   T_rho = P_0, T_u = P_1, T_t = V_t P_0 + <u^k> (a_t + a_E V_t) h,
//   T_E = (P_2 + q P_0 + <u^k> X)/2,  X = 2h (a_t.V_t + a_E vt2) + a_E bt h^2
// (the X and h terms are the covariances of v_t and of v^2+w^2+xi^2 with a.psi).
template <typename R, int D>
GKS_HD inline void tmom(const Mx<R, D>& g, const R* mk, const R* a, R bt, R* T)
{
    const R aE = a[D + 1];
    R aV = R(0);
    for (int t = 1; t < D; ++t) aV = aV + a[1 + t] * g.U[t];
    const R half = R(0.5);
    const R c0 = a[0] + aV + half * aE * g.q;
    const R P0 = c0 * mk[0] + a[1] * mk[1] + half * aE * mk[2];
    const R P1 = c0 * mk[1] + a[1] * mk[2] + half * aE * mk[3];
    const R P2 = c0 * mk[2] + a[1] * mk[3] + half * aE * mk[4];
    const R X = R(2) * g.h * (aV + aE * g.vt2) + aE * bt * g.h * g.h;
    T[0] = P0;
    T[1] = P1;
    for (int t = 1; t < D; ++t) T[1 + t] = g.U[t] * P0 + mk[0] * (a[1 + t] + aE * g.U[t]) * g.h;
    T[D + 1] = half * (P2 + g.q * P0 + mk[0] * X);
}

// Tv = <u^k v_s psi (a.psi)> for a tangential velocity v_s (s = 1 .. D-1 in the face-local
// frame), from the same u-moments.  The Maxwellian's v_s-factor obeys v_s g = V_s g +
// h dg/dV_s, and psi (a.psi) does not depend on V_s, so Tv = V_s T + h dT/dV_s with T from
// tmom; with e = a_s + a_E V_s (= dc0/dV_s), dP_j/dV_s = e <u^{k+j}>:
//   dT_rho = e <u^k>, dT_u = e <u^{k+1}>,
//   dT_t = V_t e <u^k> + [t = s] (P_0 + <u^k> a_E h),
//   dT_E = (e <u^{k+2}> + 2 V_s P_0 + q e <u^k> + <u^k> 2h (a_s + 2 a_E V_s)) / 2.
template <typename R, int D>
GKS_HD inline void tvmom(const Mx<R, D>& g, const R* mk, const R* a, R bt, int s, R* Tv)
{
    const R aE = a[D + 1];
    R aV = R(0);
    for (int t = 1; t < D; ++t) aV = aV + a[1 + t] * g.U[t];
    const R half = R(0.5);
    const R c0 = a[0] + aV + half * aE * g.q;
    const R P0 = c0 * mk[0] + a[1] * mk[1] + half * aE * mk[2];
    const R P1 = c0 * mk[1] + a[1] * mk[2] + half * aE * mk[3];
    const R P2 = c0 * mk[2] + a[1] * mk[3] + half * aE * mk[4];
    const R X = R(2) * g.h * (aV + aE * g.vt2) + aE * bt * g.h * g.h;
    const R Vs = g.U[s], h = g.h;
    const R e = a[1 + s] + aE * Vs;
    Tv[0] = Vs * P0 + h * e * mk[0];
    Tv[1] = Vs * P1 + h * e * mk[1];
    for (int t = 1; t < D; ++t) {
        const R T = g.U[t] * P0 + mk[0] * (a[1 + t] + aE * g.U[t]) * h;
        R dT = g.U[t] * e * mk[0];
        if (t == s) dT = dT + P0 + mk[0] * aE * h;
        Tv[1 + t] = Vs * T + h * dT;
    }
    const R TE = half * (P2 + g.q * P0 + mk[0] * X);
    const R dTE = half * (e * mk[2] + R(2) * Vs * P0 + g.q * e * mk[0] + mk[0] * R(2) * h * (a[1 + s] + R(2) * aE * Vs));
    Tv[D + 1] = Vs * TE + h * dTE;
}

// <u^k psi> (a = unit vector on the density slot)
template <typename R, int D>
GKS_HD inline void tmom1(const Mx<R, D>& g, const R* mk, R* T)
{
    T[0] = mk[0];
    T[1] = mk[1];
    for (int t = 1; t < D; ++t) T[1 + t] = g.U[t] * mk[0];
    T[D + 1] = R(0.5) * (mk[2] + g.q * mk[0]);
}

// Closed-form solution of <psi (a.psi)>_g = r (b = total degrees of freedom):
//   a_E = (4 lam^2 / b) [2 r_E - 2 U.r_m + r_rho (|U|^2 - b/(2 lam))]
//   a_d = 2 lam (r_d - U_d r_rho) - U_d a_E
//   a_rho = r_rho - U.a_m - a_E (|U|^2 + b/(2 lam)) / 2
template <typename R, int D>
GKS_HD inline void solve(const Mx<R, D>& g, const R* r, R b, R inv_b, R* a)
{
    R U2 = R(0), Ur = R(0);
    for (int d = 0; d < D; ++d) { U2 = U2 + g.U[d] * g.U[d]; Ur = Ur + g.U[d] * r[1 + d]; }
    const R bh = b * g.h;
    const R aE = R(4) * g.lam * g.lam * inv_b * (R(2) * r[D + 1] - R(2) * Ur + r[0] * (U2 - bh));
    R Ua = R(0);
    for (int d = 0; d < D; ++d) {
        a[1 + d] = R(2) * g.lam * (r[1 + d] - g.U[d] * r[0]) - g.U[d] * aE;
        Ua = Ua + g.U[d] * a[1 + d];
    }
    a[0] = r[0] - Ua - R(0.5) * aE * (U2 + bh);
    a[D + 1] = aE;
}

// Time weights of the Kogan solution over [0, dt] (x = dt/tau, E = e^{-x}):
//   gam0 = dt - tau(1-E), gam1 = 2tau^2(1-E) - tau dt(1+E), gam2 = dt^2/2 - tau dt + tau^2(1-E),
//   gam3 = tau(1-E), gam4 = -(2tau^2(1-E) - tau dt E), gam5 = -tau^2(1-E),
// and the ratios c1, c4, c5 = gam1, gam4, gam5 over tau*gam0 of the integrated compatibility
// condition.  Below x = 1/2 the cancelling combinations come from their power series.
template <typename R>
struct Kw {
    R g[6];
    R c1, c4, c5;
};

// Power series of the small-x weights with the leading powers factored out:
//   x - (1 - E)        = x^2 P0(x),  P0 = sum_k (-1)^k x^k / (k+2)!
//   2(1-E) - x(1+E)    = -x^3 P1(x), P1 = sum_k (-1)^k (k+1) x^k / (k+3)!
//   x^2/2 - x + (1-E)  = x^3 P2(x),  P2 = sum_k (-1)^k x^k / (k+3)!
// Only P2 is summed: P0 = 1/2 - x P2 (shift of the index), and P1 = P0 - 2 P2 because
// (k+1)/(k+3)! = 1/(k+2)! - 2/(k+3)!.  For x < 1/2 neither step loses more than a factor
// 3 to cancellation.  The coefficients (-1)^k/(k+3)! are formed at compile time (17! is
// exact in double); the first dropped term is below 2^-60 (FP64, 15 terms) or 2^-27
// (FP32, 8 terms) of P2.
template <int N>
struct KoganSeries {
    double c[N];
    constexpr KoganSeries() : c()
    {
        double f = 6.0;                                      // (k+3)!
        for (int k = 0; k < N; ++k) {
            c[k] = ((k & 1) ? -1.0 : 1.0) / f;
            f *= double(k + 4);
        }
    }
};
template <typename R> struct KoganTerms { static constexpr int N = 15; };
template <> struct KoganTerms<float> { static constexpr int N = 8; };
constexpr KoganSeries<15> KOGAN_SERIES{};

template <typename R>
GKS_HD inline Kw<R> kogan(R tau, R dt)
{
    Kw<R> k;
    if (!(tau > R(0))) {
        k.g[0] = dt; k.g[1] = R(0); k.g[2] = R(0.5) * dt * dt;
        k.g[3] = R(0); k.g[4] = R(0); k.g[5] = R(0);
        k.c1 = R(-1); k.c4 = R(0); k.c5 = R(0);
        return k;
    }
    const R x = dt * g_rcp(tau);
    R s, g0, g1, g2, g4;
    if (x < R(0.5)) {
        constexpr int N = KoganTerms<R>::N;
        R p2 = R(KOGAN_SERIES.c[N - 1]);
#pragma unroll
        for (int j = N - 2; j >= 0; --j) p2 = p2 * x + R(KOGAN_SERIES.c[j]);
        const R p0 = R(0.5) - x * p2;
        const R p1 = p0 - R(2) * p2;
        const R x2 = x * x, x3 = x2 * x;
        g0 = x2 * p0;
        g1 = -(x3 * p1);
        g2 = x3 * p2;
        s = x - g0;
        g4 = x + g1;
    } else {
        const R E = g_exp(-x);
        s = R(1) - E;
        g0 = x - s;
        g1 = R(2) * s - x * (R(1) + E);
        g2 = R(0.5) * x * x - x + s;
        g4 = R(2) * s - x * E;
    }
    const R t2 = tau * tau;
    k.g[0] = tau * g0;
    k.g[1] = t2 * g1;
    k.g[2] = t2 * g2;
    k.g[3] = tau * s;
    k.g[4] = -t2 * g4;
    k.g[5] = -t2 * s;
    const R ig0 = g_rcp(g0);
    k.c1 = g1 * ig0;
    k.c4 = -g4 * ig0;
    k.c5 = -s * ig0;
    return k;
}

// Weights when the rarefaction is measured against a resolved time scale tau_hat
// (Eqs. tautautilde, rarefactionkepsilon, epsilonkomega): the exponentials decay with
// tau_e = dt tau/tau_hat while the Chapman-Enskog parts keep the physical tau.  With
// gam'_j, c'_j the Kogan weights at tau_e (kogan(tau_e, dt)) and d = tau_e - tau (the
// Chapman-Enskog factor tau tau_e = tau_e^2 - d tau_e):
//   gam0 = gam'0, gam3 = gam'3, gam1 = gam'1 + d gam0, gam2 = gam'2 + d gam0,
//   gam4 = gam'4 + d gam3, gam5 = -tau gam3,
//   c1 = (tau_e c'1 + d)/tau, c4 = (tau_e c'4 - d c'5)/tau, c5 = c'5   (c_j = gam_j/(tau gam0)).
// tau_e = tau gives kogan(tau, dt); tau_e = 0 is the hydrodynamic limit (kogan's tau = 0
// branch corrected: no upwind part, gam1 = -tau dt, gam2 = dt^2/2 - tau dt, c1 = -1).
template <typename R>
GKS_HD inline Kw<R> kogan_e(R tau, R tau_e, R dt)
{
    Kw<R> k = kogan(tau_e, dt);
    if (tau > R(0)) {                                 // tau = 0 implies tau_e = 0: the Euler limit
        const R d = tau_e - tau, itau = g_rcp(tau);
        k.g[1] = k.g[1] + d * k.g[0];
        k.g[2] = k.g[2] + d * k.g[0];
        k.g[4] = k.g[4] + d * k.g[3];
        k.g[5] = -tau * k.g[3];
        k.c1 = (tau_e * k.c1 + d) * itau;
        k.c4 = (tau_e * k.c4 - d * k.c5) * itau;
    }
    return k;
}

// Flux modes (bits): FLUX_TAUHAT evaluates the time weights with eps = tau/tau_hat;
// FLUX_EPS_OUT also stores eps_hat = tau/tau_hat in F[D + 2] and the relaxation time tau in
// F[D + 3] (the caller provides room);
// FLUX_MULTID expands the distributions along the tangential axes too (FaceIn::tl, tr).
enum { FLUX_TAUHAT = 1, FLUX_EPS_OUT = 2, FLUX_MULTID = 4 };

// Inputs of one face in the wide type H (FP64 on the device): reconstructed states,
// minmod slopes, cell averages of the two neighbours, inverse centre-to-face distances,
// face means of k, omega and strain rate, and the step.
template <int D, typename H = double>
struct FaceIn {
    H Wl[D + 2], Wr[D + 2], sl[D + 2], sr[D + 2], Wi[D + 2], Wi1[D + 2];
    H idl, idr, kf, wf, Sf, dt;
    H tl[D - 1][D + 2], tr[D - 1][D + 2];   // tangential gradients of the two cells (FLUX_MULTID)
};

// Where the flux reads the two cells' states (the equilibrium slopes through the interface
// state): by default the copies in FaceIn; a caller whose stencil sits in LDS may pass a
// functor cs(side, m) that reads them again there at the point of use.
struct InCells {};
template <int D, typename H, typename CS>
GKS_HD __attribute__((always_inline)) inline H cell_of(const FaceIn<D, H>& in, const CS& cs, int side, int m)
{
    if constexpr (std::is_same<CS, InCells>::value) return side ? in.Wi1[m] : in.Wi[m];
    else return cs(side, m);
}

// Per-solve constants; the reciprocals are formed once on the host.
struct GasC {
    double mu, c_a, b;
    double two_over_b, inv_b, inv_cmu, pfix;   // 2/b, 1/b, 1/C_mu, 1/Pr - 1
};

// minmod: the smaller magnitude with the common sign, zero when the signs differ
template <typename H>
GKS_HD inline H minmod(H p, H q)
{
    const H m = g_copysign(g_min(g_abs(p), g_abs(q)), p);
    return (p * q > H(0)) ? m : H(0);
}

// Face geometry along the normal: inverse distances between the centres of cells
// i-1, i, i+1, i+2 (icd[0..2]), centre-to-face distances dl, dr and their inverses.
template <typename H>
struct FaceGeo {
    H icd[3], dl, dr, idl, idr;
};

// Third-order MUSCL slope towards a face (the limited kappa-scheme with kappa = 1/3): of a
// cell whose one-sided slopes are `away` (across its far face) and `toward` (across this
// face), (1/3) minmod(away, 4 toward) + (2/3) minmod(toward, 4 away).  Both minmods vanish
// unless the slopes share a sign, and then carry it, so this is one select:
//   away toward > 0 ? sign(toward) ((1/3) min(|away|, 4|toward|) + (2/3) min(|toward|, 4|away|)) : 0.
template <typename H>
GKS_HD inline H muscl3(H away, H toward)
{
    const H a = g_abs(away), t = g_abs(toward);
    const H m = H(1.0 / 3.0) * g_min(a, H(4) * t) + H(2.0 / 3.0) * g_min(t, H(4) * a);
    return (away * toward > H(0)) ? g_copysign(m, toward) : H(0);
}

// Fifth-order WENO value (Jiang and Shu) at the face between cells c and d of the five
// cell averages a..e, upwind side a..c, in index space: third-order candidates q_k of the
// stencils {a,b,c}, {b,c,d}, {c,d,e}, smoothness indicators beta_k, linear weights
// (1/10, 6/10, 3/10) and weights d_k/(eps + beta_k)^2 with eps = 1e-6.  With
// P_k = (eps + beta_k)^2 the weighted mean is written over the common denominator,
//   (d0 q0 P1 P2 + d1 q1 P0 P2 + d2 q2 P0 P1) / (d0 P1 P2 + d1 P0 P2 + d2 P0 P1),
// one reciprocal instead of four.
template <typename H>
GKS_HD inline H weno5(H a, H b, H c, H d, H e)
{
    const H sixth = H(1.0 / 6.0), c13 = H(13.0 / 12.0), qt = H(0.25), eps = H(1e-6);
    const H q0 = (H(2) * a - H(7) * b + H(11) * c) * sixth;
    const H q1 = (H(5) * c - b + H(2) * d) * sixth;
    const H q2 = (H(2) * c + H(5) * d - e) * sixth;
    const H s0 = a - H(2) * b + c, t0 = a - H(4) * b + H(3) * c;
    const H s1 = b - H(2) * c + d, t1 = b - d;
    const H s2 = c - H(2) * d + e, t2 = H(3) * c - H(4) * d + e;
    const H e0 = eps + (c13 * s0 * s0 + qt * t0 * t0);
    const H e1 = eps + (c13 * s1 * s1 + qt * t1 * t1);
    const H e2 = eps + (c13 * s2 * s2 + qt * t2 * t2);
    const H p0 = e0 * e0, p1 = e1 * e1, p2 = e2 * e2;
    const H w0 = H(0.1) * (p1 * p2), w1 = H(0.6) * (p0 * p2), w2 = H(0.3) * (p0 * p1);
    return (w0 * q0 + w1 * q1 + w2 * q2) * g_rcp(w0 + w1 + w2);
}

// Reconstruction along the face normal from the cell averages w(0..3, m) (cells i-1, i,
// i+1, i+2 around face i+1/2; with RK = 2 also w(-1, m) and w(4, m), cells i-2 and i+3),
// conservative variables, one-sided differences on centre-to-centre distances.  The
// gradients are their minmod; the face values come from those gradients (RK = 0, second
// order), from the third-order slopes above (RK = 1) or are the WENO5 values (RK = 2).
// `w(o, m)` reads component m of stencil cell o (a private array or the tile's LDS); the
// components are reconstructed one at a time, and with the wider stencils the device code
// keeps them apart, so that only one component's stencil is held at once.
template <int D, typename H, int RK = 0, typename SW>
GKS_HD inline void reconstruct_s(const SW& w, const FaceGeo<H>& geo, FaceIn<D, H>& in)
{
#pragma unroll
    for (int m = 0; m < D + 2; ++m) {
        const H c0 = w(0, m), c1 = w(1, m), c2 = w(2, m), c3 = w(3, m);
        const H d0 = (c1 - c0) * geo.icd[0];
        const H d1 = (c2 - c1) * geo.icd[1];
        const H d2 = (c3 - c2) * geo.icd[2];
        const H sl = minmod(d0, d1), sr = minmod(d1, d2);
        in.sl[m] = sl;
        in.sr[m] = sr;
        if constexpr (RK == 2) {
            const H cm = w(-1, m), c4 = w(4, m);
            in.Wl[m] = weno5(cm, c0, c1, c2, c3);
            in.Wr[m] = weno5(c4, c3, c2, c1, c0);
        } else if constexpr (RK == 1) {
            in.Wl[m] = c1 + muscl3(d0, d1) * geo.dl;
            in.Wr[m] = c2 - muscl3(d2, d1) * geo.dr;
        } else {
            in.Wl[m] = c1 + sl * geo.dl;
            in.Wr[m] = c2 - sr * geo.dr;
        }
        in.Wi[m] = c1;
        in.Wi1[m] = c2;
#ifdef __HIP_DEVICE_COMPILE__
        if constexpr (RK != 0) __builtin_amdgcn_sched_barrier(0);
#endif
    }
    in.idl = geo.idl;
    in.idr = geo.idr;
}

template <int D, typename H, int RK = 0>
GKS_HD inline void reconstruct(const H (*Wc)[D + 2], const FaceGeo<H>& geo, FaceIn<D, H>& in)
{
    reconstruct_s<D, H, RK>([Wc](int o, int m) { return Wc[o][m]; }, geo, in);
}

// Primitive recovery in the wide type: rho, 1/rho, U, p.  Returns false for rho <= 0 or
// p <= 0 (or non-finite).
template <int D, typename H>
GKS_HD inline bool prim_wide(const H* W, H two_over_b, H& rho, H& irho, H* U, H& p)
{
    rho = W[0];
    irho = g_rcp(rho);
    H ke = H(0);
    for (int d = 0; d < D; ++d) { U[d] = W[1 + d] * irho; ke = ke + U[d] * W[1 + d]; }
    p = two_over_b * (W[D + 1] - H(0.5) * ke);
    return (rho > H(0)) && (p > H(0)) && (p < H(1e300)) && (rho < H(1e300));
}

// Time weights of a face in a flux mode other than 0, in the wide type.  tau_hat =
// rho0/|D rho|, with D rho = U0 d_x rho - d_x (rho U) along the normal (mass conservation
// gives d_t rho = -d_x (rho U)) from the mean of the one-sided gradients through the
// interface state W0 (rho w00, normal momentum w01); eps_hat = tau/tau_hat, stored in
// Fout[D + 2] with FLUX_EPS_OUT.
template <int D, typename H, int MODE, typename CS = InCells>
GKS_HD __attribute__((always_inline)) inline Kw<H> mode_weights(const FaceIn<D, H>& in, H tau, const H* W0,
                                                               const H* U0d, H ir0, H* Fout, const CS& cs = CS())
{
    const H w00 = W0[0], w01 = W0[1];
    const H grho = H(0.5) * ((w00 - cell_of(in, cs, 0, 0)) * in.idl + (cell_of(in, cs, 1, 0) - w00) * in.idr);
    const H gmom = H(0.5) * ((w01 - cell_of(in, cs, 0, 1)) * in.idl + (cell_of(in, cs, 1, 1) - w01) * in.idr);
    const H eps = tau * g_abs(U0d[0] * grho - gmom) * ir0;
    if (MODE & FLUX_EPS_OUT) Fout[D + 2] = eps;
    return (MODE & FLUX_TAUHAT) ? kogan_e(tau, in.dt * eps, in.dt) : kogan(tau, in.dt);
}

template <typename R, typename H>
GKS_HD inline Kw<R> kw_narrow(const Kw<H>& k)
{
    Kw<R> r;
    for (int j = 0; j < 6; ++j) r.g[j] = R(k.g[j]);
    r.c1 = R(k.c1);
    r.c4 = R(k.c4);
    r.c5 = R(k.c5);
    return r;
}

// Narrow copy of a wide Maxwellian (vt2 and q formed in the narrow type).
template <typename R, typename H, int D>
GKS_HD inline void mx_narrow(Mx<R, D>& g, const Mx<H, D>& w, R bt)
{
    if constexpr (std::is_same<R, H>::value) {
        (void)bt;
        g = w;
    } else {
        R u[D];
        for (int d = 0; d < D; ++d) u[d] = R(w.U[d]);
        mx_set(g, R(w.rho), u, R(w.lam), R(w.h), bt);
    }
}

// The flux.  Returns 0, or 1 when a state met is non-physical (then Fout is meaningless).
// Fout receives the time-integrated flux (it already contains dt) in the face-local frame,
// in the wide type H.
//
// R is the arithmetic of the flux; H (FP64 on the device) that of the reconstructed
// states.  When R is narrower than H (the FP32-flux form), every part of the flux of size
// p dt is kept in H: the half-line moments of the two sides, the interface state W0, the
// time weights, and the two terms that hold the Euler-like part of the flux,
//   gam0 rho0 <u psi>_g0  (the Euler flux of W0)  and
//   gam3 (rho_l <u psi>_{l,>0} + rho_r <u psi>_{r,<0})  (the collisionless flux),
// with gam0 + gam3 = dt.  R then carries only the non-equilibrium terms (the slopes a, A,
// abar, Abar and their gam1, gam2, gam4, gam5 contractions), which are smaller than p dt by
// about tau |grad W|/W, so the FP32 rounding no longer sets an absolute error floor of
// order eps_32 p dt in the normal-momentum flux; the heat-flux correction is assembled in
// H as well.  When R = H the evaluation is a single pass in R.
//
// Evaluation order keeps few values live: after the interface state and tau are known,
// the equilibrium-slope terms, then the left side, then the right side are each folded
// into F and into the right-hand side Rv of the Abar system as soon as their
// coefficients exist; Abar and the remaining equilibrium terms come last.
template <typename R, int D, typename H = double, int MODE = 0, typename CS = InCells>
GKS_HD __attribute__((always_inline)) inline int face_flux(const FaceIn<D, H>& in, const GasC& gas, H* Fout,
                                                           const CS& cs = CS())
{
    constexpr int NV = D + 2;
    constexpr bool SPLIT = !std::is_same<R, H>::value;
    const R b = R(gas.b), inv_b = R(gas.inv_b), bt = R(gas.b - 1.0);
    const H btw = H(gas.b - 1.0);
    const R half = R(0.5);
    const H rsqpi_half = H(0.28209479177387814);   // 1/(2 sqrt(pi))
    const H bw = H(gas.two_over_b);

    // --- left / right Maxwellians (wide primitive recovery; narrow copies) ------------
    H rl, irl, Ul[D], pl, rr, irr, Ur[D], pr;
    if (!prim_wide<D>(in.Wl, bw, rl, irl, Ul, pl) || !prim_wide<D>(in.Wr, bw, rr, irr, Ur, pr)) return 1;
    Mx<H, D> glw, grw;
    mx_set(glw, rl, Ul, H(0.5) * rl * g_rcp(pl), pl * irl, btw);   // 1/(2 lambda) = p/rho
    mx_set(grw, rr, Ur, H(0.5) * rr * g_rcp(pr), pr * irr, btw);
    Mx<R, D> gl, gr;
    mx_narrow(gl, glw, bt);
    mx_narrow(gr, grw, bt);

    // --- half-line u-moments: left over u>0, right over u<0 (wide).  Only <u^0>, <u^1>
    //     are kept; higher ones are regenerated by the recurrence where they are used. --
    //     <u^0>_{>0} = erfc(-sqrt(lambda) U)/2, <u^0>_{<0} = erfc(sqrt(lambda) U)/2; the
    //     exp(-lambda U^2) of the first moment also scales the erfc evaluation.
    H ml01[2], mr01[2];
    {
        const H isq = g_rsqrt(glw.lam);               // 1/sqrt(lambda)
        const H U = glw.U[0];
        const H x = -glw.lam * isq * U;
        const H e = g_exp(-glw.lam * U * U);
        const H hs = H(0.5) * erfc_e(g_abs(x), e);
        ml01[0] = x >= H(0) ? hs : H(1) - hs;
        ml01[1] = U * ml01[0] + e * rsqpi_half * isq;
    }
    {
        const H isq = g_rsqrt(grw.lam);
        const H U = grw.U[0];
        const H x = grw.lam * isq * U;
        const H e = g_exp(-grw.lam * U * U);
        const H hs = H(0.5) * erfc_e(g_abs(x), e);
        mr01[0] = x >= H(0) ? hs : H(1) - hs;
        mr01[1] = U * mr01[0] - e * rsqpi_half * isq;
    }

    // --- interface equilibrium state W0 (Eq. intermediatestate), wide ----------------
    H W0[NV];
    {
        H tl[NV], tr[NV], m3[3];
        m3[0] = ml01[0]; m3[1] = ml01[1];
        urec(m3, glw.U[0], glw.h, 2);
        tmom1(glw, m3, tl);
        m3[0] = mr01[0]; m3[1] = mr01[1];
        urec(m3, grw.U[0], grw.h, 2);
        tmom1(grw, m3, tr);
        for (int m = 0; m < NV; ++m) W0[m] = glw.rho * tl[m] + grw.rho * tr[m];
    }
    H r0, ir0, U0d[D], p0;
    if (!prim_wide<D>(W0, bw, r0, ir0, U0d, p0)) return 1;
    const H h0 = p0 * ir0, ip0 = g_rcp(p0);
    Mx<R, D> g0;
    {
        R u[D];
        for (int d = 0; d < D; ++d) u[d] = R(U0d[d]);
        mx_set(g0, R(r0), u, R(H(0.5) * r0 * ip0), R(h0), bt);
    }

    // --- relaxation time (laminar + artificial + k-omega) and time weights ----------
    // tau = mu/p0 + (k/omega)(rho0/p0)/sqrt(1 + eta^2) with eta = S/(C_mu omega), written as
    // (mu + k rho0 / sqrt(omega^2 + (S/C_mu)^2)) / p0 (omega > 0).
    H tau;
    {
        const H sc = in.Sf * H(gas.inv_cmu);
        tau = ip0 * (H(gas.mu) + in.kf * r0 * g_rsqrt(in.wf * in.wf + sc * sc));
        if (gas.c_a > 0.0) tau = tau + H(gas.c_a) * g_abs(pr - pl) * g_rcp(pr + pl) * in.dt;
    }
    if (MODE & FLUX_EPS_OUT) Fout[D + 3] = tau;
    Kw<H> kwh;
    if (MODE & (FLUX_TAUHAT | FLUX_EPS_OUT)) kwh = mode_weights<D, H, MODE>(in, tau, W0, U0d, ir0, Fout, cs);
    else kwh = kogan(tau, in.dt);
    const Kw<R> kw = kw_narrow<R>(kwh);

    // --- wide part of a split evaluation: the gam0 Euler flux of W0 and the gam3
    //     collisionless flux of the two half-Maxwellians -----------------------------
    // With the heat-flux correction linear in F and in G = dt W0 + dt^2/2 Rv (below), the
    // wide part's share of q is formed here: qw = q(Fw) - U0_n dt (W0_E - U0.W0_m +
    // |U0|^2 rho0/2), where the last bracket is the internal energy b p0/2 of W0.
    [[maybe_unused]] H Fw[NV];
    [[maybe_unused]] H qw = H(0);
    if constexpr (SPLIT) {
        H m[4], T[NV];
        Mx<H, D> g0w;
        mx_set(g0w, r0, U0d, H(0.5) * r0 * ip0, h0, btw);
        m[0] = H(1);
        m[1] = U0d[0];
        urec(m, U0d[0], h0, 3);
        tmom1(g0w, m + 1, T);                          // <u psi>_g0 over all u
        for (int q = 0; q < NV; ++q) Fw[q] = kwh.g[0] * r0 * T[q];
        m[0] = ml01[0]; m[1] = ml01[1];
        urec(m, glw.U[0], glw.h, 3);
        tmom1(glw, m + 1, T);                          // <u psi>_{g_l, u>0}
        for (int q = 0; q < NV; ++q) Fw[q] = Fw[q] + kwh.g[3] * rl * T[q];
        m[0] = mr01[0]; m[1] = mr01[1];
        urec(m, grw.U[0], grw.h, 3);
        tmom1(grw, m + 1, T);                          // <u psi>_{g_r, u<0}
        for (int q = 0; q < NV; ++q) Fw[q] = Fw[q] + kwh.g[3] * rr * T[q];
        H uF = H(0), U2 = H(0);
        for (int d = 0; d < D; ++d) {
            uF = uF + U0d[d] * Fw[1 + d];
            U2 = U2 + U0d[d] * U0d[d];
        }
        qw = (Fw[D + 1] - uF + H(0.5) * U2 * Fw[0]) - U0d[0] * in.dt * (H(0.5) * H(gas.b) * p0);
    }
    const R ml01n[2] = {R(ml01[0]), R(ml01[1])}, mr01n[2] = {R(mr01[0]), R(mr01[1])};
    R F[NV];

    // Rv accumulates rho0 <psi Abar.psi>_g0 from the time-integrated compatibility condition:
    //   c1 rho0 (<u psi abar_l.psi>_{g0,>0} + <u psi abar_r.psi>_{g0,<0})
    // + c4 (rho_l <u psi a_l.psi>_{l,>0} + rho_r <u psi a_r.psi>_{r,<0})
    // + c5 (rho_l <psi A_l.psi>_{l,>0} + rho_r <psi A_r.psi>_{r,<0})
    R Rv[NV];

    // --- equilibrium slopes through W0 (Eq. eqlgform): gam1 and c1 terms -------------
    {
        R m0p[8], m0n[8];
        const R U = g0.U[0];
        const R isq = g_rsqrt(g0.lam);                 // 1/sqrt(lambda0)
        const R e = g_exp(-g0.lam * U * U);
        const R small = half * erfc_e(g_abs(g0.lam * isq * U), e);   // one erfc serves both halves
        const R tail = e * R(rsqpi_half) * isq;
        const bool upos = U >= R(0);
        m0p[0] = upos ? R(1) - small : small;
        m0n[0] = upos ? small : R(1) - small;
        m0p[1] = U * m0p[0] + tail;
        m0n[1] = U * m0n[0] - tail;
        urec(m0p, U, g0.h, 6);
        urec(m0n, U, g0.h, 6);
        R r[NV], ab[NV], T1[NV], T2[NV];
        const H il = ir0 * in.idl, ir = ir0 * in.idr;
        for (int m = 0; m < NV; ++m) r[m] = R((W0[m] - cell_of(in, cs, 0, m)) * il);
        solve(g0, r, b, inv_b, ab);
        tmom(g0, m0p + 1, ab, bt, T1);                 // <u psi abar_l.psi>_{g0,>0}
        tmom(g0, m0p + 2, ab, bt, T2);                 // <u^2 psi abar_l.psi>_{g0,>0}
        for (int m = 0; m < NV; ++m) r[m] = R((cell_of(in, cs, 1, m) - W0[m]) * ir);
        solve(g0, r, b, inv_b, ab);
        R T3[NV];
        tmom(g0, m0n + 1, ab, bt, T3);
        for (int m = 0; m < NV; ++m) Rv[m] = kw.c1 * g0.rho * (T1[m] + T3[m]);
        tmom(g0, m0n + 2, ab, bt, T3);
        for (int m = 0; m < NV; ++m) F[m] = g0.rho * kw.g[1] * (T2[m] + T3[m]);
        if constexpr ((MODE & FLUX_MULTID) != 0) {
            // tangential slopes of the interface state, from the mean tangential gradients:
            // b_bar v_t enters like abar u, over all u
            R m0f[7];
            for (int n = 0; n < 7; ++n) m0f[n] = m0p[n] + m0n[n];
            for (int s = 1; s < D; ++s) {
                for (int m = 0; m < NV; ++m) r[m] = R(H(0.5) * (in.tl[s - 1][m] + in.tr[s - 1][m]) * ir0);
                solve(g0, r, b, inv_b, ab);
                tvmom(g0, m0f, ab, bt, s, T1);
                tvmom(g0, m0f + 1, ab, bt, s, T2);
                for (int m = 0; m < NV; ++m) {
                    Rv[m] = Rv[m] + kw.c1 * g0.rho * T1[m];
                    F[m] = F[m] + g0.rho * kw.g[1] * T2[m];
                }
            }
        }
    }

    // --- one side of the initial distribution (Eq. initialf0): slopes a from dW/dx,
    //     time coefficients A from the compatibility condition at t = 0, then the
    //     gam3..gam5 flux terms (gam3 in the wide part when split) and the c4, c5 terms
    //     of Rv -------------------------------------------------------------------------
    auto side = [&](const Mx<R, D>& g, const R* m01, const H* slope, const H (*tslope)[D + 2], H irho) {
        R r[NV], a[NV], A[NV], T[NV], mf[8], mh[8];
        const R ir = R(irho);
        for (int m = 0; m < NV; ++m) r[m] = R(slope[m]) * ir;
        solve(g, r, b, inv_b, a);
        mf[0] = R(1);
        mf[1] = g.U[0];
        urec(mf, g.U[0], g.h, 5);
        tmom(g, mf + 1, a, bt, T);                     // <u psi (a.psi)> over all u
        if constexpr ((MODE & FLUX_MULTID) != 0) {
            // tangential slopes b_s: <psi (a u + b.v_t + A)> = 0 over all u, and the flux and
            // compatibility terms of b v_t beside those of a u (half line)
            mh[0] = m01[0];
            mh[1] = m01[1];
            urec(mh, g.U[0], g.h, 6);
            R bs[NV], Tv[NV], acc[NV], tacc[NV];
            for (int m = 0; m < NV; ++m) { acc[m] = R(0); tacc[m] = R(0); }
            for (int s = 1; s < D; ++s) {
                for (int m = 0; m < NV; ++m) r[m] = R(tslope[s - 1][m]) * ir;
                solve(g, r, b, inv_b, bs);
                tvmom(g, mf, bs, bt, s, Tv);
                for (int m = 0; m < NV; ++m) T[m] = T[m] + Tv[m];
                tvmom(g, mh + 1, bs, bt, s, Tv);
                for (int m = 0; m < NV; ++m) acc[m] = acc[m] + kw.g[4] * Tv[m];
                tvmom(g, mh, bs, bt, s, Tv);
                for (int m = 0; m < NV; ++m) tacc[m] = tacc[m] + kw.c4 * Tv[m];
            }
            for (int m = 0; m < NV; ++m) T[m] = -T[m];
            solve(g, T, b, inv_b, A);
            const R rg = g.rho;
            if constexpr (!SPLIT) {
                tmom1(g, mh + 1, T);
                for (int m = 0; m < NV; ++m) acc[m] = acc[m] + kw.g[3] * T[m];
            }
            tmom(g, mh + 2, a, bt, T);
            for (int m = 0; m < NV; ++m) acc[m] = acc[m] + kw.g[4] * T[m];
            tmom(g, mh + 1, A, bt, T);
            for (int m = 0; m < NV; ++m) F[m] = F[m] + rg * (acc[m] + kw.g[5] * T[m]);
            tmom(g, mh + 1, a, bt, T);
            for (int m = 0; m < NV; ++m) tacc[m] = tacc[m] + kw.c4 * T[m];
            tmom(g, mh, A, bt, T);
            for (int m = 0; m < NV; ++m) Rv[m] = Rv[m] + rg * (tacc[m] + kw.c5 * T[m]);
        } else {
            (void)tslope;
            for (int m = 0; m < NV; ++m) T[m] = -T[m];
            solve(g, T, b, inv_b, A);
            mh[0] = m01[0];
            mh[1] = m01[1];
            urec(mh, g.U[0], g.h, 6);
            const R rg = g.rho;
            R acc[NV];
            if constexpr (SPLIT) {
                tmom(g, mh + 2, a, bt, T);
                for (int m = 0; m < NV; ++m) acc[m] = kw.g[4] * T[m];
            } else {
                tmom1(g, mh + 1, T);
                for (int m = 0; m < NV; ++m) acc[m] = kw.g[3] * T[m];
                tmom(g, mh + 2, a, bt, T);
                for (int m = 0; m < NV; ++m) acc[m] = acc[m] + kw.g[4] * T[m];
            }
            tmom(g, mh + 1, A, bt, T);
            for (int m = 0; m < NV; ++m) F[m] = F[m] + rg * (acc[m] + kw.g[5] * T[m]);
            tmom(g, mh + 1, a, bt, T);
            for (int m = 0; m < NV; ++m) acc[m] = kw.c4 * T[m];
            tmom(g, mh, A, bt, T);
            for (int m = 0; m < NV; ++m) Rv[m] = Rv[m] + rg * (acc[m] + kw.c5 * T[m]);
        }
    };
    side(gl, ml01n, in.sl, in.tl, irl);
    side(gr, mr01n, in.sr, in.tr, irr);

    // --- Abar, then the gam2 (and, unsplit, gam0) equilibrium terms ------------------
    {
        R m0[8], r[NV], Ab[NV], T[NV];
        const R i0 = R(ir0);
        for (int m = 0; m < NV; ++m) r[m] = Rv[m] * i0;
        solve(g0, r, b, inv_b, Ab);
        m0[0] = R(1);
        m0[1] = g0.U[0];
        urec(m0, g0.U[0], g0.h, 5);
        if constexpr (SPLIT) {
            tmom(g0, m0 + 1, Ab, bt, T);
            for (int m = 0; m < NV; ++m) F[m] = F[m] + g0.rho * (kw.g[2] * T[m]);
        } else {
            R acc[NV];
            tmom1(g0, m0 + 1, T);
            for (int m = 0; m < NV; ++m) acc[m] = kw.g[0] * T[m];
            tmom(g0, m0 + 1, Ab, bt, T);
            for (int m = 0; m < NV; ++m) F[m] = F[m] + g0.rho * (acc[m] + kw.g[2] * T[m]);
        }
    }
    for (int m = 0; m < NV; ++m) {
        if constexpr (SPLIT) Fout[m] = Fw[m] + H(F[m]);
        else Fout[m] = F[m];
    }

    // --- Prandtl-number correction of the energy flux -------------------------------
    // q = int int (u - U0)(|u - U0|^2 + xi^2)/2 f
    //   = (F_E - U0.F_m + |U0|^2 F_rho/2) - U0_n (G_E - U0.G_m + |U0|^2 G_rho/2),
    // with G = int int psi f = dt W0 + dt^2/2 Rv (the integrated compatibility condition).
    // Split: q = qw + the same expression over the narrow F and dt^2/2 Rv alone.
    if constexpr (SPLIT) {
        const R dt = R(in.dt), hdt2 = half * dt * dt;
        R uF = R(0), uR = R(0), U2 = R(0);
        for (int d = 0; d < D; ++d) {
            uF = uF + g0.U[d] * F[1 + d];
            uR = uR + g0.U[d] * Rv[1 + d];
            U2 = U2 + g0.U[d] * g0.U[d];
        }
        const R qn = (F[D + 1] - uF + half * U2 * F[0]) - g0.U[0] * hdt2 * (Rv[D + 1] - uR + half * U2 * Rv[0]);
        Fout[D + 1] = Fout[D + 1] + H(gas.pfix) * (qw + H(qn));
    } else {
        const H pfix = H(gas.pfix);
        H Gv[NV];
        H dtq = in.dt;
#ifdef __HIP_DEVICE_COMPILE__
        // in the flux modes the weights' dt/2 would otherwise be kept from there to here
        if (MODE & (FLUX_TAUHAT | FLUX_EPS_OUT)) asm volatile("" : "+v"(dtq));
#endif
        const H hdt2 = H(0.5) * dtq * dtq;
        for (int m = 0; m < NV; ++m) Gv[m] = in.dt * W0[m] + hdt2 * H(Rv[m]);
        H uF = H(0), uG = H(0), U2 = H(0);
        for (int d = 0; d < D; ++d) {
            uF = uF + U0d[d] * Fout[1 + d];
            uG = uG + U0d[d] * Gv[1 + d];
            U2 = U2 + U0d[d] * U0d[d];
        }
        const H q = (Fout[D + 1] - uF + H(0.5) * U2 * Fout[0]) - U0d[0] * (Gv[D + 1] - uG + H(0.5) * U2 * Gv[0]);
        Fout[D + 1] = Fout[D + 1] + pfix * q;
    }
    return 0;
}

}  // namespace gks
