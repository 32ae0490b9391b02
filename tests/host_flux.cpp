// host_flux.cpp -- the HIP library's face flux (gks_flux.hpp) built for the host with plain
// arithmetic, behind one C entry point, so that CPU tests can set it beside the oracle's
// face flux.  TEST INFRASTRUCTURE ONLY: nothing in the library or the oracle uses it.
#define GKS_HD
#include <cmath>
using std::copysign;
using std::erfc;
using std::exp;
using std::fabs;
using std::fmin;
using std::sqrt;
#include "gks_flux.hpp"

namespace {
template <typename R, int D, int MODE>
int run(const double* gp, const double* const* a, const double* sc, double* F, bool source = false)
{
    constexpr int NV = D + 2;
    gks::FaceIn<D, double> in;
    for (int m = 0; m < NV; ++m) {
        in.Wl[m] = a[0][m];
        in.Wr[m] = a[1][m];
        in.sl[m] = a[2][m];
        in.sr[m] = a[3][m];
        in.Wi[m] = a[4][m];
        in.Wi1[m] = a[5][m];
    }
    for (int s = 0; s < D - 1; ++s)
        for (int m = 0; m < NV; ++m) {
            in.tl[s][m] = a[6] ? a[6][s * 5 + m] : 0.0;
            in.tr[s][m] = a[7] ? a[7][s * 5 + m] : 0.0;
        }
    in.idl = 1.0 / sc[0];
    in.idr = 1.0 / sc[1];
    in.kf = sc[2];
    in.wf = sc[3];
    in.Sf = sc[4];
    in.dt = sc[5];
    const double gamma = gp[0], prandtl = gp[1], b = 2.0 / (gamma - 1.0);
    gks::GasC gas{gp[2], gp[3], b, 2.0 / b, 1.0 / b, 1.0 / gp[4], 1.0 / prandtl - 1.0};
    if (!source) return gks::face_flux<R, D, double, MODE>(in, gas, F);
    // the two cells' states through the optional source, with the FaceIn copies spoiled, so
    // that any read of the copies shows in the flux
    for (int m = 0; m < NV; ++m) in.Wi[m] = in.Wi1[m] = std::nan("");
    auto cells = [a](int side, int m) { return a[4 + side][m]; };
    return gks::face_flux<R, D, double, MODE>(in, gas, F, cells);
}

template <typename R, int D>
int by_mode(int mode, const double* gp, const double* const* a, const double* sc, double* F, bool source)
{
    switch (mode) {
    case 0: return run<R, D, 0>(gp, a, sc, F, source);
    case gks::FLUX_TAUHAT: return run<R, D, gks::FLUX_TAUHAT>(gp, a, sc, F, source);
    case gks::FLUX_MULTID: return run<R, D, gks::FLUX_MULTID>(gp, a, sc, F, source);
    default: return run<R, D, gks::FLUX_TAUHAT | gks::FLUX_MULTID>(gp, a, sc, F, source);
    }
}

int any(int dim, int fp32, int mode, const double* gp, const double* const* a, const double* sc, double* F,
        bool source)
{
    if (dim == 2)
        return fp32 ? by_mode<float, 2>(mode, gp, a, sc, F, source) : by_mode<double, 2>(mode, gp, a, sc, F, source);
    return fp32 ? by_mode<float, 3>(mode, gp, a, sc, F, source) : by_mode<double, 3>(mode, gp, a, sc, F, source);
}
}  // namespace

// One face in the face-local frame (normal component first).  gp: gamma, Prandtl, mu, C_a,
// C_mu.  Wl, Wr, sl, sr, Wi, Wi1: nv = dim + 2 values each; tl, tr: tangential gradients of
// the two cells, (dim - 1) rows of 5 (NULL without the multi-dimensional expansion).  sc:
// centre-to-face distances dxl, dxr, face means k, omega, S, step dt.  fp32: the FP32-flux
// form.  mode: bit 0 the tau_hat time weights, bit 2 the multi-dimensional expansion.
// F: the time-integrated flux (nv values).  Returns 0, or 1 for a non-physical state.
extern "C" int hf_face_flux(int dim, int fp32, int mode, const double* gp, const double* Wl, const double* Wr,
                            const double* sl, const double* sr, const double* Wi, const double* Wi1,
                            const double* tl, const double* tr, const double* sc, double* F)
{
    const double* a[8] = {Wl, Wr, sl, sr, Wi, Wi1, tl, tr};
    return any(dim, fp32, mode, gp, a, sc, F, false);
}

// The same face with the two cells' states Wi, Wi1 handed to the flux through its optional
// source (as the 2D tile kernel does for the wider reconstructions) instead of FaceIn.
extern "C" int hf_face_flux_source(int dim, int fp32, int mode, const double* gp, const double* Wl,
                                   const double* Wr, const double* sl, const double* sr, const double* Wi,
                                   const double* Wi1, const double* tl, const double* tr, const double* sc,
                                   double* F)
{
    const double* a[8] = {Wl, Wr, sl, sr, Wi, Wi1, tl, tr};
    return any(dim, fp32, mode, gp, a, sc, F, true);
}
