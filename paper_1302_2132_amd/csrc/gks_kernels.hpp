// gks_kernels.hpp -- gfx950 kernels of the turbulent gas-kinetic step.
//
// One step of every active solve in a tile table is three launches:
//   k_strain  cell tiles: strain-rate magnitude of each cell from central differences
//             of the cell velocities (ghost neighbours synthesised from the BCs), and, in
//             the same launch, the end of the previous step of each solve (below);
//   k_face    face tiles of one (dim, precision) class: minmod reconstruction along the
//             face normal (four cells, ghosts synthesised), then the gas-kinetic flux of
//             gks_flux.hpp, written once per face (structure of arrays per axis);
//   k_update  cell tiles: conservative FP64 update, positivity check, residual partial
//             sums and the CFL rate of the new state, per tile.
// The end of a step (one workgroup per solve: residual, next dt, time, buffer swap) needs
// every update tile, and the next face pass needs its dt; the strain pass needs neither,
// so it shares a launch with it.  k_finish runs the end of the step on its own after the
// last step of a call, so the state the host reads is complete.
// All kernels walk the tile table with a grid-stride loop, so a fixed grid (and a
// captured graph) serves any membership.  Workgroup ids are remapped so that consecutive
// tiles, which share halo cells, land on the same XCD (L2).
//
// The face kernels come in variants (a bit mask V):
//   V_KW  k and omega transported (Inst::kw): the strain pass (k_strain<true>) also derives
//         k, omega and the model's sources of each cell, the face pass adds the fluxes of
//         rho k and rho omega, and the update advances them with point-implicit sinks;
//   V_TH  the degree of rarefaction measured against the resolved time scale tau_hat
//         (face_flux with FLUX_TAUHAT);
//   V_R3  third-order MUSCL face values (reconstruct<.., 1>);
//   V_MD  the multi-dimensional expansion (face_flux with FLUX_MULTID): tangential
//         gradients of the two cells of every face enter the flux (with V_KW and V_TH,
//         not with the higher-order face values);
//   V_W5  fifth-order WENO face values (reconstruct<.., 2>): six stencil cells per face,
//         three ghost layers (with V_KW and V_TH as V_R3 is).
// V = 0 is the plain scheme, untouched by the others.
//
// The table, the solve descriptors and (outside k_finish) the step state are read
// through the constant address space: nothing writes them while these kernels run, so
// their wave-uniform reads compile to scalar loads rather than chains of dependent
// per-lane vector loads.  Ghost cells are chosen with selects, not branches, so that the
// loads of a whole stencil are in flight together.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gks_device.hpp"
#include "gks_flux.hpp"

namespace gks {

template <typename T> using cptr = const __attribute__((address_space(4))) T*;
template <typename T> using cref = const __attribute__((address_space(4))) T&;

// The tile table as the stepping kernels see it (read-only, constant address space).
struct TabC {
    cptr<TabHdr> hdr;
    cptr<Inst> inst;
    cptr<int> cell_prefix, cls_member, cls_prefix;
    __device__ TabC(const void* base, int cap)
    {
        const TabView tv(const_cast<void*>(base), cap);
        hdr = (cptr<TabHdr>)tv.hdr;
        inst = (cptr<Inst>)tv.inst;
        cell_prefix = (cptr<int>)tv.cell_prefix;
        cls_member = (cptr<int>)tv.cls_member;
        cls_prefix = (cptr<int>)tv.cls_prefix;
    }
};

// Step state of a solve, for kernels that do not write the fields they read.
__device__ inline cref<State> state_of(cref<Inst> I) { return *(cptr<State>)I.st; }

// --------------------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------------------
// Tiles of a grid-stride walk, XCD-aware.  Workgroups are dispatched round-robin over the
// 8 XCDs (block b runs on XCD b % 8), and each XCD has its own L2: the tile range is split
// into 8 contiguous parts, part x walked by the blocks of XCD x, so that neighbouring
// tiles, which share halo cells, stay in one L2, and every XCD gets an equal share however
// the grid compares with the tile count.  Grids that are not a multiple of 8 walk the
// plain grid stride.
struct TileWalk {
    int first, end, stride;
};
__device__ inline TileWalk xcd_walk(int total)
{
    const int g = gridDim.x, b = blockIdx.x;
    if (g % 8) return {b, total, g};
    const int per = (total + 7) / 8;
    const int x = b % 8, lo = x * per;
    return {lo + b / 8, min(total, lo + per), g / 8};
}

// index of the member owning `tile` (prefix has count+1 entries, prefix[0] = 0)
__device__ inline int find_member(cptr<int> prefix, int count, int tile)
{
    int lo = 0, hi = count;   // invariant prefix[lo] <= tile < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= tile) lo = mid; else hi = mid;
    }
    return lo;
}

// Interior cell whose value a (possibly ghost) index i along an axis of n cells takes:
// periodic wrap, mirror behind a wall, nearest cell otherwise.
__device__ inline int image_index(int bc, int i, int n)
{
    const bool lo = i < 0;
    const int per = lo ? i + n : i - n;
    const int wal = lo ? -1 - i : 2 * n - 1 - i;
    const int cpy = lo ? 0 : n - 1;
    const int g = bc == BC_PERIODIC ? per : (bc == BC_WALL ? wal : cpy);
    return (i >= 0 && i < n) ? i : g;
}

__device__ inline int cell_index(cref<Inst> I, int i, int j, int k)
{
    return (k * I.n[1] + j) * I.n[0] + i;
}

// Conservative state of cell c (c[d] may be a ghost index in [-2, n+1]; the other
// coordinates are interior).  Ghosts take the boundary condition of axis d: an interior
// image (periodic, wall with the momentum negated, outflow), the fixed state, or the
// fixed profile at the cell's position in the boundary plane.  Source, stride and element
// are selected per lane, then every component is loaded unconditionally (the first NL
// components: all of them, or density and momenta where only velocities are needed).
template <int D, int NL = D + 2>
__device__ inline __attribute__((always_inline)) void load_state(cref<Inst> I, const double* __restrict__ W, int d,
                                                                 const int* c, double* w)
{
    constexpr int NV = NL;
    const int n = I.n[d];
    const int id = c[d];
    const bool hi = id >= n;
    const bool ghost = id < 0 || hi;
    const int bc0 = I.bc[d][0], bc1 = I.bc[d][1];
    const int bc = ghost ? (hi ? bc1 : bc0) : -1;
    int cc[3] = {c[0], c[1], D == 3 ? c[2] : 0};
    cc[d] = image_index(bc, id, n);
    int t = 0, stride = 1;                     // index in the boundary plane
    for (int a = 0; a < D; ++a) {
        if (a == d) continue;
        t += c[a] * stride;
        stride *= I.n[a];
    }
    const double* bd0 = I.bcd[d][0];
    const double* bd1 = I.bcd[d][1];
    const bool fixed = bc == BC_DIRICHLET, prof = bc == BC_PROFILE;
    const double* src = (fixed || prof) ? (hi ? bd1 : bd0) : W;
    const long long step = fixed ? 1 : (prof ? (long long)I.ntan[d] : (long long)I.ncells);
    const long long e = fixed ? 0 : (prof ? (long long)t : (long long)cell_index(I, cc[0], cc[1], cc[2]));
    const bool neg = bc == BC_WALL;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const double v = src[m * step + e];
        w[m] = (m >= 1 && m <= D && neg) ? -v : v;
    }
}

// flat index of the interior image of cell c (only c[d] may be a ghost)
template <int D>
__device__ inline int image_cell(cref<Inst> I, int d, const int* c)
{
    int cc[3] = {c[0], c[1], D == 3 ? c[2] : 0};
    const int bc0 = I.bc[d][0], bc1 = I.bc[d][1];
    cc[d] = image_index(cc[d] < 0 ? bc0 : bc1, cc[d], I.n[d]);
    return cell_index(I, cc[0], cc[1], cc[2]);
}

// State of a cell that may be a ghost along two axes (a corner cell: a tangential
// neighbour of a cell beyond the boundary).  Ghost layers are filled axis by axis: the
// later axis' rule applies to the earlier axis' ghost at the later axis' image (a fixed
// profile indexed by the cell's position clamped into the boundary plane).
template <int D>
__device__ inline void load_state_c(cref<Inst> I, const double* __restrict__ W, const int* c, double* w)
{
    constexpr int NV = D + 2;
    int ga = -1, gb = -1;
    for (int d = 0; d < D; ++d)
        if (c[d] < 0 || c[d] >= I.n[d]) {
            if (ga < 0) ga = d;
            else gb = d;
        }
    if (gb < 0) {
        load_state<D>(I, W, ga < 0 ? 0 : ga, c, w);
        return;
    }
    const bool hi = c[gb] >= I.n[gb];
    const int bc = I.bc[gb][hi ? 1 : 0];
    int ci[3] = {c[0], c[1], D == 3 ? c[2] : 0};
    ci[gb] = image_index(bc, c[gb], I.n[gb]);
    load_state<D>(I, W, ga, ci, w);
    if (bc == BC_WALL) {
        for (int m = 1; m <= D; ++m) w[m] = -w[m];
    } else if (bc == BC_DIRICHLET) {
        for (int m = 0; m < NV; ++m) w[m] = I.bcd[gb][hi ? 1 : 0][m];
    } else if (bc == BC_PROFILE) {
        int t = 0, stride = 1;
        for (int a = 0; a < D; ++a) {
            if (a == gb) continue;
            t += min(max(c[a], 0), I.n[a] - 1) * stride;
            stride *= I.n[a];
        }
        for (int m = 0; m < NV; ++m) w[m] = I.bcd[gb][hi ? 1 : 0][(long long)m * I.ntan[gb] + t];
    }
}

// Tangential gradient of one component of a cell from its neighbours along that axis
// (multi-dimensional expansion): minmod of the one-sided differences on centre distances
// (icm, icp: inverse distances to the lower and upper neighbour).
__device__ inline double tgrad(double wm, double w0, double wp, double icm, double icp)
{
    return minmod((w0 - wm) * icm, (wp - w0) * icp);
}

// --------------------------------------------------------------------------------------
// strain rate
// --------------------------------------------------------------------------------------
// Velocity of a conservative state: u_a = (rho u_a) * (1/rho), the reciprocal rounded once.
// Every strain evaluation forms its neighbours' velocities this way, so that the per-cell
// pass and the z-marching 3D pass give the same strain rate bitwise.
template <int D>
__device__ inline void velocity_of(const double* w, double* u)
{
    const double ir = 1.0 / w[0];
    for (int a = 0; a < D; ++a) u[a] = w[1 + a] * ir;
}

// Strain-rate magnitude sqrt(2 S_ab S_ab) from the velocities of a cell's lower and upper
// neighbours along each axis b (um[b], up[b]) and ih[b] = 1/(xc[i+1] - xc[i-1]): central
// differences du_a/dx_b = (up[b][a] - um[b][a]) ih[b].
// Contraction into multiply-adds is off here, so that the two passes, compiled in
// different contexts, round every operation alike.
template <int D>
__device__ inline double strain_of(const double (*um)[D], const double (*up)[D], const double* ih)
{
#pragma clang fp contract(off)
    double g[3][3];
    for (int b = 0; b < D; ++b)
        for (int a = 0; a < D; ++a) g[a][b] = (up[b][a] - um[b][a]) * ih[b];
    double ss = 0.0;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            const double s = 0.5 * (g[a][b] + g[b][a]);
            ss += s * s;
        }
    return sqrt(2.0 * ss);
}

template <int D>
__device__ inline void strain_cell(cref<Inst> I, int cell)
{
    const double* __restrict__ W = I.W[state_of(I).fresh];
    int c[3];
    c[0] = cell % I.n[0];
    c[1] = (cell / I.n[0]) % I.n[1];
    c[2] = (D == 3) ? cell / (I.n[0] * I.n[1]) : 0;
    double um[D][D], up[D][D], ih[D];
    for (int b = 0; b < D; ++b) {
        double wp[D + 2], wm[D + 2];
        int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
        cp[b] += 1;
        cm[b] -= 1;
        load_state<D, D + 1>(I, W, b, cp, wp);      // density and momenta
        load_state<D, D + 1>(I, W, b, cm, wm);
        velocity_of<D>(wp, up[b]);
        velocity_of<D>(wm, um[b]);
        ih[b] = I.ic2[b][c[b]];
    }
    I.S[cell] = strain_of<D>(um, up, ih);
}

// --------------------------------------------------------------------------------------
// k-omega transport: sources of a cell, fluxes of a face
// --------------------------------------------------------------------------------------
// Coefficients of Wilcox's 2006 k-omega model, the closure whose k and omega enter the
// turbulent relaxation time of the scheme (section on the turbulent relaxation time).
constexpr double KW_BETA_STAR = 0.09;
constexpr double KW_BETA = 0.0708;
constexpr double KW_ALPHA = 13.0 / 25.0;
constexpr double KW_SIGMA_STAR = 0.6;
constexpr double KW_SIGMA = 0.5;
constexpr double KW_SIGMA_DO = 0.125;

// Strain pass of a transported solve: besides the strain-rate magnitude S (as in
// strain_cell), k = rho k / rho, omega = rho omega / rho and rho k / omega of the cell,
// stored for the face and update passes of the step, and the explicit sources
//   Qk = mu_t (S^2 - 2/3 div^2) - 2/3 rho k div,   mu_t = rho k / (omega sqrt(1 + eta^2)),
//   Qw = alpha rho ((S^2 - 2/3 div^2)/sqrt(1 + eta^2) - 2/3 omega div)
//        + sigma_do (rho/omega) grad k . grad omega   (the last term only where positive),
// eta = S/(C_mu omega): alpha (omega/k) times the production of k, written without the
// division by k.  Gradients are central differences over the neighbouring centres; a
// ghost neighbour's k and omega are those of its interior image.  The pass is split into
// kw_grad_axis (the gradients along one axis) and kw_cell_out (the outputs), which the
// per-cell pass (strain_cell_kw) and the z-marching one (k_strain3kw) share.
//
// Gradients along axis b of a cell from its two neighbours there: velocities (up, um),
// k and omega (kp, km, qp, qm), inverse centre distance ih.  Contraction off, so that every
// pass that forms them (per cell or marching) gets the same values, bitwise.
template <int D>
__device__ inline void kw_grad_axis(const double* up, const double* um, double kp, double km, double qp, double qm,
                                    double ih, int b, double (*g)[3], double* gk, double* gw)
{
#pragma clang fp contract(off)
    for (int a = 0; a < D; ++a) g[a][b] = (up[a] - um[a]) * ih;
    gk[b] = (kp - km) * ih;
    gw[b] = (qp - qm) * ih;
}

// The cell's outputs of the transport strain pass from its gradients and its rho, rho k,
// rho omega (contraction off, as kw_grad_axis).
template <int D>
__device__ inline void kw_cell_out(cref<Inst> I, const double (*g)[3], const double* gk, const double* gw, double rho,
                                   double rk, double rw, long long cell)
{
#pragma clang fp contract(off)
    double ss = 0.0, div = 0.0, cross = 0.0;
    for (int a = 0; a < D; ++a) {
        div += g[a][a];
        cross += gk[a] * gw[a];
        for (int b = 0; b < D; ++b) {
            const double s = 0.5 * (g[a][b] + g[b][a]);
            ss += s * s;
        }
    }
    const double s2 = 2.0 * ss, S = sqrt(s2);
    const double kc = rk / rho, wc = rw / rho;
    const double eta = S / (I.c_mu * wc);
    const double root = sqrt(1.0 + eta * eta);
    const double shear = s2 - (2.0 / 3.0) * div * div;
    const double mut = rho * kc / (wc * root);
    double qw = KW_ALPHA * rho * (shear / root - (2.0 / 3.0) * wc * div);
    if (cross > 0.0) qw += KW_SIGMA_DO * rho / wc * cross;
    I.S[cell] = S;
    I.k[cell] = kc;
    I.om[cell] = wc;
    I.nt[cell] = rho * kc / wc;
    I.Qk[cell] = mut * shear - (2.0 / 3.0) * rho * kc * div;
    I.Qw[cell] = qw;
}

// k and omega of the interior image j of a (possibly ghost) cell: rho k / rho, rho omega / rho
// (a ghost's k and omega are those of its image).
__device__ inline void kw_of_image(const double* __restrict__ W, long long nc, int nv, int j, double& kq, double& wq)
{
    const double r = W[j];
    kq = W[(long long)nv * nc + j] / r;
    wq = W[(long long)(nv + 1) * nc + j] / r;
}

template <int D>
__device__ inline void strain_cell_kw(cref<Inst> I, int cell)
{
    const double* __restrict__ W = I.W[state_of(I).fresh];
    const long long nc = I.ncells;
    int c[3];
    c[0] = cell % I.n[0];
    c[1] = (cell / I.n[0]) % I.n[1];
    c[2] = (D == 3) ? cell / (I.n[0] * I.n[1]) : 0;
    double g[3][3], gk[3], gw[3];
    for (int b = 0; b < D; ++b) {
        double wp[D + 1], wm[D + 1], up[D], um[D];
        int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
        cp[b] += 1;
        cm[b] -= 1;
        load_state<D, D + 1>(I, W, b, cp, wp);      // density and momenta
        load_state<D, D + 1>(I, W, b, cm, wm);
        velocity_of<D>(wp, up);
        velocity_of<D>(wm, um);
        double kp, km, qp, qm;
        kw_of_image(W, nc, D + 2, image_cell<D>(I, b, cp), kp, qp);
        kw_of_image(W, nc, D + 2, image_cell<D>(I, b, cm), km, qm);
        kw_grad_axis<D>(up, um, kp, km, qp, qm, I.ic2[b][c[b]], b, g, gk, gw);
    }
    kw_cell_out<D>(I, g, gk, gw, W[cell], W[(D + 2) * nc + cell], W[(D + 3) * nc + cell], cell);
}

// Time-integrated fluxes of rho k and rho omega through a face: convection by the face's
// time-integrated mass flux frho with the upwind cell's k (omega), and diffusion with the
// coefficient mu + sigma* (sigma for omega) times the mean eddy viscosity rho k/omega
// (nl, nr) of the two cells, over the centre distance (1/icdn).  A ghost's k, omega and
// rho k/omega are those of its interior image.  (A template so that the host can count
// its operations.)
template <typename T>
__host__ __device__ inline void kw_face_t(T mu, T frho, T kl, T kr, T wl, T wr, T nl, T nr, T icdn, T dt, T& Fk,
                                          T& Fw)
{
    const T nut = T(0.5) * (nl + nr);
    const bool up = frho >= T(0.0);
    Fk = frho * (up ? kl : kr) - dt * (mu + T(KW_SIGMA_STAR) * nut) * (kr - kl) * icdn;
    Fw = frho * (up ? wl : wr) - dt * (mu + T(KW_SIGMA) * nut) * (wr - wl) * icdn;
}

__device__ inline void kw_face(cref<Inst> I, double frho, double kl, double kr, double wl, double wr, double nl,
                               double nr, double icdn, double dt, double& Fk, double& Fw)
{
    kw_face_t<double>(I.mu, frho, kl, kr, wl, wr, nl, nr, icdn, dt, Fk, Fw);
}

// --------------------------------------------------------------------------------------
// face fluxes
// --------------------------------------------------------------------------------------
// Flux through the face at position i (0..n) along axis DIR from its four stencil cells
// Wc (i-2 .. i+1, ghosts already synthesised); k, omega and strain rate are averaged over
// elements il, ir of the arrays kk, ww, ss (HBM or LDS: P is the pointer type).  Fg
// receives the time-integrated flux with the momentum components in the global axis
// order, in FP64 in both precision forms (the FP32-flux form keeps the parts of size
// p dt in FP64, see face_flux).  Returns nonzero for a non-physical state.  The axis is a
// template parameter so that every index and the rotation to the face-local frame are
// compile-time (no private arrays).
enum { V_KW = 1, V_TH = 2, V_R3 = 4, V_MD = 8, V_W5 = 16 };

// reconstruction of a variant (0 second-order MUSCL, 1 third-order MUSCL, 2 WENO5) and the
// number of stencil cells on each side of a face (three for WENO5, else two)
template <int V> constexpr int recon_of() { return (V & V_W5) ? 2 : ((V & V_R3) ? 1 : 0); }
template <int V> constexpr int halo_of() { return (V & V_W5) ? 3 : 2; }

// tg_l, tg_r: with FLUX_MULTID, the tangential gradients of the two cells, [(D-1) x (D+2)]
// in the global component order, tangential axes in increasing order.
template <typename R, int D, int DIR, int MODE, int RK, typename P, typename SW, typename CS = InCells>
__device__ __attribute__((always_inline)) inline int face_eval_s(cref<Inst> I, int i, const SW& Wc, P kk, P ww, P ss,
                                                                 int il, int ir, double dt, double* Fg,
                                                                 const double* tg_l = nullptr,
                                                                 const double* tg_r = nullptr, const CS& cs = CS())
{
    constexpr int NV = D + 2;
    FaceGeo<double> geo;
    {
        const double* __restrict__ icd = I.icd[DIR];
        geo.icd[0] = icd[i - 2];
        geo.icd[1] = icd[i - 1];
        geo.icd[2] = icd[i];
        const double* __restrict__ fg = I.fgeo[DIR] + 4 * i;
        geo.dl = fg[0];
        geo.dr = fg[1];
        geo.idl = fg[2];
        geo.idr = fg[3];
    }
    FaceIn<D, double> in;
    reconstruct_s<D, double, RK>(Wc, geo, in);

    // face-local frame: normal momentum first, then the remaining axes in order
    constexpr int P1 = DIR == 0 ? 1 : 0;             // first tangential axis
    constexpr int P2 = DIR == 2 ? 1 : 2;             // second tangential axis (3D)
    if (DIR != 0) {
        double* v[6] = {in.Wl, in.Wr, in.sl, in.sr, in.Wi, in.Wi1};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const double mn = v[q][1 + DIR], t1 = v[q][1 + P1];
            double t2 = 0.0;
            if (D == 3) t2 = v[q][1 + P2];
            v[q][1] = mn;
            v[q][2] = t1;
            if (D == 3) v[q][3] = t2;
        }
    }
    if constexpr ((MODE & FLUX_MULTID) != 0) {
        for (int s = 0; s < D - 1; ++s)
            for (int m = 0; m < NV; ++m) {
                const int src = (m == 1) ? 1 + DIR : (m == 2 ? 1 + P1 : (m == 3 && D == 3 ? 1 + P2 : m));
                in.tl[s][m] = tg_l[s * NV + src];
                in.tr[s][m] = tg_r[s * NV + src];
            }
    }
    in.kf = 0.5 * (kk[il] + kk[ir]);
    in.wf = 0.5 * (ww[il] + ww[ir]);
    in.Sf = 0.5 * (ss[il] + ss[ir]);
    in.dt = dt;
    GasC gas{I.mu, I.c_a, I.b, I.two_over_b, I.inv_b, I.inv_cmu, I.pfix};
    double F[NV + ((MODE & FLUX_EPS_OUT) ? 2 : 0)];
    int bad;
    if constexpr (std::is_same<CS, InCells>::value) {
        bad = face_flux<R, D, double, MODE>(in, gas, F);
    } else {
        // cs reads global components; the flux asks for face-local ones
        auto local = [&](int side, int m) {
            return cs(side, m == 1 ? 1 + DIR : (m == 2 ? 1 + P1 : ((m == 3 && D == 3) ? 1 + P2 : m)));
        };
        bad = face_flux<R, D, double, MODE>(in, gas, F, local);
    }
    Fg[0] = F[0];
    Fg[1 + DIR] = F[1];
    Fg[1 + P1] = F[2];
    if (D == 3) Fg[1 + P2] = F[3];
    Fg[D + 1] = F[D + 1];
    if (MODE & FLUX_EPS_OUT) {
        Fg[D + 2] = F[(MODE & FLUX_EPS_OUT) ? D + 2 : 0];
        Fg[D + 3] = F[(MODE & FLUX_EPS_OUT) ? D + 3 : 0];
    }
    return bad;
}

// The same with the stencil in a private array: Wc[o][m], o from -1 (WENO5) to 4.
template <typename R, int D, int DIR, int MODE, int RK, typename P>
__device__ __attribute__((always_inline)) inline int face_eval(cref<Inst> I, int i, const double (*Wc)[D + 2],
                                                               P kk, P ww, P ss, int il, int ir, double dt, double* Fg,
                                                               const double* tg_l = nullptr,
                                                               const double* tg_r = nullptr)
{
    return face_eval_s<R, D, DIR, MODE, RK>(I, i, [Wc](int o, int m) { return Wc[o][m]; }, kk, ww, ss, il, ir, dt,
                                            Fg, tg_l, tg_r);
}

// One face normal to axis DIR, stencil read from the state in HBM, flux written to the
// axis' face-flux array (structure of arrays).
template <typename R, int D, int DIR, int V>
__device__ __attribute__((always_inline)) inline void face_one(cref<Inst> I, int f)
{
    constexpr bool KW = V & V_KW;
    constexpr int NV = D + 2;
    // face coordinates: the face lies on the low side of cell fc along axis DIR
    const int fn0 = I.n[0] + (DIR == 0), fn1 = I.n[1] + (DIR == 1);
    int fc[3];
    fc[0] = f % fn0;
    fc[1] = (f / fn0) % fn1;
    fc[2] = (D == 3) ? f / (fn0 * fn1) : 0;
    const double* __restrict__ W = I.W[state_of(I).parity];

    // Stencil cells i-NS .. i+NS-1 along DIR (cell i = fc, on the face's high side; NS = 2,
    // or 3 for WENO5) and the two cells sharing the face (il, ir).  When every lane's
    // stencil is interior (a wave-uniform test) they are indexed directly; otherwise ghosts
    // come from the boundary conditions.  Wc points at cell i-2.
    constexpr int NS = halo_of<V>();
    double Wx[2 * NS][NV];
    const double(*Wc)[NV] = Wx + (NS - 2);
    int il, ir;
    if (__all(fc[DIR] >= NS && fc[DIR] <= I.n[DIR] - NS)) {
        const int st = DIR == 0 ? 1 : (DIR == 1 ? I.n[0] : I.n[0] * I.n[1]);
        const long long nc = I.ncells;
        ir = cell_index(I, fc[0], fc[1], fc[2]);
        il = ir - st;
#pragma unroll
        for (int o = 0; o < 2 * NS; ++o)
#pragma unroll
            for (int m = 0; m < NV; ++m) Wx[o][m] = W[m * nc + ir + (o - NS) * st];
    } else {
#pragma unroll
        for (int o = 0; o < 2 * NS; ++o) {
            int c[3] = {fc[0], fc[1], fc[2]};
            c[DIR] += o - NS;
            load_state<D>(I, W, DIR, c, Wx[o]);
        }
        int cl[3] = {fc[0], fc[1], fc[2]};
        cl[DIR] -= 1;
        il = image_cell<D>(I, DIR, cl);
        ir = image_cell<D>(I, DIR, fc);
    }
    double F[NV];
    const double* kk = I.k;
    const double* ww = I.om;
    const double* ss = I.S;
    const double dt = state_of(I).dt;
    constexpr int FMODE = ((V & V_TH) ? FLUX_TAUHAT : 0) | ((V & V_MD) ? FLUX_MULTID : 0);
    double tg[2][(D - 1) * NV];
    if constexpr ((V & V_MD) != 0) {
        // tangential gradients of the two cells from their neighbours along each
        // tangential axis (ghosts, corners included, from the boundary conditions)
        for (int side = 0; side < 2; ++side) {
            int cc[3] = {fc[0], fc[1], fc[2]};
            cc[DIR] -= 1 - side;
            for (int s = 0; s < D - 1; ++s) {
                const int a = s == 0 ? (DIR == 0 ? 1 : 0) : (DIR == 2 ? 1 : 2);
                int cp[3] = {cc[0], cc[1], cc[2]}, cm[3] = {cc[0], cc[1], cc[2]};
                cp[a] += 1;
                cm[a] -= 1;
                double wp[NV], wm[NV];
                load_state_c<D>(I, W, cp, wp);
                load_state_c<D>(I, W, cm, wm);
                const double icm = I.icd[a][cc[a] - 1], icp = I.icd[a][cc[a]];
                for (int m = 0; m < NV; ++m) tg[side][s * NV + m] = tgrad(wm[m], Wc[1 + side][m], wp[m], icm, icp);
            }
        }
    }
    if (face_eval<R, D, DIR, FMODE, recon_of<V>()>(I, fc[DIR], Wc, kk, ww, ss, il, ir, dt, F, tg[0], tg[1]))
        atomicOr(&I.st->err, 1);
    double* __restrict__ out = (double*)I.F[DIR];
    const long long nf = I.nface[DIR];   // 64-bit: component offsets m * nf may pass 2^31
    out[f] = F[0];
    out[nf + f] = F[1];
    out[2 * nf + f] = F[2];
    if (D == 3) out[3 * nf + f] = F[3];
    out[(long long)(D + 1) * nf + f] = F[D + 1];
    if (KW) {
        // The two cells' indices are derived again from an opaque copy of the face index,
        // so that neither they nor the cell values are kept live across the flux.
        int g = f;
        asm volatile("" : "+v"(g));
        int gc[3];
        gc[0] = g % fn0;
        gc[1] = (g / fn0) % fn1;
        gc[2] = (D == 3) ? g / (fn0 * fn1) : 0;
        const int jr = image_cell<D>(I, DIR, gc);
        const int fd = gc[DIR];
        gc[DIR] -= 1;
        const int jl = image_cell<D>(I, DIR, gc);
        const double* nt = I.nt;
        double Fk, Fw;
        kw_face(I, F[0], kk[jl], kk[jr], ww[jl], ww[jr], nt[jl], nt[jr], I.icd[DIR][fd - 1], dt, Fk, Fw);
        out[(long long)(D + 2) * nf + f] = Fk;
        out[(long long)(D + 3) * nf + f] = Fw;
    }
}

#ifndef GKS_FACE_WAVES_FP64
#define GKS_FACE_WAVES_FP64 2
#endif
#ifndef GKS_FACE_WAVES_FP32
#define GKS_FACE_WAVES_FP32 3
#endif
// Register budget of the face kernel (instantiated for 3D; 2D steps use k_tile2): at least
// this many waves per SIMD (2 leaves 256 VGPRs per lane for the 3D FP64 flux, 3 leaves 168
// for the FP32 flux, whose FP64 share -- interface state, Euler and collisionless parts --
// needs more than 128; the third-order and WENO5 reconstructions and the
// multi-dimensional expansion take the FP32 form to 2; the multi-dimensional FP64 form
// keeps 2 with a spill of a few values per face, as its tangential gradients stay live
// through the flux).  TILE faces per workgroup (64, 128 or 256: a batch's autotuned shape).
template <typename R, int D, int TILE, int V>
__global__ __launch_bounds__(TILE)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? GKS_FACE_WAVES_FP32 - ((V & (V_MD | V_R3 | V_W5)) ? 1 : 0)
                                                   : GKS_FACE_WAVES_FP64)))
void k_face(const void* __restrict__ table, int cap, int cls)
{
    const TabC tv(table, cap);
    const int count = tv.hdr->ncls[cls];
    const int total = tv.hdr->total_face[cls];
    cptr<int> prefix = tv.cls_prefix + cls * (cap + 1);
    cptr<int> member = tv.cls_member + cls * cap;
    for (TileWalk tw = xcd_walk(total); tw.first < tw.end; tw.first += tw.stride) {
        const int tile = tw.first;
        const int mj = find_member(prefix, count, tile);
        cref<Inst> I = tv.inst[member[mj]];
        // a batch launches each variant present over its class; other variants' tiles pass
        if (I.variant != V || !state_of(I).active) continue;
        int lt = tile - prefix[mj];
        if (lt < I.ntile_face[0]) {
            const int f = lt * TILE + (int)threadIdx.x;
            if (f < I.nface[0]) face_one<R, D, 0, V>(I, f);
            continue;
        }
        lt -= I.ntile_face[0];
        if (D == 2 || lt < I.ntile_face[1]) {
            const int f = lt * TILE + (int)threadIdx.x;
            if (f < I.nface[1]) face_one<R, D, 1, V>(I, f);
            continue;
        }
        lt -= I.ntile_face[1];
        const int f = lt * TILE + (int)threadIdx.x;
        if (f < I.nface[2]) face_one<R, D, (D == 3 ? 2 : 1), V>(I, f);
    }
}

// --------------------------------------------------------------------------------------
// update, reductions and end of step
// --------------------------------------------------------------------------------------
__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Everything the update of one cell reads: old state, the fluxes through its low and high
// faces per axis, inverse widths, k and omega, and with transport (KW) also rho k, rho
// omega, their face fluxes and their sources qk, qw.
template <int D, bool KW = false>
struct CellRead {
    static constexpr int NX = D + 2 + (KW ? 2 : 0);
    double old[NX], fl[D][NX], fh[D][NX], idx[D], kc, wc, qk, qw;
};

template <int D, typename RF, bool KW = false>
__device__ inline void update_read(cref<Inst> I, const double* __restrict__ Wo, int cell, CellRead<D, KW>& x)
{
    constexpr int NV = CellRead<D, KW>::NX;
    int c[3];
    c[0] = cell % I.n[0];
    c[1] = (cell / I.n[0]) % I.n[1];
    c[2] = (D == 3) ? cell / (I.n[0] * I.n[1]) : 0;
#pragma unroll
    for (int d = 0; d < D; ++d) x.idx[d] = I.idx[d][c[d]];
#pragma unroll
    for (int m = 0; m < NV; ++m) x.old[m] = Wo[(long long)m * I.ncells + cell];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int fn0 = I.n[0] + (d == 0), fn1 = I.n[1] + (d == 1);
        const int lo = (c[2] * fn1 + c[1]) * fn0 + c[0];
        const int hi = lo + (d == 0 ? 1 : (d == 1 ? fn0 : fn0 * fn1));
        const long long nf = I.nface[d];
        const RF* __restrict__ F = (const RF*)I.F[d];
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            x.fl[d][m] = double(F[m * nf + lo]);
            x.fh[d][m] = double(F[m * nf + hi]);
        }
    }
    x.kc = I.k[cell];
    x.wc = I.om[cell];
    if (KW) {
        x.qk = I.Qk[cell];
        x.qw = I.Qw[cell];
    }
}

// CFL rate of a cell of conservative state w (flow variables), k/omega `kow` and inverse
// widths idx:  sum_d (|U_d| + c)/dx_d + 2 nu_eff sum_d 1/dx_d^2 with
// nu_eff = (mu/rho + k/omega) max(4/3, gamma/Pr).  False when rho or p is not positive and
// finite, or the rate is not finite (a non-finite k or omega, which the relaxation time
// would otherwise pass on unnoticed).  The end of every step and the initial rate pass both
// use it, so a solve re-initialised from a saved state takes the same time steps, bitwise.
template <int D>
__device__ inline bool cell_rate(cref<Inst> I, const double* w, double kow, const double* idx, double& rate)
{
    double ke = 0.0, U[3];
    const double rho = w[0], irho = 1.0 / rho;
    for (int d = 0; d < D; ++d) { U[d] = w[1 + d] * irho; ke += U[d] * w[1 + d]; }
    const double p = I.two_over_b * (w[D + 1] - 0.5 * ke);
    if (!(rho > 0.0) || !(p > 0.0) || !(rho < 1e300) || !(p < 1e300)) return false;
    const double cs = sqrt(I.gamma * p * irho);
    const double fac = fmax(4.0 / 3.0, I.gamma / I.prandtl);
    const double nu = (I.mu * irho + kow) * fac;
    double r = 0.0, r2s = 0.0;
    for (int d = 0; d < D; ++d) {
        r += (fabs(U[d]) + cs) * idx[d];
        r2s += idx[d] * idx[d];
    }
    rate = r + 2.0 * nu * r2s;
    return rate < 1e300;
}

// New state of one cell (stored when `store`), its squared residual components added to
// r2 (flow variables only), its CFL rate folded into `rate` (max), a non-physical state
// flagged in `bad`.  With transport, rho k and rho omega take their flux differences and
// sources explicitly and their sinks beta* omega rho k, beta omega rho omega point-
// implicitly with the omega the step started from:
//   rho k' = (rho k - flux out + dt Qk) / (1 + dt beta* omega),  likewise for rho omega.
template <int D, bool KW = false>
__device__ inline void update_apply(cref<Inst> I, double* __restrict__ Wn, int cell, bool store,
                                    const CellRead<D, KW>& x, double dt, double idt, double* r2, double& rate,
                                    int& bad)
{
    constexpr int NV = D + 2;
    double w[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        double acc = x.old[m];
#pragma unroll
        for (int d = 0; d < D; ++d) acc -= (x.fh[d][m] - x.fl[d][m]) * x.idx[d];
        w[m] = acc;
        if (store) Wn[(long long)m * I.ncells + cell] = acc;
        const double r = (acc - x.old[m]) * idt;
        r2[m] += store ? r * r : 0.0;
    }
    double kow = x.kc / x.wc;      // k/omega of the new state, for the CFL rate
    if (KW) {
        double ak = x.old[NV], aw = x.old[NV + 1];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ak -= (x.fh[d][NV] - x.fl[d][NV]) * x.idx[d];
            aw -= (x.fh[d][NV + 1] - x.fl[d][NV + 1]) * x.idx[d];
        }
        const double rk = (ak + dt * x.qk) / (1.0 + dt * KW_BETA_STAR * x.wc);
        const double rw = (aw + dt * x.qw) / (1.0 + dt * KW_BETA * x.wc);
        if (!store) return;
        Wn[(long long)NV * I.ncells + cell] = rk;
        Wn[(long long)(NV + 1) * I.ncells + cell] = rw;
        if (!(rk >= 0.0) || !(rw > 0.0) || !(rk < 1e300) || !(rw < 1e300)) { bad = 1; return; }
        kow = rk / rw;
    }
    if (!store) return;
    // positivity and the CFL rate of the new state
    double cr;
    if (!cell_rate<D>(I, w, kow, x.idx, cr)) { bad = 1; return; }
    rate = fmax(rate, cr);
}

// Update of one cell from the face fluxes in HBM: every read first (the compiler cannot
// move a load above a store through another pointer), then the stores.
template <int D, typename RF, bool KW>
__device__ inline void update_cell(cref<Inst> I, int cell, double dt, double* r2, double& rate, int& bad)
{
    const int cur = state_of(I).parity;
    CellRead<D, KW> x;
    update_read<D, RF, KW>(I, I.W[cur], cell, x);
    update_apply<D, KW>(I, I.W[cur ^ 1], cell, true, x, dt, 1.0 / dt, r2, rate, bad);
}

// --------------------------------------------------------------------------------------
// fused 2D step: a tile's fluxes computed into LDS, then the tile's update
// --------------------------------------------------------------------------------------
// A workgroup of T2_THREADS threads owns a tile of T2X x T2Y cells.  It stages the state
// of the tile and its two-cell halo (three with WENO5; no corners: every stencil is
// one-dimensional, except the corner cells the multi-dimensional expansion reads) and k,
// omega, strain rate on a one-cell halo in LDS, synthesising ghosts once; computes the
// (T2X+1) x T2Y x-faces and T2X x (T2Y+1) y-faces of the tile into LDS (one of each per
// thread; faces on the tile edge are also computed by the neighbouring tile); then
// updates its cells from LDS.  Fluxes never go to HBM, and the update needs no launch of
// its own.  The arithmetic of every face and cell is that of k_face and k_update.
constexpr int T2X = 16, T2Y = 15, T2_THREADS = 256;
// Tile shapes of the fused 2D kernel (shape code S): 16 x 15 (the default), 32 x 7 and
// 8 x 28 cells, each with at most one x-face, one y-face and one cell per thread.  A batch's
// autotuner picks one per class for the plain scheme; the options keep 16 x 15.
constexpr int NSHAPE2 = 3;
__host__ __device__ constexpr int tile2_x(int S) { return S == 1 ? 32 : (S == 2 ? 8 : T2X); }
__host__ __device__ constexpr int tile2_y(int S) { return S == 1 ? 7 : (S == 2 ? 28 : T2Y); }
template <int S>
struct Shape2 {
    static constexpr int X = tile2_x(S), Y = tile2_y(S);
    static constexpr int KX = X + 2, KY = Y + 2;                  // k, omega, strain window
    static constexpr int NFX = (X + 1) * Y, NFY = X * (Y + 1);
    static_assert(NFX <= T2_THREADS && NFY <= T2_THREADS && X * Y <= T2_THREADS,
                  "one x-face, one y-face and one cell per thread");
};

// Register budget: 3 waves per SIMD leave 168 VGPRs per lane, enough for the 2D FP64 flux;
// the plain FP32-flux form gets 4 (128 VGPRs), its variants 3 (the transported ones are
// held to 3 by their LDS, six FP64 flux components per face), and the multi-dimensional
// expansion one wave less in both forms.
#ifndef GKS_TILE2_WAVES_FP64
#define GKS_TILE2_WAVES_FP64 3
#endif
#ifndef GKS_TILE2_WAVES_FP32
#define GKS_TILE2_WAVES_FP32 4
#endif

template <typename R, int V, int S = 0>
__global__ __launch_bounds__(T2_THREADS)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? (V == 0 ? GKS_TILE2_WAVES_FP32 : 3) - ((V & V_MD) ? 1 : 0)
                                                   : GKS_TILE2_WAVES_FP64 - ((V & V_MD) ? 1 : 0))))
void k_tile2(const void* __restrict__ table, int cap, int cls)
{
    constexpr int T2X = Shape2<S>::X, T2Y = Shape2<S>::Y;
    constexpr int T2_KX = Shape2<S>::KX, T2_KY = Shape2<S>::KY;
    constexpr int T2_NFX = Shape2<S>::NFX, T2_NFY = Shape2<S>::NFY;
    constexpr bool KW = V & V_KW;
    constexpr bool MD = V & V_MD;
    constexpr int FMODE = ((V & V_TH) ? FLUX_TAUHAT : 0) | (MD ? FLUX_MULTID : 0);
    constexpr int RK = recon_of<V>();
    constexpr int HW = halo_of<V>();             // halo of the state window (3 for WENO5)
    constexpr int WX = T2X + 2 * HW, WY = T2Y + 2 * HW;
    constexpr int NV = 4;
    constexpr int NX = NV + (KW ? 2 : 0);     // with transport: fluxes of rho k, rho omega too
    __shared__ double sW[NV][WX * WY];
    __shared__ double sK[KW ? 4 : 3][T2_KX * T2_KY];   // k, omega, strain rate (, rho k/omega)
    __shared__ double sFx[NX][T2_NFX];
    __shared__ double sFy[NX][T2_NFY];
    __shared__ double sh_sum[5 * 4];
    __shared__ double sh_max[4];
    __shared__ int sh_bad[4];
    const TabC tv(table, cap);
    const int count = tv.hdr->ncls[cls];
    const int total = tv.hdr->total_face[cls];
    cptr<int> prefix = tv.cls_prefix + cls * (cap + 1);
    cptr<int> member = tv.cls_member + cls * cap;
    for (TileWalk tw = xcd_walk(total); tw.first < tw.end; tw.first += tw.stride) {
        const int tile = tw.first;
        // A tile's prologue and staging run at a raised wave priority, so that a workgroup
        // that has just started issues its loads ahead of the flux arithmetic of the other
        // workgroups on its compute unit; the flux passes run at the normal priority.
        __builtin_amdgcn_s_setprio(2);
        // The thread index is made opaque per tile so that the LDS offsets derived from it
        // are recomputed (a few integer operations) rather than kept live across the tile
        // loop, where they would take registers from the flux evaluation.
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, wv = tid >> 6;
        const int mj = find_member(prefix, count, tile);
        cref<Inst> I = tv.inst[member[mj]];
        if (I.variant != V || !state_of(I).active) continue;   // another variant's tile (batches)
        const int lt = tile - prefix[mj];
        const int n0 = I.n[0], n1 = I.n[1];
        const int nbx = (n0 + T2X - 1) / T2X;
        const int x0 = (lt % nbx) * T2X, y0 = (lt / nbx) * T2Y;
        const int tx = min(T2X, n0 - x0), ty = min(T2Y, n1 - y0);
        const int cur = state_of(I).parity;
        const double* __restrict__ W = I.W[cur];
        const double dt = state_of(I).dt;

        // Stage the state window (tile rows with the x halo, tile columns with the y halo;
        // with the multi-dimensional expansion also the four diagonal neighbours of the
        // tile's corner cells, for the tangential gradients of the edge faces' cells) and
        // k, omega and strain rate on the one-cell halo.  Every load of the tile is issued
        // before the first LDS store, so that the tile waits on one round trip to memory
        // rather than one per pass of each loop; a thread with no cell in a pass loads the
        // tile's first cell and stores nothing.
        constexpr int NWI = (WX * WY + T2_THREADS - 1) / T2_THREADS;
        constexpr int NKI = (T2_KX * T2_KY + T2_THREADS - 1) / T2_THREADS;
        constexpr int NKC = KW ? 4 : 3;
        double ws[NWI][NV], ks[NKI][NKC];
        bool wu[NWI], ku[NKI];
        // A tile whose window lies inside the mesh (most tiles) addresses its cells directly;
        // the others take the ghost rules of load_state and image_cell, which give the same
        // values for interior cells.
        const bool inner = x0 >= HW && y0 >= HW && x0 + tx + HW <= n0 && y0 + ty + HW <= n1;
        if (inner) {
            const long long nc = I.ncells;
#pragma unroll
            for (int it = 0; it < NWI; ++it) {
                const int e = tid + it * T2_THREADS;
                const int a = e % WX, b = e / WX;
                const bool row = b >= HW && b < ty + HW && a < tx + 2 * HW;
                const bool col = a >= HW && a < tx + HW && b < ty + 2 * HW;
                const bool corner = MD && (a == HW - 1 || a == tx + HW) && (b == HW - 1 || b == ty + HW);
                wu[it] = e < WX * WY && (row || col || corner);
                const int cell = wu[it] ? (y0 - HW + b) * n0 + x0 - HW + a : y0 * n0 + x0;
#pragma unroll
                for (int m = 0; m < NV; ++m) ws[it][m] = W[(long long)m * nc + cell];
            }
#pragma unroll
            for (int it = 0; it < NKI; ++it) {
                const int e = tid + it * T2_THREADS;
                const int a = e % T2_KX, b = e / T2_KX;
                const bool row = b >= 1 && b < ty + 1 && a < tx + 2;
                const bool col = a >= 1 && a < tx + 1 && b < ty + 2;
                ku[it] = e < T2_KX * T2_KY && (row || col);
                const int ic = ku[it] ? (y0 - 1 + b) * n0 + x0 - 1 + a : y0 * n0 + x0;
                ks[it][0] = I.k[ic];
                ks[it][1] = I.om[ic];
                ks[it][2] = I.S[ic];
                if (KW) ks[it][NKC - 1] = I.nt[ic];
            }
        } else {
#pragma unroll
            for (int it = 0; it < NWI; ++it) {
                const int e = tid + it * T2_THREADS;
                const int a = e % WX, b = e / WX;
                const bool row = b >= HW && b < ty + HW && a < tx + 2 * HW;
                const bool col = a >= HW && a < tx + HW && b < ty + 2 * HW;
                const bool corner = MD && (a == HW - 1 || a == tx + HW) && (b == HW - 1 || b == ty + HW);
                wu[it] = e < WX * WY && (row || col || corner);
                const int c[3] = {wu[it] ? x0 - HW + a : x0, wu[it] ? y0 - HW + b : y0, 0};
                if (MD && wu[it] && corner) {
                    load_state_c<2>(I, W, c, ws[it]);
                } else {
                    const int d = (c[0] < 0 || c[0] >= n0) ? 0 : 1;     // the ghost axis, if any
                    load_state<2>(I, W, d, c, ws[it]);
                }
            }
#pragma unroll
            for (int it = 0; it < NKI; ++it) {
                const int e = tid + it * T2_THREADS;
                const int a = e % T2_KX, b = e / T2_KX;
                const bool row = b >= 1 && b < ty + 1 && a < tx + 2;
                const bool col = a >= 1 && a < tx + 1 && b < ty + 2;
                ku[it] = e < T2_KX * T2_KY && (row || col);
                const int c[3] = {ku[it] ? x0 - 1 + a : x0, ku[it] ? y0 - 1 + b : y0, 0};
                const int d = (c[0] < 0 || c[0] >= n0) ? 0 : 1;
                const int ic = image_cell<2>(I, d, c);
                ks[it][0] = I.k[ic];
                ks[it][1] = I.om[ic];
                ks[it][2] = I.S[ic];
                if (KW) ks[it][NKC - 1] = I.nt[ic];
            }
        }
#pragma unroll
        for (int it = 0; it < NWI; ++it)
            if (wu[it]) {
                const int e = tid + it * T2_THREADS;
#pragma unroll
                for (int m = 0; m < NV; ++m) sW[m][e] = ws[it][m];
            }
#pragma unroll
        for (int it = 0; it < NKI; ++it)
            if (ku[it]) {
                const int e = tid + it * T2_THREADS;
#pragma unroll
                for (int q = 0; q < NKC; ++q) sK[q][e] = ks[it][q];
            }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);

        {   // x-face (i, j): between cells x0+i-1 and x0+i of row y0+j
            const int i = tid % (T2X + 1), j = tid / (T2X + 1);
            if (tid < T2_NFX && i <= tx && j < ty) {
                double Wx[2 * HW][NV];               // cells x0+i-HW .. x0+i+HW-1
#pragma unroll
                for (int o = 0; o < 2 * HW; ++o)
#pragma unroll
                    for (int m = 0; m < NV; ++m) Wx[o][m] = sW[m][(j + HW) * WX + i + o];
                const double(*Wc)[NV] = Wx + (HW - 2);
                const int kl = (j + 1) * T2_KX + i;
                double tg[2][NV];
                if constexpr (MD) {      // y gradients of the two cells of the x-face
                    const double icm = I.icd[1][y0 + j - 1], icp = I.icd[1][y0 + j];
                    for (int side = 0; side < 2; ++side) {
                        const int e0 = (j + HW) * WX + i + HW - 1 + side;
#pragma unroll
                        for (int m = 0; m < NV; ++m)
                            tg[side][m] = tgrad(sW[m][e0 - WX], sW[m][e0], sW[m][e0 + WX], icm, icp);
                    }
                }
                double F[NV];
                int bad;
                if constexpr (RK == 0) {
                    bad = face_eval<R, 2, 0, FMODE, RK>(I, x0 + i, Wc, &sK[0][0], &sK[1][0], &sK[2][0], kl, kl + 1,
                                                        dt, F, tg[0], tg[1]);
                } else {
                    // the wider stencils are read from LDS one component at a time
                    (void)Wc;
                    const int e0 = (j + HW) * WX + i + HW - 2;
                    // The two cells' states are read again from LDS where the flux uses them
                    // (the equilibrium slopes), through an opaque index so that the earlier
                    // reads are not reused: eight values fewer stay live through the flux,
                    // which the wider reconstructions' face values would otherwise spill.
                    auto cells = [&](int side, int m) {
                        int e = e0;
                        asm volatile("" : "+v"(e));
                        return sW[m][e + 1 + side];
                    };
                    bad = face_eval_s<R, 2, 0, FMODE, RK>(I, x0 + i, [&](int o, int m) { return sW[m][e0 + o]; },
                                                          &sK[0][0], &sK[1][0], &sK[2][0], kl, kl + 1, dt, F, tg[0],
                                                          tg[1], cells);
                }
                if (bad) atomicOr(&I.st->err, 1);
                sFx[0][tid] = F[0];
                sFx[1][tid] = F[1];
                sFx[2][tid] = F[2];
                sFx[3][tid] = F[3];
                if (KW) {
                    int q = kl;                  // reloaded, not kept live across the flux
                    asm volatile("" : "+v"(q));
                    double Fk, Fw;
                    kw_face(I, F[0], sK[0][q], sK[0][q + 1], sK[1][q], sK[1][q + 1], sK[KW ? 3 : 0][q],
                            sK[KW ? 3 : 0][q + 1], I.icd[0][x0 + i - 1], dt, Fk, Fw);
                    sFx[NX - 2][tid] = Fk;
                    sFx[NX - 1][tid] = Fw;
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);      // keep the two passes' registers apart
        {   // y-face (i, j): between cells y0+j-1 and y0+j of column x0+i
            const int i = tid % T2X, j = tid / T2X;
            if (tid < T2_NFY && i < tx && j <= ty) {
                double Wx[2 * HW][NV];               // cells y0+j-HW .. y0+j+HW-1
#pragma unroll
                for (int o = 0; o < 2 * HW; ++o)
#pragma unroll
                    for (int m = 0; m < NV; ++m) Wx[o][m] = sW[m][(j + o) * WX + i + HW];
                const double(*Wc)[NV] = Wx + (HW - 2);
                const int kl = j * T2_KX + i + 1;
                double tg[2][NV];
                if constexpr (MD) {      // x gradients of the two cells of the y-face
                    const double icm = I.icd[0][x0 + i - 1], icp = I.icd[0][x0 + i];
                    for (int side = 0; side < 2; ++side) {
                        const int e0 = (j + HW - 1 + side) * WX + i + HW;
#pragma unroll
                        for (int m = 0; m < NV; ++m) tg[side][m] = tgrad(sW[m][e0 - 1], sW[m][e0], sW[m][e0 + 1], icm, icp);
                    }
                }
                double F[NV];
                int bad;
                if constexpr (RK == 0) {
                    bad = face_eval<R, 2, 1, FMODE, RK>(I, y0 + j, Wc, &sK[0][0], &sK[1][0], &sK[2][0], kl,
                                                        kl + T2_KX, dt, F, tg[0], tg[1]);
                } else {
                    (void)Wc;
                    const int e0 = (j + HW - 2) * WX + i + HW;
                    auto cells = [&](int side, int m) {
                        int e = e0;
                        asm volatile("" : "+v"(e));
                        return sW[m][e + (1 + side) * WX];
                    };
                    bad = face_eval_s<R, 2, 1, FMODE, RK>(I, y0 + j, [&](int o, int m) { return sW[m][e0 + o * WX]; },
                                                          &sK[0][0], &sK[1][0], &sK[2][0], kl, kl + T2_KX, dt, F,
                                                          tg[0], tg[1], cells);
                }
                if (bad) atomicOr(&I.st->err, 1);
                sFy[0][tid] = F[0];
                sFy[1][tid] = F[1];
                sFy[2][tid] = F[2];
                sFy[3][tid] = F[3];
                if (KW) {
                    int q = kl;
                    asm volatile("" : "+v"(q));
                    double Fk, Fw;
                    kw_face(I, F[0], sK[0][q], sK[0][q + T2_KX], sK[1][q], sK[1][q + T2_KX],
                            sK[KW ? 3 : 0][q], sK[KW ? 3 : 0][q + T2_KX], I.icd[1][y0 + j - 1], dt, Fk, Fw);
                    sFy[NX - 2][tid] = Fk;
                    sFy[NX - 1][tid] = Fw;
                }
            }
        }
        __syncthreads();

        // update of cell (i, j) of the tile
        double r2[5] = {0, 0, 0, 0, 0};
        double rate = 0.0;
        int bad = 0;
        {
            const int i = tid % T2X, j = tid / T2X;
            const bool own = tid < T2X * T2Y && i < tx && j < ty;
            const int ii = own ? i : 0, jj = own ? j : 0;
            CellRead<2, KW> x;
            const int ew = (jj + HW) * WX + ii + HW, ek = (jj + 1) * T2_KX + ii + 1;
            const int fx = jj * (T2X + 1) + ii, fy = jj * T2X + ii;
            const int cell = (y0 + jj) * n0 + x0 + ii;
#pragma unroll
            for (int m = 0; m < NX; ++m) {
                x.old[m] = m < NV ? sW[m < NV ? m : 0][ew] : W[(long long)m * I.ncells + cell];
                x.fl[0][m] = sFx[m][fx];
                x.fh[0][m] = sFx[m][fx + 1];
                x.fl[1][m] = sFy[m][fy];
                x.fh[1][m] = sFy[m][fy + T2X];
            }
            x.idx[0] = I.idx[0][x0 + ii];
            x.idx[1] = I.idx[1][y0 + jj];
            x.kc = sK[0][ek];
            x.wc = sK[1][ek];
            if (KW) {
                x.qk = I.Qk[cell];
                x.qw = I.Qw[cell];
            }
            update_apply<2, KW>(I, I.W[cur ^ 1], cell, own, x, dt, 1.0 / dt, r2, rate, bad);
        }
        // tile partials in a fixed order
        for (int m = 0; m < NV; ++m) {
            const double s = wave_sum(r2[m]);
            if (lane == 0) sh_sum[m * 4 + wv] = s;
        }
        {
            const double mx = wave_max(rate);
            const int any = __any(bad);
            if (lane == 0) { sh_max[wv] = mx; sh_bad[wv] = any; }
        }
        __syncthreads();
        if (tid == 0) {
            State* st = I.st;                    // every workgroup of the solve writes the same values
            st->fresh = cur ^ 1;
            st->pending = 1;
            double* part = I.part + (long long)lt * PSTRIDE;
            for (int m = 0; m < NV; ++m)
                part[m] = (sh_sum[m * 4 + 0] + sh_sum[m * 4 + 1]) + (sh_sum[m * 4 + 2] + sh_sum[m * 4 + 3]);
            part[5] = fmax(fmax(sh_max[0], sh_max[1]), fmax(sh_max[2], sh_max[3]));
            if (sh_bad[0] | sh_bad[1] | sh_bad[2] | sh_bad[3]) atomicOr(&I.st->err, 1);
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------------------
// fused 3D step: an x-y tile marching along z
// --------------------------------------------------------------------------------------
// A workgroup of T2_THREADS threads owns a column of T3X x T3Y cells over a run of
// I.seg3 planes (fewer at the top; I.nseg3 runs per column).  For each plane k it holds in
// LDS the tile's state on planes k-1 .. k+2 (a ring of four planes), the two-cell x- and
// y-halos of plane k (arms, ghosts synthesised), and k, omega, strain rate of plane k on a
// one-cell halo.  Each thread computes one x-face and one y-face of plane k (fluxes into
// LDS) and the z-face above its own cell; the face below was computed on the previous
// plane and kept in LDS.  Then every thread updates its own cell of plane k.  The z-faces
// are computed once, the x- and y-faces on the tile's side edges twice (by both
// neighbouring tiles); no flux goes to HBM and the update needs no launch of its own.
// Residual sums and the CFL rate accumulate per thread over the run and are reduced once.
// The arithmetic of every face and cell is that of k_face and k_update.  Variants: the
// second- and third-order MUSCL face values with either eps mode (two-cell stencils), with
// frozen or transported k and omega; WENO5 and the multi-dimensional expansion use k_face
// and k_update.  With transport, each cell's update forms the rho k and rho omega fluxes of
// its six faces itself (kw_face, as k_face does, from the face's mass flux in LDS and the
// two cells' k, omega and rho k/omega; a face's pair is formed by both its cells, 18 flops
// each), so the plane's LDS holds no more than the frozen form's.
constexpr int T3X = 16, T3Y = 15;
constexpr int T3_NC = T3X * T3Y;                        // cells per plane of a tile
constexpr int T3_KX = T3X + 2, T3_KY = T3Y + 2;         // k, omega, strain window
template <int V> constexpr bool fused3_variant() { return (V & (V_MD | V_W5)) == 0; }
static_assert(T3_NC <= T2_THREADS, "one z-face and one cell per thread");

#ifndef GKS_TILE3_WAVES_FP64
#define GKS_TILE3_WAVES_FP64 2
#endif
#ifndef GKS_TILE3_WAVES_FP32
#define GKS_TILE3_WAVES_FP32 2
#endif

// LDS of a fused 3D tile.
struct Tile3Lds {
    double R[4][5][T3_NC];           // planes k-1 .. k+2 (slot z & 3)
    double XA[5][T3Y * 4];           // x-halo of plane k: a = -2, -1, tx, tx+1 per row
    double YA[5][T3X * 4];           // y-halo of plane k: b = -2, -1, ty, ty+1 per column
    double K[3][T3_KX * T3_KY];      // k, omega, strain rate of plane k (one-cell halo)
    double Fx[5][(T3X + 1) * T3Y];
    double Fy[5][T3X * (T3Y + 1)];
    double Fz[5][T3_NC];             // z-face below each cell of plane k
};

// Geometry of one fused 3D tile: origin, extent and z-run.
struct Tile3 {
    int x0, y0, tx, ty, z0, z1;
    __device__ bool owns(int t) const { return t < T3_NC && t % T3X < tx && t / T3X < ty; }
};

// Stage the tile's state on plane z (possibly a ghost plane) into its ring slot.
__device__ inline void t3_stage_plane(cref<Inst> I, const Tile3& g, Tile3Lds& L, int t, int z)
{
    if (!g.owns(t)) return;
    const double* __restrict__ W = I.W[state_of(I).parity];
    const int c[3] = {g.x0 + t % T3X, g.y0 + t / T3X, z};
    double w[5];
    load_state<3>(I, W, 2, c, w);
    const int s = (z + 4) & 3;
#pragma unroll
    for (int m = 0; m < 5; ++m) L.R[s][m][t] = w[m];
}

// Stage plane k+2 into the slot of plane k-2 and, on a full plane, the x- and y-halo arms
// and k, omega, S of plane k (one-cell halo).  Every load is issued before the first LDS
// store, so that a plane waits on one round trip to memory rather than one per array; a
// thread with nothing to stage in a part loads an interior cell of the tile and stores
// nothing.
__device__ inline void t3_stage(cref<Inst> I, const Tile3& g, Tile3Lds& L, int t, int k, bool full)
{
    const double* __restrict__ W = I.W[state_of(I).parity];
    constexpr int NKI = (T3_KX * T3_KY + T2_THREADS - 1) / T2_THREADS;
    const int n0 = I.n[0], n1 = I.n[1];
    const long long nc = I.ncells;
    // Planes inside the mesh and tiles whose x-y window lies inside it (most of them)
    // address their cells directly; the others take the ghost rules of load_state and
    // image_cell, which give the same values for interior cells.
    const bool inner = g.x0 >= 2 && g.y0 >= 2 && g.x0 + g.tx + 2 <= n0 && g.y0 + g.ty + 2 <= n1;
    const bool po = g.owns(t);
    double wp[5];
    {
        const int tt = po ? t : 0;
        const int c[3] = {g.x0 + tt % T3X, g.y0 + tt / T3X, k + 2};
        if (k + 2 < I.n[2]) {
            const int cell = (c[2] * n1 + c[1]) * n0 + c[0];
#pragma unroll
            for (int m = 0; m < 5; ++m) wp[m] = W[m * nc + cell];
        } else {
            load_state<3>(I, W, 2, c, wp);
        }
    }
    if (full) {                 // uniform over the workgroup
        const bool xarm = t < 4 * T3Y;
        const int q = xarm ? t : t - 4 * T3Y;
        const int line = q >> 2, s = q & 3;
        const bool au = t < 4 * (T3Y + T3X) && line < (xarm ? g.ty : g.tx);
        double wa[5], ks[NKI][3];
        bool ku[NKI];
        {
            const int off = s < 2 ? s - 2 : s - 2 + (xarm ? g.tx : g.ty);     // -2, -1, t_, t_+1
            const int c[3] = {au ? (xarm ? g.x0 + off : g.x0 + line) : g.x0,
                              au ? (xarm ? g.y0 + line : g.y0 + off) : g.y0, k};
            if (inner) {
                const int cell = (k * n1 + c[1]) * n0 + c[0];
#pragma unroll
                for (int m = 0; m < 5; ++m) wa[m] = W[m * nc + cell];
            } else {
                load_state<3>(I, W, xarm ? 0 : 1, c, wa);
            }
        }
#pragma unroll
        for (int it = 0; it < NKI; ++it) {
            const int e = t + it * T2_THREADS;
            const int a = e % T3_KX, b = e / T3_KX;
            const bool row = b >= 1 && b < g.ty + 1 && a < g.tx + 2;
            const bool colm = a >= 1 && a < g.tx + 1 && b < g.ty + 2;
            ku[it] = e < T3_KX * T3_KY && (row || colm);
            const int c[3] = {ku[it] ? g.x0 - 1 + a : g.x0, ku[it] ? g.y0 - 1 + b : g.y0, k};
            int ic;
            if (inner) {
                ic = (k * n1 + c[1]) * n0 + c[0];
            } else {
                const int d = (c[0] < 0 || c[0] >= n0) ? 0 : 1;
                ic = image_cell<3>(I, d, c);
            }
            ks[it][0] = I.k[ic];
            ks[it][1] = I.om[ic];
            ks[it][2] = I.S[ic];
        }
        if (au) {
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                if (xarm) L.XA[m][q] = wa[m];
                else L.YA[m][q] = wa[m];
            }
        }
#pragma unroll
        for (int it = 0; it < NKI; ++it)
            if (ku[it]) {
                const int e = t + it * T2_THREADS;
                L.K[0][e] = ks[it][0];
                L.K[1][e] = ks[it][1];
                L.K[2][e] = ks[it][2];
            }
    }
    if (po) {
        const int s = (k + 2 + 4) & 3;
#pragma unroll
        for (int m = 0; m < 5; ++m) L.R[s][m][t] = wp[m];
    }
}

// Flux through a face normal to axis `dir` at position `fpos` along it, from its four
// stencil cells Wc already in the face-local component order (normal momentum first), the
// face means of k, omega and strain rate, and the step; F in the face-local order.  The
// axis is a runtime value here (one inlined flux serves the three axes of the fused 3D
// kernel), so only the geometry arrays are selected by it.
template <typename R, int MODE, int RK>
__device__ __attribute__((always_inline)) inline int face_local3(cref<Inst> I, int dir, int fpos,
                                                                 const double (*Wc)[5], double kf, double wf,
                                                                 double Sf, double dt, double* F)
{
    FaceGeo<double> geo;
    {
        const double* __restrict__ icd = I.icd[dir];
        geo.icd[0] = icd[fpos - 2];
        geo.icd[1] = icd[fpos - 1];
        geo.icd[2] = icd[fpos];
        const double* __restrict__ fg = I.fgeo[dir] + 4 * fpos;
        geo.dl = fg[0];
        geo.dr = fg[1];
        geo.idl = fg[2];
        geo.idr = fg[3];
    }
    FaceIn<3, double> in;
    reconstruct<3, double, RK>(Wc, geo, in);
    in.kf = kf;
    in.wf = wf;
    in.Sf = Sf;
    in.dt = dt;
    GasC gas{I.mu, I.c_a, I.b, I.two_over_b, I.inv_b, I.inv_cmu, I.pfix};
    return face_flux<R, 3, double, MODE>(in, gas, F);
}

template <typename R, int V>
__global__ __launch_bounds__(T2_THREADS)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? GKS_TILE3_WAVES_FP32 : GKS_TILE3_WAVES_FP64)))
void k_tile3(const void* __restrict__ table, int cap, int cls)
{
    static_assert(fused3_variant<V>(), "variant without a fused 3D step");
    constexpr int FMODE = (V & V_TH) ? FLUX_TAUHAT : 0;
    constexpr bool KW = (V & V_KW) != 0;
    constexpr int RK = recon_of<V>();
    constexpr int NV = 5;
    __shared__ Tile3Lds L;
    __shared__ double sh_sum[5 * 4];
    __shared__ double sh_max[4];
    __shared__ int sh_bad[4];
    const TabC tv(table, cap);
    const int count = tv.hdr->ncls[cls];
    const int total = tv.hdr->total_face[cls];
    cptr<int> prefix = tv.cls_prefix + cls * (cap + 1);
    cptr<int> member = tv.cls_member + cls * cap;
    for (TileWalk tw = xcd_walk(total); tw.first < tw.end; tw.first += tw.stride) {
        const int tile = tw.first;
        const int mj = find_member(prefix, count, tile);
        const int mi = member[mj];
        {
            cref<Inst> I = tv.inst[mi];
            if (I.variant != V || !state_of(I).active) continue;   // another variant's tile (batches)
        }
        const int lt = tile - prefix[mj];
        Tile3 g;
        int cur;
        {
            cref<Inst> I = tv.inst[mi];
            const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
            const int ntx = (n0 + T3X - 1) / T3X, nty = (n1 + T3Y - 1) / T3Y;
            const int col = lt % (ntx * nty), seg = lt / (ntx * nty);
            g.x0 = (col % ntx) * T3X;
            g.y0 = (col / ntx) * T3Y;
            g.tx = min(T3X, n0 - g.x0);
            g.ty = min(T3Y, n1 - g.y0);
            g.z0 = seg * I.seg3;
            g.z1 = min(n2, g.z0 + I.seg3);
            cur = state_of(I).parity;
            // planes z0-2 .. z0: the march below first stages z0+1 and makes the z-face under z0
            for (int z = g.z0 - 2; z <= g.z0; ++z) t3_stage_plane(I, g, L, (int)threadIdx.x, z);
        }

        double r2[5] = {0, 0, 0, 0, 0};
        double rate = 0.0;
        int bad = 0;
        // Plane k = z0-1 only makes the z-face under plane z0; every later plane also makes
        // its x- and y-faces and updates its cells.
        for (int k = g.z0 - 1; k < g.z1; ++k) {
            // The member and the thread index are re-read opaquely on every plane, so that
            // the loads of the descriptor and the values derived from the thread index are
            // made again per plane instead of being kept live across the march, where they
            // would take registers from the flux evaluation.
            int mo = mi, t = (int)threadIdx.x;
            asm volatile("" : "+s"(mo));
            asm volatile("" : "+v"(t));
            cref<Inst> I = tv.inst[mo];
            const double dt = state_of(I).dt;
            const bool full = k >= g.z0;

            // plane k+2 into the slot of plane k-2; halo arms and k, omega, S of plane k
            __builtin_amdgcn_s_setprio(2);         // staging ahead of the other workgroup's flux
            t3_stage(I, g, L, t, k, full);
            __syncthreads();
            __builtin_amdgcn_s_setprio(0);

            const int sk = (k + 4) & 3;
            double Fz[NV] = {0, 0, 0, 0, 0};       // z-face above this thread's cell, face-local order
            // one flux evaluation for the three axes: pass 0 the x-face, pass 1 the y-face
            // (both into LDS), pass 2 the z-face above the thread's cell
#pragma unroll 1
            for (int pass = full ? 0 : 2; pass < 3; ++pass) {
                int u = (int)threadIdx.x;
                asm volatile("" : "+v"(u));
                // component order of the face-local frame: rho, normal momentum, the two
                // tangential momenta in axis order, energy
                const int c1 = 1 + pass, c2 = pass == 0 ? 2 : 1, c3 = pass == 2 ? 2 : 3;
                const int comp[NV] = {0, c1, c2, c3, 4};
                bool act;
                int fpos;
                double Wc[4][NV], kf, wf, Sf;
                if (pass == 0) {          // x-face (i, j): between cells x0+i-1 and x0+i of row y0+j
                    const int i = u % (T3X + 1), j = u / (T3X + 1);
                    act = u < (T3X + 1) * T3Y && i <= g.tx && j < g.ty;
                    fpos = g.x0 + i;
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        const int a = i - 2 + o;
                        const bool in = a >= 0 && a < g.tx;
                        const double* src = in ? &L.R[sk][0][j * T3X + (in ? a : 0)]
                                               : &L.XA[0][j * 4 + (a < 0 ? a + 2 : a - g.tx + 2)];
                        const int str = in ? T3_NC : T3Y * 4;
#pragma unroll
                        for (int m = 0; m < NV; ++m) Wc[o][m] = act ? src[comp[m] * str] : 1.0;
                    }
                    const int kl = act ? (j + 1) * T3_KX + i : 0;
                    kf = 0.5 * (L.K[0][kl] + L.K[0][kl + 1]);
                    wf = 0.5 * (L.K[1][kl] + L.K[1][kl + 1]);
                    Sf = 0.5 * (L.K[2][kl] + L.K[2][kl + 1]);
                } else if (pass == 1) {   // y-face (i, j): between cells y0+j-1 and y0+j of column x0+i
                    const int i = u % T3X, j = u / T3X;
                    act = u < T3X * (T3Y + 1) && i < g.tx && j <= g.ty;
                    fpos = g.y0 + j;
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        const int b = j - 2 + o;
                        const bool in = b >= 0 && b < g.ty;
                        const double* src = in ? &L.R[sk][0][(in ? b : 0) * T3X + i]
                                               : &L.YA[0][i * 4 + (b < 0 ? b + 2 : b - g.ty + 2)];
                        const int str = in ? T3_NC : T3X * 4;
#pragma unroll
                        for (int m = 0; m < NV; ++m) Wc[o][m] = act ? src[comp[m] * str] : 1.0;
                    }
                    const int kl = act ? j * T3_KX + i + 1 : 0;
                    kf = 0.5 * (L.K[0][kl] + L.K[0][kl + T3_KX]);
                    wf = 0.5 * (L.K[1][kl] + L.K[1][kl + T3_KX]);
                    Sf = 0.5 * (L.K[2][kl] + L.K[2][kl + T3_KX]);
                } else {                  // z-face between planes k and k+1 of this thread's column
                    act = g.owns(u);
                    fpos = k + 1;
                    const int uu = act ? u : 0;
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        const int s = (k - 1 + o + 4) & 3;
#pragma unroll
                        for (int m = 0; m < NV; ++m) Wc[o][m] = act ? L.R[s][comp[m]][uu] : 1.0;
                    }
                    int cl[3] = {g.x0 + uu % T3X, g.y0 + uu / T3X, k}, cr[3] = {g.x0 + uu % T3X, g.y0 + uu / T3X, k + 1};
                    const int il = image_cell<3>(I, 2, cl), ir = image_cell<3>(I, 2, cr);
                    kf = 0.5 * (I.k[il] + I.k[ir]);
                    wf = 0.5 * (I.om[il] + I.om[ir]);
                    Sf = 0.5 * (I.S[il] + I.S[ir]);
                }
                if (act) {
                    double F[NV];
                    if (face_local3<R, FMODE, RK>(I, pass, fpos, Wc, kf, wf, Sf, dt, F)) atomicOr(&I.st->err, 1);
                    if (pass == 2) {
#pragma unroll
                        for (int m = 0; m < NV; ++m) Fz[m] = F[m];
                    } else {
                        double* out = pass == 0 ? &L.Fx[0][u] : &L.Fy[0][u];
                        const int str = pass == 0 ? (T3X + 1) * T3Y : T3X * (T3Y + 1);
#pragma unroll
                        for (int m = 0; m < NV; ++m) out[comp[m] * str] = F[m];
                    }
                }
            }
            __syncthreads();

            {   // update of this thread's cell on plane k (plane z0-1: keep the z-face only)
                int u = (int)threadIdx.x;
                asm volatile("" : "+v"(u));
                const bool own = g.owns(u);
                // the z-face in global component order (face-local: rho, m_z, m_x, m_y, E)
                const double Fzg[NV] = {Fz[0], Fz[2], Fz[3], Fz[1], Fz[4]};
                if (full) {
                    const int ii = own ? u % T3X : 0, jj = own ? u / T3X : 0;
                    CellRead<3, KW> x;
                    const int fx = jj * (T3X + 1) + ii, fy = jj * T3X + ii, e = jj * T3X + ii;
                    const int cell = (k * I.n[1] + g.y0 + jj) * I.n[0] + g.x0 + ii;
#pragma unroll
                    for (int m = 0; m < NV; ++m) {
                        x.old[m] = L.R[sk][m][e];
                        x.fl[0][m] = L.Fx[m][fx];
                        x.fh[0][m] = L.Fx[m][fx + 1];
                        x.fl[1][m] = L.Fy[m][fy];
                        x.fh[1][m] = L.Fy[m][fy + T3X];
                        x.fl[2][m] = L.Fz[m][e];
                        x.fh[2][m] = Fzg[m];
                    }
                    x.idx[0] = I.idx[0][g.x0 + ii];
                    x.idx[1] = I.idx[1][g.y0 + jj];
                    x.idx[2] = I.idx[2][k];
                    const int ek = (jj + 1) * T3_KX + ii + 1;
                    x.kc = L.K[0][ek];
                    x.wc = L.K[1][ek];
                    if constexpr (KW) {
                        // rho k, rho omega of the cell and their sources; k, omega, rho k/omega
                        // of the six neighbours (x, y: k and omega from the staged window; the
                        // rest from memory, a ghost taking its interior image's)
                        const double* __restrict__ Wo = I.W[cur];
                        const long long nc = I.ncells;
                        x.old[NV] = Wo[(long long)NV * nc + cell];
                        x.old[NV + 1] = Wo[(long long)(NV + 1) * nc + cell];
                        x.qk = I.Qk[cell];
                        x.qw = I.Qw[cell];
                        const int cx = g.x0 + ii, cy = g.y0 + jj;
                        int jn[6];                          // x-1, x+1, y-1, y+1, z-1, z+1
#pragma unroll
                        for (int q = 0; q < 6; ++q) {
                            int c[3] = {cx, cy, k};
                            c[q >> 1] += (q & 1) ? 1 : -1;
                            jn[q] = image_cell<3>(I, q >> 1, c);
                        }
                        const double nc0 = I.nt[cell];
                        double nn[6], kz[2], wz[2];
#pragma unroll
                        for (int q = 0; q < 6; ++q) nn[q] = I.nt[jn[q]];
                        kz[0] = I.k[jn[4]];
                        kz[1] = I.k[jn[5]];
                        wz[0] = I.om[jn[4]];
                        wz[1] = I.om[jn[5]];
                        const double kn[4] = {L.K[0][ek - 1], L.K[0][ek + 1], L.K[0][ek - T3_KX], L.K[0][ek + T3_KX]};
                        const double wn[4] = {L.K[1][ek - 1], L.K[1][ek + 1], L.K[1][ek - T3_KX], L.K[1][ek + T3_KX]};
                        const int cc[3] = {cx, cy, k};
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double klo = d < 2 ? kn[2 * d] : kz[0], khi = d < 2 ? kn[2 * d + 1] : kz[1];
                            const double wlo = d < 2 ? wn[2 * d] : wz[0], whi = d < 2 ? wn[2 * d + 1] : wz[1];
                            const double* __restrict__ icd = I.icd[d];
                            // low face (the neighbour on the left) and high face
                            kw_face(I, x.fl[d][0], klo, x.kc, wlo, x.wc, nn[2 * d], nc0, icd[cc[d] - 1], dt,
                                    x.fl[d][NV], x.fl[d][NV + 1]);
                            kw_face(I, x.fh[d][0], x.kc, khi, x.wc, whi, nc0, nn[2 * d + 1], icd[cc[d]], dt,
                                    x.fh[d][NV], x.fh[d][NV + 1]);
                        }
                    }
                    update_apply<3, KW>(I, I.W[cur ^ 1], cell, own, x, dt, 1.0 / dt, r2, rate, bad);
                }
                if (own) {
#pragma unroll
                    for (int m = 0; m < NV; ++m) L.Fz[m][u] = Fzg[m];   // the face below plane k+1
                }
            }
            __syncthreads();
        }

        // tile partials in a fixed order
        const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
        for (int m = 0; m < NV; ++m) {
            const double s = wave_sum(r2[m]);
            if (lane == 0) sh_sum[m * 4 + wv] = s;
        }
        {
            const double mx = wave_max(rate);
            const int any = __any(bad);
            if (lane == 0) { sh_max[wv] = mx; sh_bad[wv] = any; }
        }
        __syncthreads();
        if (tid == 0) {
            cref<Inst> I = tv.inst[mi];
            State* st = I.st;                    // every workgroup of the solve writes the same values
            st->fresh = cur ^ 1;
            st->pending = 1;
            double* part = I.part + (long long)lt * PSTRIDE;
            for (int m = 0; m < NV; ++m)
                part[m] = (sh_sum[m * 4 + 0] + sh_sum[m * 4 + 1]) + (sh_sum[m * 4 + 2] + sh_sum[m * 4 + 3]);
            part[5] = fmax(fmax(sh_max[0], sh_max[1]), fmax(sh_max[2], sh_max[3]));
            if (sh_bad[0] | sh_bad[1] | sh_bad[2] | sh_bad[3]) atomicOr(&I.st->err, 1);
        }
        __syncthreads();
    }
}

// time step following a state whose max CFL rate is `rate`, and the time it ends at
__device__ inline void next_step(cref<Inst> I, State* st, double rate, double t)
{
    double dt = I.cfl / rate, ta = t + dt;
    if (I.t_end > 0.0) {
        if (t >= I.t_end) st->active = 0;
        else if (ta >= I.t_end) { dt = I.t_end - t; ta = I.t_end; }
    }
    if (!(rate > 0.0) || !(dt > 0.0)) st->active = 0;
    st->dt = dt;
    st->t_after = ta;
}

template <bool KW>
__global__ __launch_bounds__(CELL_TILE) void k_update(const void* __restrict__ table, int cap)
{
    const TabC tv(table, cap);
    const int count = tv.hdr->count;
    const int total = tv.hdr->total_cell;
    __shared__ double sh_sum[5 * 4];
    __shared__ double sh_max[4];
    __shared__ int sh_bad[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (TileWalk tw = xcd_walk(total); tw.first < tw.end; tw.first += tw.stride) {
        const int tile = tw.first;
        const int mi = find_member(tv.cell_prefix, count, tile);
        cref<Inst> I = tv.inst[mi];
        // 2D solves update in k_tile2 and fused 3D solves in k_tile3; a batch launches the
        // transported form separately
        if (I.dim == 2 || I.fused3 || I.kw != (KW ? 1 : 0) || !state_of(I).active) continue;
        const int lt = tile - tv.cell_prefix[mi];
        const int cell = lt * CELL_TILE + (int)threadIdx.x;
        double r2[5] = {0, 0, 0, 0, 0};
        double rate = 0.0;
        int bad = 0;
        const double dt = state_of(I).dt;
        if (cell < I.ncells) update_cell<3, double, KW>(I, cell, dt, r2, rate, bad);
        // workgroup reductions in a fixed order
        for (int m = 0; m < I.nv; ++m) {
            const double s = wave_sum(r2[m]);
            if (lane == 0) sh_sum[m * 4 + wv] = s;
        }
        {
            const double mx = wave_max(rate);
            const int any = __any(bad);
            if (lane == 0) { sh_max[wv] = mx; sh_bad[wv] = any; }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            State* st = I.st;                    // every workgroup of the solve writes the same values
            st->fresh = state_of(I).parity ^ 1;
            st->pending = 1;
            double* part = I.part + (long long)lt * PSTRIDE;
            for (int m = 0; m < I.nv; ++m)
                part[m] = (sh_sum[m * 4 + 0] + sh_sum[m * 4 + 1]) + (sh_sum[m * 4 + 2] + sh_sum[m * 4 + 3]);
            part[5] = fmax(fmax(sh_max[0], sh_max[1]), fmax(sh_max[2], sh_max[3]));
            if (sh_bad[0] | sh_bad[1] | sh_bad[2] | sh_bad[3]) atomicOr(&I.st->err, 1);
        }
        __syncthreads();
    }
}

// Max CFL rate of the current state of each member (first step at init), by the same
// arithmetic as the end of a step: k/omega from the frozen fields, or with transport from
// the state's rho k / rho omega.
template <int D>
__device__ inline bool init_rate(cref<Inst> I, const double* __restrict__ W, int cell, double& rate)
{
    double w[D + 2], idx[D];
    for (int m = 0; m < D + 2; ++m) w[m] = W[(long long)m * I.ncells + cell];
    int c[3];
    c[0] = cell % I.n[0];
    c[1] = (cell / I.n[0]) % I.n[1];
    c[2] = (D == 3) ? cell / (I.n[0] * I.n[1]) : 0;
    for (int d = 0; d < D; ++d) idx[d] = I.idx[d][c[d]];
    double kow;
    if (I.kw) {
        const double rk = W[(long long)(D + 2) * I.ncells + cell], rw = W[(long long)(D + 3) * I.ncells + cell];
        if (!(rk >= 0.0) || !(rw > 0.0) || !(rk < 1e300) || !(rw < 1e300)) return false;
        kow = rk / rw;
    } else {
        kow = I.k[cell] / I.om[cell];
    }
    return cell_rate<D>(I, w, kow, idx, rate);
}

#ifdef GKS_LIB_UNIT   // defined in the library unit only
__global__ __launch_bounds__(CELL_TILE) void k_rate(const void* __restrict__ table, int cap)
{
    const TabC tv(table, cap);
    const int count = tv.hdr->count;
    const int total = tv.hdr->total_cell;
    __shared__ double sh_max[4];
    __shared__ int sh_bad[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (TileWalk tw = xcd_walk(total); tw.first < tw.end; tw.first += tw.stride) {
        const int tile = tw.first;
        const int mi = find_member(tv.cell_prefix, count, tile);
        cref<Inst> I = tv.inst[mi];
        const int lt = tile - tv.cell_prefix[mi];
        const int cell = lt * CELL_TILE + (int)threadIdx.x;
        double rate = 0.0;
        int bad = 0;
        if (cell < I.ncells) {
            const double* W = I.W[state_of(I).parity];
            const bool ok = I.dim == 2 ? init_rate<2>(I, W, cell, rate) : init_rate<3>(I, W, cell, rate);
            if (!ok) { bad = 1; rate = 0.0; }
        }
        const double mx = wave_max(rate);
        const int any = __any(bad);
        if (lane == 0) { sh_max[wv] = mx; sh_bad[wv] = any; }
        __syncthreads();
        if (threadIdx.x == 0) {
            I.part[(long long)lt * PSTRIDE + 5] = fmax(fmax(sh_max[0], sh_max[1]), fmax(sh_max[2], sh_max[3]));
            if (sh_bad[0] | sh_bad[1] | sh_bad[2] | sh_bad[3]) atomicOr(&I.st->err, 1);
        }
        __syncthreads();
    }
}
#else
extern __global__ void k_rate(const void* __restrict__ table, int cap);
#endif

// End of a step (mode 0) or of the initial rate pass (mode 1) of one member, by one
// workgroup: residual from the per-tile partial sums and the CFL rate from the per-tile
// maxima (fixed stride per thread, fixed reduction tree: deterministic), then time,
// buffer swap and the next CFL step.  Runs in a launch after k_update / k_rate, so the
// kernel boundary orders every partial before it.  Loads of four tiles are issued
// together to hide their latency.  `sh` holds 6 x 4 doubles of workgroup scratch.
__device__ inline void finish_member(cref<Inst> I, int mode, double* sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    State* st = I.st;
    if (mode == 0 && !st->pending) return;
    const int nv = I.nv, nt = mode == 0 ? I.nstep_part : I.ntile_cell;
    const int first = mode == 0 ? 0 : 5;    // mode 1 needs the rate only
    double acc[5] = {0, 0, 0, 0, 0}, rmax = 0.0;
    const double* __restrict__ part = I.part;
    for (int t0 = threadIdx.x; t0 < nt; t0 += 4 * CELL_TILE) {
        double v[4][6];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = t0 + q * CELL_TILE;
#pragma unroll
            for (int m = 0; m < 6; ++m)
                v[q][m] = (t < nt && (m >= first) && (m < nv || m == 5)) ? part[(long long)t * PSTRIDE + m] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            for (int m = 0; m < 5; ++m) acc[m] += v[q][m];
            rmax = fmax(rmax, v[q][5]);
        }
    }
    for (int m = 0; m < nv; ++m) {
        const double s = wave_sum(acc[m]);
        if (lane == 0) sh[m * 4 + wv] = s;
    }
    {
        const double s = wave_max(rmax);
        if (lane == 0) sh[5 * 4 + wv] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double rate = fmax(fmax(sh[20], sh[21]), fmax(sh[22], sh[23]));
        if (mode == 1) {
            st->active = 1;
        } else {
            const double N = (double)I.ncells;
            for (int m = 0; m < nv; ++m) {
                const double s = (sh[m * 4 + 0] + sh[m * 4 + 1]) + (sh[m * 4 + 2] + sh[m * 4 + 3]);
                st->res[m] = sqrt(s / N);
            }
            st->dt_last = st->dt;
            st->t = st->t_after;
            st->steps += 1;
            if (st->steps == 1)
                for (int m = 0; m < nv; ++m) st->res_first[m] = st->res[m];
            st->parity ^= 1;
            st->pending = 0;
        }
        next_step(I, st, rate, st->t);
        if (st->err) st->active = 0;
        if (I.max_steps > 0 && st->steps >= I.max_steps) st->active = 0;
        if (I.res_tol > 0.0 && st->steps >= 2) {      // (mode 1: a resumed solve)
            // residual fall of the flow fields whose first-step residual is positive
            double worst = -1.0;
            for (int m = 0; m < nv; ++m)
                if (st->res_first[m] > 0.0) worst = fmax(worst, st->res[m] / st->res_first[m]);
            if (worst >= 0.0 && worst <= I.res_tol) st->active = 0;
        }
    }
    __syncthreads();
}

#ifdef GKS_LIB_UNIT   // defined in the library unit only
__global__ __launch_bounds__(CELL_TILE) void k_finish(const void* __restrict__ table, int cap, int mode)
{
    const TabC tv(table, cap);
    const int count = tv.hdr->count;
    __shared__ double sh[6 * 4];
    for (int mi = blockIdx.x; mi < count; mi += gridDim.x) finish_member(tv.inst[mi], mode, sh);
}
#else
extern __global__ void k_finish(const void* __restrict__ table, int cap, int mode);
#endif

// Strain pass over every cell tile of the table (of active members unless `force`).
// With `finish` set, the first `count` work items instead end the pending step of each
// member (the strain items read W[fresh], which ending a step leaves alone).  DIM = 2
// builds the pass for tables of 2D solves only (a single 2D solve's steps): without the
// 3D path's registers it holds more workgroups per compute unit; DIM = 0 serves any table.
template <bool KW, int DIM = 0>
__global__ __launch_bounds__(CELL_TILE) void k_strain(const void* __restrict__ table, int cap, int force, int finish)
{
    const TabC tv(table, cap);
    const int count = tv.hdr->count;
    const int head = finish ? count : 0;
    const int total = head + tv.hdr->total_cell;
    __shared__ double sh[6 * 4];
    for (TileWalk tw = xcd_walk(total); tw.first < tw.end; tw.first += tw.stride) {
        const int item = tw.first;
        if (item < head) {
            finish_member(tv.inst[item], 0, sh);
            continue;
        }
        const int tile = item - head;
        const int mi = find_member(tv.cell_prefix, count, tile);
        cref<Inst> I = tv.inst[mi];
        if (I.kw != (KW ? 1 : 0) || (!force && !state_of(I).active)) continue;   // the other form's solves
        const int cell = (tile - tv.cell_prefix[mi]) * CELL_TILE + (int)threadIdx.x;
        if (cell >= I.ncells) continue;
        if constexpr (DIM == 2) {
            if (KW) strain_cell_kw<2>(I, cell);
            else strain_cell<2>(I, cell);
        } else if (KW) {
            if (I.dim == 2) strain_cell_kw<2>(I, cell);
            else strain_cell_kw<3>(I, cell);
        } else {
            if (I.dim == 2) strain_cell<2>(I, cell);
            else strain_cell<3>(I, cell);
        }
    }
}

// Strain pass of a single 3D solve with frozen k and omega, marching along z: a workgroup
// owns a 64 x 4 column of cells (a wave per row, so that every load is a contiguous row
// segment) over a run of `seg` planes (`nseg` runs per column).  Each
// thread keeps the velocities of its own column on planes k-1, k, k+1 in registers; the
// velocities of plane k on the column and its one-cell x/y ring (ghost-filled along the
// ring's axis) go through LDS for the x and y differences.  Every cell's state is read
// about 1.3 times (the ring, and two extra planes per run) instead of once per neighbour,
// and the arithmetic is strain_cell's (velocity_of, strain_of): the same strain rate,
// bitwise.  With `finish` set, work item 0 ends the pending step first, as in k_strain.
constexpr int S3X = 64, S3Y = 4;
#ifdef GKS_LIB_UNIT   // defined in the library unit only
__global__ __launch_bounds__(CELL_TILE) void k_strain3(const void* __restrict__ table, int finish, int seg, int nseg)
{
    static_assert(S3X * S3Y == CELL_TILE, "one column per thread");
    constexpr int RX = S3X + 2, RY = S3Y + 2;
    const TabC tv(table, 1);
    cref<Inst> I = tv.inst[0];
    __shared__ double sh[6 * 4];
    __shared__ double sV[3][RX * RY];      // velocities of plane k: column and one-cell ring
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
    const int ntx = (n0 + S3X - 1) / S3X, nty = (n1 + S3Y - 1) / S3Y;
    const int head = finish ? 1 : 0;
    const int total = head + ntx * nty * nseg;
    for (TileWalk tw = xcd_walk(total); tw.first < tw.end; tw.first += tw.stride) {
        const int item = tw.first;
        if (item < head) {
            finish_member(I, 0, sh);
            continue;
        }
        if (!state_of(I).active) continue;
        const double* __restrict__ W = I.W[state_of(I).fresh];
        const int lt = item - head, col = lt % (ntx * nty), run = lt / (ntx * nty);
        const int x0 = (col % ntx) * S3X, y0 = (col / ntx) * S3Y;
        const int tx = min(S3X, n0 - x0), ty = min(S3Y, n1 - y0);
        const int z0 = run * seg, z1 = min(n2, z0 + seg);
        const int t = (int)threadIdx.x, i = t % S3X, j = t / S3X;
        const bool own = i < tx && j < ty;
        const int ci = own ? i : 0, cj = own ? j : 0;
        // the ring cell this thread stages (threads 0 .. 2 (tx + ty) - 1): left, right, bottom, top
        const int nr = 2 * (tx + ty);
        int ra = -1, rb = -1, rd = 0;
        if (t < nr) {
            if (t < ty) { ra = -1; rb = t; rd = 0; }
            else if (t < 2 * ty) { ra = tx; rb = t - ty; rd = 0; }
            else if (t < 2 * ty + tx) { ra = t - 2 * ty; rb = -1; rd = 1; }
            else { ra = t - 2 * ty - tx; rb = ty; rd = 1; }
        }
        auto column = [&](int z, double* u) {      // velocity of this thread's column at plane z
            const int c[3] = {x0 + ci, y0 + cj, z};
            double w[4];
            load_state<3, 4>(I, W, 2, c, w);
            velocity_of<3>(w, u);
        };
        double um[3], uc[3], up[3];
        column(z0 - 1, um);
        column(z0, uc);
        for (int k = z0; k < z1; ++k) {
            column(k + 1, up);
            if (t < nr) {
                const int c[3] = {x0 + ra, y0 + rb, k};
                double w[4], u[3];
                load_state<3, 4>(I, W, rd, c, w);
                velocity_of<3>(w, u);
                const int e = (rb + 1) * RX + ra + 1;
                sV[0][e] = u[0];
                sV[1][e] = u[1];
                sV[2][e] = u[2];
            }
            {
                const int e = (cj + 1) * RX + ci + 1;
                if (own) {
                    sV[0][e] = uc[0];
                    sV[1][e] = uc[1];
                    sV[2][e] = uc[2];
                }
            }
            __syncthreads();
            if (own) {
                const int e = (cj + 1) * RX + ci + 1;
                double vm[3][3], vp[3][3], ih[3];
                for (int a = 0; a < 3; ++a) {
                    vm[0][a] = sV[a][e - 1];
                    vp[0][a] = sV[a][e + 1];
                    vm[1][a] = sV[a][e - RX];
                    vp[1][a] = sV[a][e + RX];
                    vm[2][a] = um[a];
                    vp[2][a] = up[a];
                }
                ih[0] = I.ic2[0][x0 + ci];
                ih[1] = I.ic2[1][y0 + cj];
                ih[2] = I.ic2[2][k];
                I.S[(long long)(k * n1 + y0 + cj) * n0 + x0 + ci] = strain_of<3>(vm, vp, ih);
            }
            __syncthreads();
            for (int a = 0; a < 3; ++a) {
                um[a] = uc[a];
                uc[a] = up[a];
            }
        }
    }
}

// The transport strain pass of a single 3D solve, marching along z like k_strain3: besides
// the velocities, each column carries k and omega of planes k-1, k, k+1 (those of a ghost
// plane from its interior image) and rho, rho k, rho omega of plane k, and the one-cell ring
// of plane k goes through LDS with its velocities, k and omega.  The arithmetic is
// strain_cell_kw's (velocity_of, kw_grad_axis per axis in order, kw_cell_out): the same
// outputs, bitwise.  With `finish` set, work item 0 ends the pending step first.
__global__ __launch_bounds__(CELL_TILE) void k_strain3kw(const void* __restrict__ table, int finish, int seg, int nseg)
{
    static_assert(S3X * S3Y == CELL_TILE, "one column per thread");
    constexpr int RX = S3X + 2, RY = S3Y + 2;
    const TabC tv(table, 1);
    cref<Inst> I = tv.inst[0];
    __shared__ double sh[6 * 4];
    __shared__ double sV[5][RX * RY];      // velocities, k, omega of plane k: column and ring
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
    const long long nc = I.ncells;
    const int ntx = (n0 + S3X - 1) / S3X, nty = (n1 + S3Y - 1) / S3Y;
    const int head = finish ? 1 : 0;
    const int total = head + ntx * nty * nseg;
    for (TileWalk tw = xcd_walk(total); tw.first < tw.end; tw.first += tw.stride) {
        const int item = tw.first;
        if (item < head) {
            finish_member(I, 0, sh);
            continue;
        }
        if (!state_of(I).active) continue;
        const double* __restrict__ W = I.W[state_of(I).fresh];
        const int lt = item - head, col = lt % (ntx * nty), run = lt / (ntx * nty);
        const int x0 = (col % ntx) * S3X, y0 = (col / ntx) * S3Y;
        const int tx = min(S3X, n0 - x0), ty = min(S3Y, n1 - y0);
        const int z0 = run * seg, z1 = min(n2, z0 + seg);
        const int t = (int)threadIdx.x, i = t % S3X, j = t / S3X;
        const bool own = i < tx && j < ty;
        const int ci = own ? i : 0, cj = own ? j : 0;
        const int nr = 2 * (tx + ty);
        int ra = -1, rb = -1, rd = 0;
        if (t < nr) {
            if (t < ty) { ra = -1; rb = t; rd = 0; }
            else if (t < 2 * ty) { ra = tx; rb = t - ty; rd = 0; }
            else if (t < 2 * ty + tx) { ra = t - 2 * ty; rb = -1; rd = 1; }
            else { ra = t - 2 * ty - tx; rb = ty; rd = 1; }
        }
        // velocity, k and omega of this thread's column at plane z (ghost planes: velocity
        // from the ghost state, k and omega from the image), and rho, rho k, rho omega there
        auto column = [&](int z, double* u, double& kq, double& wq, double* raw) {
            const int c[3] = {x0 + ci, y0 + cj, z};
            double w[4];
            load_state<3, 4>(I, W, 2, c, w);
            velocity_of<3>(w, u);
            const int jz = image_cell<3>(I, 2, c);
            raw[0] = W[jz];
            raw[1] = W[5 * nc + jz];
            raw[2] = W[6 * nc + jz];
            kw_of_image(W, nc, 5, jz, kq, wq);
        };
        double um[3], uc[3], up[3], km, kc, kp, wm, wc, wp, rm[3], rc[3], rp[3];
        column(z0 - 1, um, km, wm, rm);
        column(z0, uc, kc, wc, rc);
        for (int k = z0; k < z1; ++k) {
            column(k + 1, up, kp, wp, rp);
            if (t < nr) {
                const int c[3] = {x0 + ra, y0 + rb, k};
                double w[4], u[3], kq, wq;
                load_state<3, 4>(I, W, rd, c, w);
                velocity_of<3>(w, u);
                kw_of_image(W, nc, 5, image_cell<3>(I, rd, c), kq, wq);
                const int e = (rb + 1) * RX + ra + 1;
                sV[0][e] = u[0];
                sV[1][e] = u[1];
                sV[2][e] = u[2];
                sV[3][e] = kq;
                sV[4][e] = wq;
            }
            {
                const int e = (cj + 1) * RX + ci + 1;
                if (own) {
                    sV[0][e] = uc[0];
                    sV[1][e] = uc[1];
                    sV[2][e] = uc[2];
                    sV[3][e] = kc;
                    sV[4][e] = wc;
                }
            }
            __syncthreads();
            if (own) {
                const int e = (cj + 1) * RX + ci + 1;
                double g[3][3], gk[3], gw[3];
                const int off[2] = {1, RX};
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double vp[3] = {sV[0][e + off[b]], sV[1][e + off[b]], sV[2][e + off[b]]};
                    const double vm[3] = {sV[0][e - off[b]], sV[1][e - off[b]], sV[2][e - off[b]]};
                    const double ih = I.ic2[b][b == 0 ? x0 + ci : y0 + cj];
                    kw_grad_axis<3>(vp, vm, sV[3][e + off[b]], sV[3][e - off[b]], sV[4][e + off[b]], sV[4][e - off[b]],
                                    ih, b, g, gk, gw);
                }
                kw_grad_axis<3>(up, um, kp, km, wp, wm, I.ic2[2][k], 2, g, gk, gw);
                kw_cell_out<3>(I, g, gk, gw, rc[0], rc[1], rc[2], (long long)(k * n1 + y0 + cj) * n0 + x0 + ci);
            }
            __syncthreads();
            for (int a = 0; a < 3; ++a) {
                um[a] = uc[a];
                uc[a] = up[a];
                rm[a] = rc[a];
                rc[a] = rp[a];
            }
            km = kc; kc = kp;
            wm = wc; wc = wp;
        }
    }
}
#else
extern __global__ void k_strain3(const void* __restrict__ table, int finish, int seg, int nseg);
extern __global__ void k_strain3kw(const void* __restrict__ table, int finish, int seg, int nseg);
#endif

// Degree of rarefaction eps_hat = tau/tau_hat of the faces of each cell at the current
// state and step (the strain rate, k and omega of that state already in place), largest
// over the cell's 2 D faces, into out[cell] (which = 0), or the faces' relaxation time tau
// (which = 1).  V selects the solve's time weights and reconstruction, so that the
// evaluation is that of the step.  A diagnostic: each face is evaluated by both of its cells.
template <int D, int V>
__device__ inline double cell_eps(cref<Inst> I, int cell, int which)
{
    constexpr int NV = D + 2;
    const double* __restrict__ W = I.W[state_of(I).parity];
    const double dt = state_of(I).dt;
    int c[3];
    c[0] = cell % I.n[0];
    c[1] = (cell / I.n[0]) % I.n[1];
    c[2] = (D == 3) ? cell / (I.n[0] * I.n[1]) : 0;
    double mx = 0.0;
    auto face = [&](auto dirc, int side) {
        constexpr int DIR = decltype(dirc)::value;
        int fc[3] = {c[0], c[1], c[2]};
        fc[DIR] += side;                               // the face lies on the low side of cell fc
        constexpr int NS = halo_of<V>();
        double Wx[2 * NS][NV];
        for (int o = 0; o < 2 * NS; ++o) {
            int cc[3] = {fc[0], fc[1], fc[2]};
            cc[DIR] += o - NS;
            load_state<D>(I, W, DIR, cc, Wx[o]);
        }
        const double(*Wc)[NV] = Wx + (NS - 2);
        int cl[3] = {fc[0], fc[1], fc[2]};
        cl[DIR] -= 1;
        const int il = image_cell<D>(I, DIR, cl), ir = image_cell<D>(I, DIR, fc);
        double F[NV + 2];
        if (face_eval<double, D, DIR, FLUX_EPS_OUT | ((V & V_TH) ? FLUX_TAUHAT : 0), recon_of<V>()>(
                I, fc[DIR], Wc, I.k, I.om, I.S, il, ir, dt, F))
            atomicOr(&I.st->err, 1);
        mx = fmax(mx, which ? F[NV + 1] : F[NV]);
    };
    using D0 = std::integral_constant<int, 0>;
    using D1 = std::integral_constant<int, 1>;
    using D2 = std::integral_constant<int, D == 3 ? 2 : 1>;
    face(D0{}, 0); face(D0{}, 1);
    face(D1{}, 0); face(D1{}, 1);
    if (D == 3) { face(D2{}, 0); face(D2{}, 1); }
    return mx;
}

template <int V>
__global__ __launch_bounds__(64) void k_eps(const void* __restrict__ table, int cap, double* __restrict__ out,
                                            int which)
{
    const TabC tv(table, cap);
    cref<Inst> I = tv.inst[0];
    for (int cell = blockIdx.x * blockDim.x + (int)threadIdx.x; cell < I.ncells; cell += gridDim.x * blockDim.x)
        out[cell] = I.dim == 2 ? cell_eps<2, V>(I, cell, which) : cell_eps<3, V>(I, cell, which);
}

// Copy of every member's step state into one array, so that a batch's states come back
// to the host in one read.
#ifdef GKS_LIB_UNIT   // defined in the library unit only
__global__ __launch_bounds__(64) void k_states(const void* __restrict__ table, int cap, State* __restrict__ out)
{
    const TabC tv(table, cap);
    const int count = tv.hdr->count;
    for (int i = blockIdx.x * blockDim.x + (int)threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const State* __restrict__ st = tv.inst[i].st;
        out[i] = *st;
    }
}
#else
extern __global__ void k_states(const void* __restrict__ table, int cap, State* __restrict__ out);
#endif

// The face-kernel instantiations are defined in the gks_inst_*.hip units, which the build
// compiles in parallel; every other unit sees these declarations only.  GKS_TILE2_VARIANTS
// and GKS_FACE_VARIANTS list every (tile, variant) pair the library launches.
#define GKS_TILE2_VARIANTS(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(16) X(17) X(18) X(19)
#define GKS_FACE_VARIANTS(X) \
    X(64, 8) X(64, 9) X(64, 10) X(64, 11) X(64, 16) X(64, 17) X(64, 18) X(64, 19)
#define GKS_TILE2_DECL(V)                                                         \
    extern template __global__ void k_tile2<double, V, 0>(const void*, int, int); \
    extern template __global__ void k_tile2<float, V, 0>(const void*, int, int);
// the plain scheme's other tile shapes
extern template __global__ void k_tile2<double, 0, 1>(const void*, int, int);
extern template __global__ void k_tile2<float, 0, 1>(const void*, int, int);
extern template __global__ void k_tile2<double, 0, 2>(const void*, int, int);
extern template __global__ void k_tile2<float, 0, 2>(const void*, int, int);
#define GKS_FACE_DECL(T, V)                                                           \
    extern template __global__ void k_face<double, 3, T, V>(const void*, int, int); \
    extern template __global__ void k_face<float, 3, T, V>(const void*, int, int);
#define GKS_TILE3_VARIANTS(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)
#define GKS_TILE3_DECL(V)                                                      \
    extern template __global__ void k_tile3<double, V>(const void*, int, int); \
    extern template __global__ void k_tile3<float, V>(const void*, int, int);
GKS_TILE2_VARIANTS(GKS_TILE2_DECL)
GKS_FACE_VARIANTS(GKS_FACE_DECL)
GKS_TILE3_VARIANTS(GKS_TILE3_DECL)
#undef GKS_TILE2_DECL
#undef GKS_FACE_DECL
#undef GKS_TILE3_DECL

}  // namespace gks
