// gks_lib.hip -- host side of libgks: the C ABI declared in include/gks.h.
//
// Device memory is the caller's: every solve lives in one workspace laid out by
// `layout()`; a batch keeps only its tile table in its own workspace.  Nothing here
// calls hipMalloc.  Host inputs are validated and copied during gks_init.
#include <bitset>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gks.h"
#define GKS_LIB_UNIT
#include "gks_kernels.hpp"

using namespace gks;

namespace gks {
template __global__ void k_eps<0>(const void*, int, double*, int);
template __global__ void k_eps<V_TH>(const void*, int, double*, int);
template __global__ void k_eps<V_R3>(const void*, int, double*, int);
template __global__ void k_eps<V_W5>(const void*, int, double*, int);
template __global__ void k_eps<V_TH | V_W5>(const void*, int, double*, int);
template __global__ void k_eps<V_TH | V_R3>(const void*, int, double*, int);
template __global__ void k_update<false>(const void*, int);
template __global__ void k_update<true>(const void*, int);
template __global__ void k_strain<false>(const void*, int, int, int);
template __global__ void k_strain<true>(const void*, int, int, int);
template __global__ void k_strain<false, 2>(const void*, int, int, int);
template __global__ void k_strain<true, 2>(const void*, int, int, int);
}  // namespace gks

// A named range around an entry point, for the marker traces of profilers (rocprofv3
// --marker-trace shows where the host enqueued which steps); a few nanoseconds when no
// profiler listens.
struct MarkerRange {
    explicit MarkerRange(const char* name) { roctxRangePushA(name); }
    ~MarkerRange() { roctxRangePop(); }
};

namespace {

thread_local std::string g_last_error;

struct Layout {
    size_t W[2], k, om, S, Qk, Qw, nt, F[3], xf[3], xc[3], dx[3], idx[3], ic2[3], icd[3], fgeo[3], bcd[3][2], part, st, tab, total;
    long long ncells, nface[3];
    int ntan[3];
    int ntile_cell, ntile_face[3];
    int ntile2;        // fused 2D tiles (2D only)
    int fused3, seg3, nseg3, ntile3;   // fused 3D step: planes per z-run, runs per column, tiles
    int nstep_part;    // partial slots of a step
};

// fused 2D tiles of an n0 x n1 mesh in tile shape `shape`
static int tiles2(long long n0, long long n1, int shape = 0)
{
    const long long tx = tile2_x(shape), ty = tile2_y(shape);
    return (int)(((n0 + tx - 1) / tx) * ((n1 + ty - 1) / ty));
}

// Options whose 3D step runs in the fused tile kernel (two-cell stencils and face values
// from the cells of the face's own line: not the multi-dimensional expansion or WENO5).
static bool fused3_config(const gks_config* c)
{
    return c->dim == 3 && !c->multi_d && c->recon != GKS_RECON_WENO5;
}

// z-runs of a fused 3D mesh: about 4608 tiles in all (enough rounds of workgroups to keep
// every CU busy to the end), runs of at least four planes.
static void runs3(long long n0, long long n1, long long n2, int* seg, int* nseg)
{
    const long long cols = ((n0 + T3X - 1) / T3X) * ((n1 + T3Y - 1) / T3Y);
    long long ns = std::max<long long>(1, std::min<long long>(n2 / 4, (4608 + cols - 1) / cols));
    const long long s = (n2 + ns - 1) / ns;
    *seg = (int)s;
    *nseg = (int)((n2 + s - 1) / s);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int nvar_of(const gks_config* c) { return c->dim + 2; }
// components of the stored state: the flow variables, then rho k and rho omega when transported
int nstate_of(const gks_config* c) { return c->dim + 2 + (c->turb_transport ? 2 : 0); }

bool config_ok(const gks_config* c, std::string* why)
{
    auto fail = [&](const char* m) { if (why) *why = m; return false; };
    if (!c) return fail("config is NULL");
    if (c->dim != 2 && c->dim != 3) return fail("dim must be 2 or 3");
    for (int d = 0; d < c->dim; ++d) {
        if (c->n[d] < 2) return fail("every axis needs at least 2 cells");
        if (c->n[d] > (1 << 24)) return fail("axis too long");
        if (!c->xf[d]) return fail("face coordinates missing");
        for (long long i = 0; i < c->n[d]; ++i)
            if (!(c->xf[d][i + 1] > c->xf[d][i])) return fail("face coordinates must increase");
        for (int s = 0; s < 2; ++s) {
            const int bc = c->bc[d][s];
            if (bc < GKS_BC_PERIODIC || bc > GKS_BC_OUTFLOW) return fail("unknown boundary condition");
            if ((bc == GKS_BC_DIRICHLET || bc == GKS_BC_PROFILE) && !c->bc_data[d][s])
                return fail("boundary data missing");
        }
        if ((c->bc[d][0] == GKS_BC_PERIODIC) != (c->bc[d][1] == GKS_BC_PERIODIC))
            return fail("periodic boundaries come in pairs");
    }
    long long nc = 1;
    for (int d = 0; d < c->dim; ++d) nc *= c->n[d];
    if (nc > (1ll << 29)) return fail("too many cells");
    if (!(c->gamma > 1.0)) return fail("gamma must exceed 1");
    if (2.0 / (c->gamma - 1.0) < c->dim) return fail("gamma leaves no room for the internal degrees of freedom");
    if (!(c->prandtl > 0.0) || !(c->mu >= 0.0) || !(c->c_a >= 0.0) || !(c->c_mu > 0.0) || !(c->cfl > 0.0) ||
        !(c->t_end >= 0.0))
        return fail("gas or time-step parameter out of range");
    if (c->precision != GKS_FP64 && c->precision != GKS_FP32_FLUX) return fail("unknown precision");
    if (c->max_steps < 0) return fail("max_steps must be >= 0");
    if (!(c->res_tol >= 0.0) || !isfinite(c->res_tol)) return fail("res_tol must be finite and >= 0");
    if (c->turb_transport != 0 && c->turb_transport != 1) return fail("turb_transport must be 0 or 1");
    if (c->eps_mode != GKS_EPS_DT && c->eps_mode != GKS_EPS_TAUHAT) return fail("unknown eps_mode");
    if (c->recon != GKS_RECON_MUSCL2 && c->recon != GKS_RECON_MUSCL3 && c->recon != GKS_RECON_WENO5)
        return fail("unknown reconstruction");
    if (c->multi_d != 0 && c->multi_d != 1) return fail("multi_d must be 0 or 1");
    if (c->multi_d && c->recon != GKS_RECON_MUSCL2)
        return fail("the multi-dimensional expansion takes second-order MUSCL face values");
    if (c->recon == GKS_RECON_WENO5) {
        for (int d = 0; d < c->dim; ++d)
            if (c->n[d] < 3) return fail("WENO5 needs at least 3 cells per axis (three ghost layers)");
    }
    return true;
}

void layout(const gks_config* c, Layout* L)
{
    const int nv = nvar_of(c), nx = nstate_of(c), D = c->dim;
    long long n[3] = {c->n[0], c->n[1], D == 3 ? c->n[2] : 1};
    L->ncells = n[0] * n[1] * n[2];
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
    const size_t cellb = sizeof(double) * (size_t)L->ncells;
    L->W[0] = take(cellb * nx);
    L->W[1] = take(cellb * nx);
    L->k = take(cellb);
    L->om = take(cellb);
    L->S = take(cellb);
    L->Qk = c->turb_transport ? take(cellb) : 0;
    L->Qw = c->turb_transport ? take(cellb) : 0;
    L->nt = c->turb_transport ? take(cellb) : 0;
    const size_t fb = sizeof(double);   // face fluxes are FP64 in both precision forms
    for (int d = 0; d < 3; ++d) {
        L->nface[d] = 0;
        L->ntile_face[d] = 0;
        L->ntan[d] = 1;
        L->F[d] = L->xf[d] = L->xc[d] = L->dx[d] = L->idx[d] = L->ic2[d] = L->icd[d] = L->fgeo[d] = 0;
        L->bcd[d][0] = L->bcd[d][1] = 0;
        if (d >= D) continue;
        L->nface[d] = L->ncells / n[d] * (n[d] + 1);
        L->ntan[d] = (int)(L->ncells / n[d]);
        L->ntile_face[d] = (int)((L->nface[d] + FACE_TILE - 1) / FACE_TILE);
        if (D == 3 && !fused3_config(c)) L->F[d] = take(fb * nx * (size_t)L->nface[d]);   // else in LDS
        L->xf[d] = take(sizeof(double) * (n[d] + 5));
        L->xc[d] = take(sizeof(double) * (n[d] + 4));
        L->dx[d] = take(sizeof(double) * (n[d] + 4));
        L->idx[d] = take(sizeof(double) * (n[d] + 4));
        L->ic2[d] = take(sizeof(double) * n[d]);
        L->icd[d] = take(sizeof(double) * (n[d] + 3));
        L->fgeo[d] = take(sizeof(double) * 4 * (n[d] + 1));
        for (int s = 0; s < 2; ++s) {
            if (c->bc[d][s] == GKS_BC_DIRICHLET) L->bcd[d][s] = take(sizeof(double) * nv);
            else if (c->bc[d][s] == GKS_BC_PROFILE) L->bcd[d][s] = take(sizeof(double) * nv * (size_t)L->ntan[d]);
        }
    }
    L->ntile_cell = (int)((L->ncells + CELL_TILE - 1) / CELL_TILE);
    L->ntile2 = D == 2 ? tiles2(n[0], n[1]) : 0;
    L->fused3 = fused3_config(c) ? 1 : 0;
    L->seg3 = L->nseg3 = L->ntile3 = 0;
    if (L->fused3) {
        runs3(n[0], n[1], n[2], &L->seg3, &L->nseg3);
        L->ntile3 = (int)(((n[0] + T3X - 1) / T3X) * ((n[1] + T3Y - 1) / T3Y)) * L->nseg3;
    }
    L->nstep_part = D == 2 ? L->ntile2 : (L->fused3 ? L->ntile3 : L->ntile_cell);
    // partial slots for the largest tile count a step can make (any 2D tile shape)
    int slots = std::max(L->ntile_cell, L->nstep_part);
    if (D == 2)
        for (int s = 0; s < NSHAPE2; ++s) slots = std::max(slots, tiles2(n[0], n[1], s));
    L->part = take(sizeof(double) * PSTRIDE * (size_t)slots);
    L->st = take(sizeof(State));
    L->tab = take(TabView::bytes(1));
    L->total = off;
}

// extended face coordinates, centres and widths (two ghost layers per side), inverse
// centre-to-centre distances, and per-face centre-to-face distances with their inverses
void metrics(const gks_config* c, int d, std::vector<double>& xf, std::vector<double>& xc, std::vector<double>& dx,
             std::vector<double>& idx, std::vector<double>& ic2, std::vector<double>& icd, std::vector<double>& fgeo)
{
    const long long n = c->n[d];
    const double* f = c->xf[d];
    xf.assign(n + 5, 0.0);
    for (long long i = 0; i <= n; ++i) xf[i + 2] = f[i];
    const bool per = c->bc[d][0] == GKS_BC_PERIODIC;
    for (int m = 1; m <= 2; ++m) {
        xf[2 - m] = per ? f[0] - (f[n] - f[n - m]) : 2.0 * f[0] - f[m];
        xf[n + 2 + m] = per ? f[n] + (f[m] - f[0]) : 2.0 * f[n] - f[n - m];
    }
    xc.assign(n + 4, 0.0);
    dx.assign(n + 4, 0.0);
    for (long long i = 0; i < n + 4; ++i) {
        xc[i] = 0.5 * (xf[i] + xf[i + 1]);
        dx[i] = xf[i + 1] - xf[i];
    }
    idx.assign(n + 4, 0.0);
    for (long long i = 0; i < n + 4; ++i) idx[i] = 1.0 / dx[i];
    ic2.assign(n, 0.0);
    for (long long i = 0; i < n; ++i) ic2[i] = 1.0 / (xc[i + 3] - xc[i + 1]);
    icd.assign(n + 3, 0.0);
    for (long long i = 0; i < n + 3; ++i) icd[i] = 1.0 / (xc[i + 1] - xc[i]);
    fgeo.assign(4 * (n + 1), 0.0);
    for (long long f = 0; f <= n; ++f) {
        const double dl = xf[f + 2] - xc[f + 1], dr = xc[f + 2] - xf[f + 2];
        fgeo[4 * f + 0] = dl;
        fgeo[4 * f + 1] = dr;
        fgeo[4 * f + 2] = 1.0 / dl;
        fgeo[4 * f + 3] = 1.0 / dr;
    }
}

bool state_ok(int D, const double* w, double gamma)
{
    const double rho = w[0];
    double ke = 0.0;
    for (int d = 0; d < D; ++d) ke += w[1 + d] * w[1 + d] / rho;
    const double p = (gamma - 1.0) * (w[D + 1] - 0.5 * ke);
    return rho > 0.0 && p > 0.0 && isfinite(rho) && isfinite(p);
}

}  // namespace

struct gks_ctx {
    gks_config cfg;
    int nv, cls;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    Layout L;
    Inst inst;      // host copy of the device descriptor
    void* tab;      // single-member tile table (device)
    State* st;      // device step state
    std::string err;
    bool broken;
    bool pristine;  // no step taken and in no batch yet: gks_resume is allowed
    int grid_cell, grid_face;
    bool timing;
    hipStream_t batch_stream;         // stream of the batch that last advanced this solve
    std::vector<hipEvent_t> events;   // pool, a start/stop pair per timed launch
    std::vector<int> timed_kind;      // launch kind of each pair: 0 strain, 1 face, 2 update, 3 finish
    size_t events_used;
    long long steps_timed;
};

// What a batch step launches: the face kernel of each (class, variant) pair among the
// members, and the strain and 3D update passes of the frozen and transported forms.
struct Present {
    std::bitset<NCLS * 32> face;      // bit cls * 32 + variant
    bool strain[2] = {false, false};  // frozen, transported
    bool update[2] = {false, false};  // 3D frozen, 3D transported (members outside k_tile3)
    bool covers(const Present& o) const
    {
        return (o.face & ~face).none() && (strain[0] || !o.strain[0]) && (strain[1] || !o.strain[1]) &&
               (update[0] || !o.update[0]) && (update[1] || !o.update[1]);
    }
};

struct gks_batch_ctx {
    std::vector<gks_handle> members;
    int cap;
    hipStream_t stream;
    void* tab;
    int grid[6];
    bool captured;
    int graph_steps;                  // steps one replay of the captured graph advances
    int shape2[2] = {0, 0};           // fused 2D tile shape of the plain scheme, per 2D class
    hipGraph_t graph;
    hipGraphExec_t exec;
    Present present;                  // launches the current (or captured) step makes
    std::vector<char> host_tab;
    std::string err;
    int static_dev = -1;              // device whose static scratch holds the table, or -1
};

static gks_status fail_h(gks_ctx* h, gks_status s, const std::string& msg)
{
    if (h) h->err = msg;
    g_last_error = msg;
    return s;
}

#define HIP_TRY(h, call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail_h((h), GKS_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

// Work on a solve may have been enqueued by a batch on the batch's stream: wait for it
// before the handle's own stream reads the state.
static gks_status sync_batch(gks_ctx* h)
{
    if (h->batch_stream && h->batch_stream != h->stream) HIP_TRY(h, hipStreamSynchronize(h->batch_stream));
    return GKS_OK;
}

static int cls_of(int dim, int precision) { return (dim == 3 ? 2 : 0) + (precision ? 1 : 0); }
static int round8(int n) { return (n + 7) & ~7; }

static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

// Fill a host image of a tile table for `members` (capacity cap): cell tiles of every
// member, and the face-kernel tiles of each class (fused 2D tiles in the class's shape
// shape2[cls] for the plain scheme and 16 x 15 for the options, fused 3D tiles, or
// FACE_TILE faces for the 3D face kernel of the options outside k_tile3).
static void build_table(std::vector<char>& img, int cap, const std::vector<const Inst*>& members,
                        const int* shape2 = nullptr)
{
    img.assign(TabView::bytes(cap), 0);
    TabView tv(img.data(), cap);
    tv.hdr->count = (int)members.size();
    int cells = 0, faces[NCLS] = {0, 0, 0, 0};
    tv.cell_prefix[0] = 0;
    for (int c = 0; c < NCLS; ++c) tv.cls_prefix[c * (cap + 1)] = 0;
    for (size_t i = 0; i < members.size(); ++i) {
        tv.inst[i] = *members[i];
        Inst& I = tv.inst[i];
        if (I.dim == 2) {                        // fused 2D kernel: cell tiles of the class's shape
            I.face_tile = T2_THREADS;
            I.shape2 = (shape2 && I.variant == 0) ? shape2[I.cls] : 0;
            I.ntile_face_all = tiles2(I.n[0], I.n[1], I.shape2);
            I.nstep_part = I.ntile_face_all;
        } else if (I.fused3) {                   // fused 3D kernel: column tiles times z-runs
            I.face_tile = T2_THREADS;
            I.ntile_face_all = ((I.n[0] + T3X - 1) / T3X) * ((I.n[1] + T3Y - 1) / T3Y) * I.nseg3;
        } else {
            const int ft = FACE_TILE;
            I.face_tile = ft;
            I.ntile_face_all = 0;
            for (int d = 0; d < 3; ++d) {
                I.ntile_face[d] = d < I.dim ? (I.nface[d] + ft - 1) / ft : 0;
                I.ntile_face_all += I.ntile_face[d];
            }
        }
        cells += I.ntile_cell;
        tv.cell_prefix[i + 1] = cells;
        const int c = I.cls;
        const int j = tv.hdr->ncls[c]++;
        tv.cls_member[c * cap + j] = (int)i;
        faces[c] += I.ntile_face_all;
        tv.cls_prefix[c * (cap + 1) + j + 1] = faces[c];
    }
    tv.hdr->total_cell = cells;
    for (int c = 0; c < NCLS; ++c) tv.hdr->total_face[c] = faces[c];
}

typedef void (*face_kernel_t)(const void*, int, int);
template <int V>
static face_kernel_t tile2_kernel(int cls)
{
    return cls == 1 ? k_tile2<float, V, 0> : k_tile2<double, V, 0>;
}
// the plain scheme's fused 2D kernel in tile shape `shape`
static face_kernel_t tile2_plain(int cls, int shape)
{
    const bool f = cls == 1;
    if (shape == 1) return f ? k_tile2<float, 0, 1> : k_tile2<double, 0, 1>;
    if (shape == 2) return f ? k_tile2<float, 0, 2> : k_tile2<double, 0, 2>;
    return f ? k_tile2<float, 0, 0> : k_tile2<double, 0, 0>;
}
template <int V>
static face_kernel_t face3_kernel(int cls)
{
    return cls == 3 ? k_face<float, 3, FACE_TILE, V> : k_face<double, 3, FACE_TILE, V>;
}
// Fused 3D kernel of a precision and variant (the variants fused3_config admits).
static face_kernel_t tile3_kernel(int cls, int variant)
{
    const bool f = cls == 3;
    switch (variant) {
    case V_TH: return f ? k_tile3<float, V_TH> : k_tile3<double, V_TH>;
    case V_R3: return f ? k_tile3<float, V_R3> : k_tile3<double, V_R3>;
    case V_TH | V_R3: return f ? k_tile3<float, V_TH | V_R3> : k_tile3<double, V_TH | V_R3>;
    case V_KW: return f ? k_tile3<float, V_KW> : k_tile3<double, V_KW>;
    case V_KW | V_TH: return f ? k_tile3<float, V_KW | V_TH> : k_tile3<double, V_KW | V_TH>;
    case V_KW | V_R3: return f ? k_tile3<float, V_KW | V_R3> : k_tile3<double, V_KW | V_R3>;
    case V_KW | V_TH | V_R3: return f ? k_tile3<float, V_KW | V_TH | V_R3> : k_tile3<double, V_KW | V_TH | V_R3>;
    default: return f ? k_tile3<float, 0> : k_tile3<double, 0>;
    }
}
static bool fused3_variant_rt(int variant) { return (variant & (V_MD | V_W5)) == 0; }

// Face kernel of a class and variant (V_KW and V_TH with one of V_R3, V_W5, V_MD): the
// fused 2D tile kernel for the 2D classes; for 3D the fused tile kernel, or the face kernel
// (FACE_TILE faces per workgroup, then k_update) for WENO5 and the multi-dimensional
// expansion.
static face_kernel_t face_kernel(int cls, int variant, int shape2 = 0)
{
    if (cls >= 2 && fused3_variant_rt(variant)) return tile3_kernel(cls, variant);
    if (cls < 2) {
        switch (variant) {
        case 0: return tile2_plain(cls, shape2);
        case 1: return tile2_kernel<1>(cls);
        case 2: return tile2_kernel<2>(cls);
        case 3: return tile2_kernel<3>(cls);
        case 4: return tile2_kernel<4>(cls);
        case 5: return tile2_kernel<5>(cls);
        case 6: return tile2_kernel<6>(cls);
        case 7: return tile2_kernel<7>(cls);
        case V_MD: return tile2_kernel<V_MD>(cls);
        case V_MD | V_KW: return tile2_kernel<V_MD | V_KW>(cls);
        case V_MD | V_TH: return tile2_kernel<V_MD | V_TH>(cls);
        case V_MD | V_KW | V_TH: return tile2_kernel<V_MD | V_KW | V_TH>(cls);
        case V_W5: return tile2_kernel<V_W5>(cls);
        case V_W5 | V_KW: return tile2_kernel<V_W5 | V_KW>(cls);
        case V_W5 | V_TH: return tile2_kernel<V_W5 | V_TH>(cls);
        case V_W5 | V_KW | V_TH: return tile2_kernel<V_W5 | V_KW | V_TH>(cls);
        default: return tile2_plain(cls, 0);
        }
    }
    switch (variant) {
    case V_MD: return face3_kernel<V_MD>(cls);
    case V_MD | V_KW: return face3_kernel<V_MD | V_KW>(cls);
    case V_MD | V_TH: return face3_kernel<V_MD | V_TH>(cls);
    case V_MD | V_KW | V_TH: return face3_kernel<V_MD | V_KW | V_TH>(cls);
    case V_W5: return face3_kernel<V_W5>(cls);
    case V_W5 | V_KW: return face3_kernel<V_W5 | V_KW>(cls);
    case V_W5 | V_TH: return face3_kernel<V_W5 | V_TH>(cls);
    default: return face3_kernel<V_W5 | V_KW | V_TH>(cls);
    }
}
static int variant_of(const gks_config* c)
{
    return (c->turb_transport ? V_KW : 0) | (c->eps_mode == GKS_EPS_TAUHAT ? V_TH : 0) |
           (c->recon == GKS_RECON_MUSCL3 ? V_R3 : 0) | (c->multi_d ? V_MD : 0) |
           (c->recon == GKS_RECON_WENO5 ? V_W5 : 0);
}
static int face_block(int cls, int variant)
{
    return (cls < 2 || fused3_variant_rt(variant)) ? T2_THREADS : FACE_TILE;
}

extern "C" {

gks_status gks_workspace_bytes(const gks_config* cfg, size_t* bytes)
{
    std::string why;
    if (!bytes) return fail_h(nullptr, GKS_ERR_ARG, "bytes is NULL");
    if (!config_ok(cfg, &why)) return fail_h(nullptr, GKS_ERR_ARG, why);
    Layout L;
    layout(cfg, &L);
    *bytes = L.total;
    return GKS_OK;
}

gks_status gks_init(const gks_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
                    const double* W, const double* k, const double* omega, gks_handle* out)
{
    MarkerRange marker("gks_init");
    std::string why;
    if (!out) return fail_h(nullptr, GKS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!config_ok(cfg, &why)) return fail_h(nullptr, GKS_ERR_ARG, why);
    if (!W || !k || !omega || !dev_workspace) return fail_h(nullptr, GKS_ERR_ARG, "NULL input array");
    if (((uintptr_t)dev_workspace) & 255) return fail_h(nullptr, GKS_ERR_ARG, "workspace must be 256-byte aligned");
    Layout L;
    layout(cfg, &L);
    if (bytes < L.total) return fail_h(nullptr, GKS_ERR_NOMEM, "workspace too small");
    const int nv = nvar_of(cfg), D = cfg->dim;
    const long long N = L.ncells;
    // validate the initial state and the frozen turbulence fields
    for (long long i = 0; i < N; ++i) {
        double w[5];
        for (int m = 0; m < nv; ++m) w[m] = W[m * N + i];
        if (!state_ok(D, w, cfg->gamma)) return fail_h(nullptr, GKS_ERR_NONPHYSICAL, "initial state has rho <= 0 or p <= 0");
        if (!(k[i] >= 0.0) || !isfinite(k[i])) return fail_h(nullptr, GKS_ERR_ARG, "k must be finite and >= 0");
        if (!(omega[i] > 0.0) || !isfinite(omega[i])) return fail_h(nullptr, GKS_ERR_ARG, "omega must be finite and > 0");
    }
    for (int d = 0; d < D; ++d)
        for (int s = 0; s < 2; ++s) {
            const int bc = cfg->bc[d][s];
            if (bc == GKS_BC_DIRICHLET && !state_ok(D, cfg->bc_data[d][s], cfg->gamma))
                return fail_h(nullptr, GKS_ERR_NONPHYSICAL, "Dirichlet state is not physical");
            if (bc == GKS_BC_PROFILE)
                for (int t = 0; t < L.ntan[d]; ++t) {
                    double w[5];
                    for (int m = 0; m < nv; ++m) w[m] = cfg->bc_data[d][s][(long long)m * L.ntan[d] + t];
                    if (!state_ok(D, w, cfg->gamma)) return fail_h(nullptr, GKS_ERR_NONPHYSICAL, "profile state is not physical");
                }
        }

    // owned until the call succeeds: every early return below frees the context
    std::unique_ptr<gks_ctx> owner(new gks_ctx());
    gks_ctx* h = owner.get();
    h->cfg = *cfg;
    for (int d = 0; d < 3; ++d) {
        h->cfg.xf[d] = nullptr;
        h->cfg.bc_data[d][0] = h->cfg.bc_data[d][1] = nullptr;
    }
    h->nv = nv;
    h->cls = cls_of(D, cfg->precision);
    h->stream = (hipStream_t)hip_stream;
    h->ws = (char*)dev_workspace;
    h->ws_bytes = bytes;
    h->L = L;
    h->broken = false;
    h->pristine = true;
    h->timing = false;
    h->batch_stream = nullptr;
    h->events_used = 0;
    h->steps_timed = 0;
    char* ws = h->ws;
    hipStream_t s = h->stream;
    const size_t cellb = sizeof(double) * (size_t)N;

    Inst& I = h->inst;
    memset(&I, 0, sizeof(I));
    I.dim = D;
    I.nv = nv;
    I.precision = cfg->precision;
    I.cls = h->cls;
    I.kw = cfg->turb_transport;
    I.variant = variant_of(cfg);
    for (int d = 0; d < 3; ++d) {
        I.n[d] = d < D ? (int)cfg->n[d] : 1;
        I.ntan[d] = L.ntan[d];
        I.nface[d] = (int)L.nface[d];
        I.ntile_face[d] = L.ntile_face[d];
        for (int sd = 0; sd < 2; ++sd) I.bc[d][sd] = d < D ? cfg->bc[d][sd] : GKS_BC_PERIODIC;
    }
    I.ncells = (int)N;
    I.gamma = cfg->gamma;
    I.prandtl = cfg->prandtl;
    I.mu = cfg->mu;
    I.c_a = cfg->c_a;
    I.c_mu = cfg->c_mu;
    I.cfl = cfg->cfl;
    I.t_end = cfg->t_end;
    I.b = 2.0 / (cfg->gamma - 1.0);
    I.two_over_b = cfg->gamma - 1.0;
    I.inv_b = 1.0 / I.b;
    I.inv_cmu = 1.0 / cfg->c_mu;
    I.pfix = 1.0 / cfg->prandtl - 1.0;
    I.max_steps = cfg->max_steps;
    I.fused3 = L.fused3;
    I.seg3 = L.seg3;
    I.nseg3 = L.nseg3;
    I.res_tol = cfg->res_tol;
    I.W[0] = (double*)(ws + L.W[0]);
    I.W[1] = (double*)(ws + L.W[1]);
    I.k = (double*)(ws + L.k);
    I.om = (double*)(ws + L.om);
    I.S = (double*)(ws + L.S);
    I.Qk = cfg->turb_transport ? (double*)(ws + L.Qk) : nullptr;
    I.Qw = cfg->turb_transport ? (double*)(ws + L.Qw) : nullptr;
    I.nt = cfg->turb_transport ? (double*)(ws + L.nt) : nullptr;
    I.part = (double*)(ws + L.part);
    I.st = (State*)(ws + L.st);
    I.ntile_cell = L.ntile_cell;
    I.nstep_part = L.nstep_part;
    I.face_tile = (D == 2 || L.fused3) ? T2_THREADS : FACE_TILE;
    I.ntile_face_all = D == 2 ? L.ntile2 : (L.fused3 ? L.ntile3 : L.ntile_face[0] + L.ntile_face[1] + L.ntile_face[2]);

    HIP_TRY(h, hipMemcpyAsync(I.W[0], W, cellb * nv, hipMemcpyHostToDevice, s));
    HIP_TRY(h, hipMemcpyAsync((void*)I.k, k, cellb, hipMemcpyHostToDevice, s));
    HIP_TRY(h, hipMemcpyAsync((void*)I.om, omega, cellb, hipMemcpyHostToDevice, s));
    std::vector<double> turb;
    if (cfg->turb_transport) {
        // transported: the state carries rho k and rho omega after the flow variables
        turb.resize(2 * (size_t)N);
        for (long long i = 0; i < N; ++i) {
            turb[i] = W[i] * k[i];
            turb[N + i] = W[i] * omega[i];
        }
        HIP_TRY(h, hipMemcpyAsync(I.W[0] + (size_t)nv * N, turb.data(), 2 * cellb, hipMemcpyHostToDevice, s));
    }
    for (int d = 0; d < D; ++d) {
        std::vector<double> xf, xc, dx, idx, ic2, icd, fgeo;
        metrics(cfg, d, xf, xc, dx, idx, ic2, icd, fgeo);
        I.F[d] = L.F[d] ? (void*)(ws + L.F[d]) : nullptr;
        I.xf[d] = (const double*)(ws + L.xf[d]) + 2;
        I.xc[d] = (const double*)(ws + L.xc[d]) + 2;
        I.dx[d] = (const double*)(ws + L.dx[d]) + 2;
        I.idx[d] = (const double*)(ws + L.idx[d]) + 2;
        I.ic2[d] = (const double*)(ws + L.ic2[d]);
        HIP_TRY(h, hipMemcpyAsync(ws + L.idx[d], idx.data(), sizeof(double) * idx.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ws + L.ic2[d], ic2.data(), sizeof(double) * ic2.size(), hipMemcpyHostToDevice, s));
        I.icd[d] = (const double*)(ws + L.icd[d]) + 2;
        I.fgeo[d] = (const double*)(ws + L.fgeo[d]);
        HIP_TRY(h, hipMemcpyAsync(ws + L.icd[d], icd.data(), sizeof(double) * icd.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ws + L.fgeo[d], fgeo.data(), sizeof(double) * fgeo.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ws + L.xf[d], xf.data(), sizeof(double) * xf.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ws + L.xc[d], xc.data(), sizeof(double) * xc.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ws + L.dx[d], dx.data(), sizeof(double) * dx.size(), hipMemcpyHostToDevice, s));
        for (int sd = 0; sd < 2; ++sd) {
            const int bc = cfg->bc[d][sd];
            if (bc == GKS_BC_DIRICHLET || bc == GKS_BC_PROFILE) {
                const size_t nb = sizeof(double) * nv * (bc == GKS_BC_PROFILE ? (size_t)L.ntan[d] : 1);
                I.bcd[d][sd] = (const double*)(ws + L.bcd[d][sd]);
                HIP_TRY(h, hipMemcpyAsync(ws + L.bcd[d][sd], cfg->bc_data[d][sd], nb, hipMemcpyHostToDevice, s));
            }
        }
    }
    State st0;
    memset(&st0, 0, sizeof(st0));
    st0.active = 1;
    HIP_TRY(h, hipMemcpyAsync(I.st, &st0, sizeof(State), hipMemcpyHostToDevice, s));
    h->st = I.st;
    h->tab = ws + L.tab;
    std::vector<char> img;
    std::vector<const Inst*> mem{&I};
    build_table(img, 1, mem);
    HIP_TRY(h, hipMemcpyAsync(h->tab, img.data(), img.size(), hipMemcpyHostToDevice, s));
    // one workgroup per tile, rounded up to a multiple of the 8 XCDs so that the kernels'
    // walk gives each XCD a contiguous eighth of the tiles (the extra groups find none)
    h->grid_cell = round8(L.ntile_cell);
    h->grid_face = round8(I.ntile_face_all);
    hipLaunchKernelGGL(k_rate, dim3(h->grid_cell), dim3(CELL_TILE), 0, s, (const void*)h->tab, 1);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(CELL_TILE), 0, s, (const void*)h->tab, 1, 1);
    HIP_TRY(h, hipGetLastError());
    State st;
    HIP_TRY(h, hipMemcpyAsync(&st, I.st, sizeof(State), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (st.err) return fail_h(nullptr, GKS_ERR_NONPHYSICAL, "initial state is not physical");
    *out = owner.release();
    return GKS_OK;
}

static gks_status next_event(gks_ctx* h, hipEvent_t* ev)
{
    if (h->events_used == h->events.size()) {
        hipEvent_t e;
        HIP_TRY(h, hipEventCreate(&e));
        h->events.push_back(e);
    }
    *ev = h->events[h->events_used++];
    return GKS_OK;
}

// A 3D step is three launches (strain with the previous step's end folded in, face,
// update); a 2D step two (strain, fused tile kernel).  One trailing k_finish ends the last
// step so the state is complete when the call's work has run.
#ifndef GKS_STRAIN3_ITEMS
#define GKS_STRAIN3_ITEMS 8192     // work items of the z-marching strain pass (columns x runs)
#endif
static gks_status enqueue_steps(gks_ctx* h, int32_t nsteps)
{
    hipStream_t s = h->stream;
    const void* tab = h->tab;
    const bool kw = h->cfg.turb_transport != 0;
    face_kernel_t fk = face_kernel(h->cls, variant_of(&h->cfg));
    const dim3 fblock(face_block(h->cls, variant_of(&h->cfg)));
    const bool upd = h->cfg.dim == 3 && !h->inst.fused3;
    // a single 2D solve's strain pass is built for 2D tables only (fewer registers)
    const bool d2 = h->cfg.dim == 2;
    void (*ks)(const void*, int, int, int) =
        kw ? (d2 ? k_strain<true, 2> : k_strain<true>) : (d2 ? k_strain<false, 2> : k_strain<false>);
    void (*ku)(const void*, int) = kw ? k_update<true> : k_update<false>;
    const int grid_head = round8(h->inst.ntile_cell + 1);
    // a 3D solve takes the z-marching strain pass (runs of planes over 64 x 4 columns, about
    // 8192 work items; with transport the pass that also forms k, omega and the sources), a
    // 2D one the per-cell pass
    const bool strain3 = h->cfg.dim == 3;
    int seg3s = 1, nseg3s = 1, grid3s = 8;
    if (strain3) {
        const int n0 = h->inst.n[0], n1 = h->inst.n[1], n2 = h->inst.n[2];
        const int cols = ((n0 + S3X - 1) / S3X) * ((n1 + S3Y - 1) / S3Y);
        nseg3s = std::max(1, std::min(std::max(1, n2 / 4), (GKS_STRAIN3_ITEMS + cols - 1) / cols));
        seg3s = (n2 + nseg3s - 1) / nseg3s;
        nseg3s = (n2 + seg3s - 1) / seg3s;
        grid3s = round8(1 + cols * nseg3s);
    }
    if (nsteps == 0) return GKS_OK;
    if (!h->timing) {
        for (int i = 0; i < nsteps; ++i) {
            if (strain3) hipLaunchKernelGGL(kw ? k_strain3kw : k_strain3, dim3(grid3s), dim3(CELL_TILE), 0, s, tab, 1,
                                            seg3s, nseg3s);
            else hipLaunchKernelGGL(ks, dim3(grid_head), dim3(CELL_TILE), 0, s, tab, 1, 0, 1);
            hipLaunchKernelGGL(fk, dim3(h->grid_face), fblock, 0, s, tab, 1, h->cls);
            if (upd) hipLaunchKernelGGL(ku, dim3(h->grid_cell), dim3(CELL_TILE), 0, s, tab, 1);
        }
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(CELL_TILE), 0, s, tab, 1, 0);
    } else {
        // timed: the runtime stamps each launch's own start and end into its event pair
        hipEvent_t ev[6];
        for (int i = 0; i < nsteps; ++i) {
            for (int q = 0; q < (upd ? 6 : 4); ++q) {
                gks_status r = next_event(h, &ev[q]);
                if (r != GKS_OK) return r;
            }
            if (strain3)
                hipExtLaunchKernelGGL(kw ? k_strain3kw : k_strain3, dim3(grid3s), dim3(CELL_TILE), 0, s, ev[0], ev[1], 0,
                                      tab, 1, seg3s, nseg3s);
            else
                hipExtLaunchKernelGGL(ks, dim3(grid_head), dim3(CELL_TILE), 0, s, ev[0], ev[1], 0, tab, 1, 0, 1);
            hipExtLaunchKernelGGL(fk, dim3(h->grid_face), fblock, 0, s, ev[2], ev[3], 0, tab, 1, h->cls);
            h->timed_kind.insert(h->timed_kind.end(), {0, 1});
            if (upd) {
                hipExtLaunchKernelGGL(ku, dim3(h->grid_cell), dim3(CELL_TILE), 0, s, ev[4], ev[5], 0, tab, 1);
                h->timed_kind.push_back(2);
            }
            h->steps_timed += 1;
        }
        for (int q = 0; q < 2; ++q) {
            gks_status r = next_event(h, &ev[q]);
            if (r != GKS_OK) return r;
        }
        hipExtLaunchKernelGGL(k_finish, dim3(1), dim3(CELL_TILE), 0, s, ev[0], ev[1], 0, tab, 1, 0);
        h->timed_kind.push_back(3);
    }
    HIP_TRY(h, hipGetLastError());
    return GKS_OK;
}

gks_status gks_step(gks_handle h, int32_t nsteps)
{
    MarkerRange marker("gks_step");
    if (!h) return fail_h(nullptr, GKS_ERR_ARG, "NULL handle");
    if (nsteps < 0) return fail_h(h, GKS_ERR_ARG, "nsteps < 0");
    if (h->broken) return fail_h(h, GKS_ERR_STATE, "handle is in the error state");
    gks_status r = sync_batch(h);
    if (r != GKS_OK) return r;
    if (nsteps > 0) h->pristine = false;
    return enqueue_steps(h, nsteps);
}

static gks_status read_state(gks_ctx* h, State* st)
{
    gks_status r = sync_batch(h);
    if (r != GKS_OK) return r;
    HIP_TRY(h, hipMemcpyAsync(st, h->st, sizeof(State), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (st->err) {
        h->broken = true;
        return fail_h(h, GKS_ERR_NONPHYSICAL, "non-physical state (rho <= 0 or p <= 0 or non-finite)");
    }
    return GKS_OK;
}

gks_status gks_residual(gks_handle h, double* res, double* res_first, double* dt_last, double* t,
                        int64_t* steps_done)
{
    if (!h) return fail_h(nullptr, GKS_ERR_ARG, "NULL handle");
    State st;
    gks_status r = read_state(h, &st);
    if (res) for (int m = 0; m < h->nv; ++m) res[m] = st.res[m];
    if (res_first) for (int m = 0; m < h->nv; ++m) res_first[m] = st.res_first[m];
    if (dt_last) *dt_last = st.dt_last;
    if (t) *t = st.t;
    if (steps_done) *steps_done = st.steps;
    return r;
}

gks_status gks_fields(gks_handle h, int32_t which, double* host_out)
{
    MarkerRange marker("gks_fields");
    if (!h || !host_out) return fail_h(h, GKS_ERR_ARG, "NULL argument");
    if (which < GKS_FIELD_CONS || which > GKS_FIELD_TURB_CONS) return fail_h(h, GKS_ERR_ARG, "unknown field");
    if (which == GKS_FIELD_TURB_CONS && !h->cfg.turb_transport)
        return fail_h(h, GKS_ERR_ARG, "TURB_CONS needs turb_transport");
    gks_status rs = sync_batch(h);
    if (rs != GKS_OK) return rs;
    State st;
    HIP_TRY(h, hipMemcpyAsync(&st, h->st, sizeof(State), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const long long N = h->L.ncells;
    const int nv = h->nv, D = h->cfg.dim;
    const bool diag = which == GKS_FIELD_EPS || which == GKS_FIELD_TAU;
    if (which == GKS_FIELD_STRAIN || diag || (which == GKS_FIELD_TURB && h->cfg.turb_transport)) {
        // a strain pass over the current state (with transport it also writes k and omega)
        hipLaunchKernelGGL(h->cfg.turb_transport ? k_strain<true> : k_strain<false>, dim3(h->grid_cell),
                           dim3(CELL_TILE), 0, h->stream, (const void*)h->tab, 1, 1, 0);
        HIP_TRY(h, hipGetLastError());
    }
    if (which == GKS_FIELD_STRAIN) {
        HIP_TRY(h, hipMemcpyAsync(host_out, h->inst.S, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        return GKS_OK;
    }
    if (diag) {
        // into the older state buffer, which no step reads again before writing it
        double* out = h->inst.W[st.parity ^ 1];
        const int grid = (int)std::min<long long>((N + 63) / 64, 1 << 20);
        const int v = variant_of(&h->cfg) & (V_TH | V_R3 | V_W5);
        void (*ke)(const void*, int, double*, int) = k_eps<0>;
        switch (v) {
        case V_TH: ke = k_eps<V_TH>; break;
        case V_R3: ke = k_eps<V_R3>; break;
        case V_TH | V_R3: ke = k_eps<V_TH | V_R3>; break;
        case V_W5: ke = k_eps<V_W5>; break;
        case V_TH | V_W5: ke = k_eps<V_TH | V_W5>; break;
        default: break;
        }
        hipLaunchKernelGGL(ke, dim3(grid), dim3(64), 0, h->stream, (const void*)h->tab, 1, out,
                           which == GKS_FIELD_TAU ? 1 : 0);
        HIP_TRY(h, hipGetLastError());
        HIP_TRY(h, hipMemcpyAsync(host_out, out, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        return GKS_OK;
    }
    if (which == GKS_FIELD_TURB_CONS) {
        HIP_TRY(h, hipMemcpyAsync(host_out, h->inst.W[st.parity] + (size_t)nv * N, sizeof(double) * 2 * N,
                                  hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        return GKS_OK;
    }
    if (which == GKS_FIELD_TURB) {
        HIP_TRY(h, hipMemcpyAsync(host_out, h->inst.k, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipMemcpyAsync(host_out + N, h->inst.om, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        return GKS_OK;
    }
    HIP_TRY(h, hipMemcpyAsync(host_out, h->inst.W[st.parity], sizeof(double) * N * nv, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (which == GKS_FIELD_PRIM) {
        for (long long i = 0; i < N; ++i) {
            const double rho = host_out[i];
            double ke = 0.0;
            for (int d = 0; d < D; ++d) {
                const double u = host_out[(1 + d) * N + i] / rho;
                ke += u * host_out[(1 + d) * N + i];
                host_out[(1 + d) * N + i] = u;
            }
            host_out[(D + 1) * N + i] = (h->cfg.gamma - 1.0) * (host_out[(D + 1) * N + i] - 0.5 * ke);
        }
    }
    return GKS_OK;
}

gks_status gks_resume(gks_handle h, const double* res, const double* res_first, double dt_last, double t,
                      int64_t steps_done, const double* turb_cons)
{
    MarkerRange marker("gks_resume");
    if (!h) return fail_h(nullptr, GKS_ERR_ARG, "NULL handle");
    if (h->broken || !h->pristine) return fail_h(h, GKS_ERR_STATE, "resume needs a handle that has taken no step");
    if (!(t >= 0.0) || !isfinite(t) || !(dt_last >= 0.0) || !isfinite(dt_last) || steps_done < 0)
        return fail_h(h, GKS_ERR_ARG, "bad progress values");
    const int nv = h->nv;
    for (int m = 0; m < nv; ++m)
        if ((res && (!(res[m] >= 0.0) || !isfinite(res[m]))) ||
            (res_first && (!(res_first[m] >= 0.0) || !isfinite(res_first[m]))))
            return fail_h(h, GKS_ERR_ARG, "residuals must be finite and >= 0");
    if (turb_cons && !h->cfg.turb_transport) return fail_h(h, GKS_ERR_ARG, "turb_cons needs turb_transport");
    const long long N = h->L.ncells;
    if (turb_cons)
        for (long long i = 0; i < N; ++i)
            if (!(turb_cons[i] >= 0.0) || !isfinite(turb_cons[i]) || !(turb_cons[N + i] > 0.0) ||
                !isfinite(turb_cons[N + i]))
                return fail_h(h, GKS_ERR_ARG, "rho k must be finite and >= 0, rho omega finite and > 0");
    hipStream_t s = h->stream;
    State st;
    HIP_TRY(h, hipMemcpyAsync(&st, h->st, sizeof(State), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (turb_cons)
        HIP_TRY(h, hipMemcpyAsync(h->inst.W[st.parity] + (size_t)nv * N, turb_cons, sizeof(double) * 2 * N,
                                  hipMemcpyHostToDevice, s));
    st.t = t;
    st.steps = steps_done;
    st.dt_last = dt_last;
    for (int m = 0; m < 5; ++m) {
        st.res[m] = res && m < nv ? res[m] : 0.0;
        st.res_first[m] = res_first && m < nv ? res_first[m] : 0.0;
    }
    HIP_TRY(h, hipMemcpyAsync(h->st, &st, sizeof(State), hipMemcpyHostToDevice, s));
    // the first step again, from the restored time, step count and (with transport) rho k
    hipLaunchKernelGGL(k_rate, dim3(h->grid_cell), dim3(CELL_TILE), 0, s, (const void*)h->tab, 1);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(CELL_TILE), 0, s, (const void*)h->tab, 1, 1);
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipMemcpyAsync(&st, h->st, sizeof(State), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (st.err) {
        h->broken = true;
        return fail_h(h, GKS_ERR_NONPHYSICAL, "resumed state is not physical");
    }
    return GKS_OK;
}

gks_status gks_state_device_ptr(gks_handle h, const double** dev_W)
{
    if (!h || !dev_W) return fail_h(h, GKS_ERR_ARG, "NULL argument");
    gks_status rs = sync_batch(h);
    if (rs != GKS_OK) return rs;
    State st;
    HIP_TRY(h, hipMemcpyAsync(&st, h->st, sizeof(State), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    *dev_W = h->inst.W[st.parity];
    return GKS_OK;
}

gks_status gks_set_timing(gks_handle h, int32_t enable)
{
    if (!h) return fail_h(nullptr, GKS_ERR_ARG, "NULL handle");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->timing = enable != 0;
    h->events_used = 0;
    h->timed_kind.clear();
    h->steps_timed = 0;
    return GKS_OK;
}

gks_status gks_kernel_times(gks_handle h, double* ms, int64_t* steps_timed)
{
    if (!h || !ms) return fail_h(h, GKS_ERR_ARG, "NULL argument");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int q = 0; q < 4; ++q) ms[q] = 0.0;
    for (size_t i = 0; i < h->timed_kind.size() && 2 * i + 1 < h->events_used; ++i) {
        float t = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&t, h->events[2 * i], h->events[2 * i + 1]));
        ms[h->timed_kind[i]] += t;
    }
    if (steps_timed) *steps_timed = h->steps_timed;
    return GKS_OK;
}

gks_status gks_destroy(gks_handle h)
{
    if (!h) return GKS_OK;
    State st;
    gks_status r = GKS_OK;
    if (h->batch_stream && h->batch_stream != h->stream) (void)hipStreamSynchronize(h->batch_stream);
    if (hipMemcpyAsync(&st, h->st, sizeof(State), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        r = GKS_ERR_DEVICE;
    else if (st.err && !h->broken)
        r = GKS_ERR_NONPHYSICAL;
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    delete h;
    return r;
}

const char* gks_last_error(gks_handle h)
{
    if (h) return h->err.c_str();
    return g_last_error.c_str();
}

// ------------------------------------------------------------------------------------
// batch
// ------------------------------------------------------------------------------------
// Batch workspace: the tile table, then an array of cap step states (the read-back buffer
// of gks_batch_status).
static constexpr size_t batch_bytes(int cap) { return TabView::bytes(cap) + tab_align(sizeof(State) * (size_t)cap); }

// Scratch of the workspace-free batch (gks_batch_create_static): the tile table and the
// read-back array of one batch of up to GKS_BATCH_STATIC_CAPACITY members per device, in a
// file-scope device array that each device holds until the process ends.  In host code
// `scratch` names a host-side stand-in: its device address comes from hipGetSymbolAddress,
// taken once per device with that device current and kept in g_static[dev].ptr, and only
// that address is ever handed to kernels or copies.
constexpr size_t kStaticScratchBytes = batch_bytes(GKS_BATCH_STATIC_CAPACITY);
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
struct StaticSlot {
    void* ptr = nullptr;   // device address of `scratch` on this device
    bool busy = false;     // a workspace-free batch exists on this device
};
std::mutex g_static_mu;
StaticSlot g_static[kMaxDevices];
}  // namespace

// Claim the current device's scratch for one batch: its device address (looked up on the
// first claim) or an error when the device's scratch already serves a live batch.
static gks_status claim_static(int* dev_out, void** ptr_out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail_h(nullptr, GKS_ERR_DEVICE, "no current HIP device");
    if (dev >= kMaxDevices) return fail_h(nullptr, GKS_ERR_ARG, "device ordinal beyond the library's static table");
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticSlot& slot = g_static[dev];
    if (slot.busy)
        return fail_h(nullptr, GKS_ERR_STATE,
                      "a workspace-free batch already exists on this device (destroy it first)");
    if (!slot.ptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail_h(nullptr, GKS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        slot.ptr = p;
    }
    slot.busy = true;
    *dev_out = dev;
    *ptr_out = slot.ptr;
    return GKS_OK;
}

static void release_static(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[dev].busy = false;
}
static State* batch_states(gks_batch b) { return (State*)((char*)b->tab + TabView::bytes(b->cap)); }

gks_status gks_batch_workspace_bytes(int32_t capacity, size_t* bytes)
{
    if (capacity < 1 || !bytes) return fail_h(nullptr, GKS_ERR_ARG, "bad capacity");
    *bytes = batch_bytes(capacity);
    return GKS_OK;
}

static gks_status batch_upload(gks_batch b)
{
    std::vector<const Inst*> mem;
    Present present;
    for (gks_handle h : b->members) {
        // work the member enqueued on its own stream must finish before batch work starts
        if (h->stream != b->stream && hipStreamSynchronize(h->stream) != hipSuccess) {
            b->err = "member stream sync failed";
            g_last_error = b->err;
            return GKS_ERR_DEVICE;
        }
        h->batch_stream = b->stream;
        mem.push_back(&h->inst);
        const int kw = h->cfg.turb_transport ? 1 : 0;
        present.face.set(h->cls * 32 + variant_of(&h->cfg));
        present.strain[kw] = true;
        if (h->cfg.dim == 3 && !h->inst.fused3) present.update[kw] = true;
    }
    build_table(b->host_tab, b->cap, mem, b->shape2);
    if (hipMemcpyAsync(b->tab, b->host_tab.data(), b->host_tab.size(), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        b->err = "table upload failed";
        g_last_error = b->err;
        return GKS_ERR_DEVICE;
    }
    // a captured step graph stays valid while it launches every kernel the members need
    if (b->captured && !b->present.covers(present)) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->captured = false;
    }
    if (!b->captured) b->present = present;
    return GKS_OK;
}

// A batch over `hs` whose table lives at `tab` (a caller workspace or a device's scratch).
static gks_status batch_make(const gks_handle* hs, int32_t count, int32_t capacity, void* tab, void* hip_stream,
                             int static_dev, gks_batch* out)
{
    gks_batch b = new gks_batch_ctx();
    b->members.assign(hs, hs + count);
    for (int i = 0; i < count; ++i) hs[i]->pristine = false;
    b->cap = capacity;
    b->stream = (hipStream_t)hip_stream;
    b->tab = tab;
    b->captured = false;
    b->graph_steps = 1;
    b->static_dev = static_dev;
    const int cus = device_cus();
    b->grid[0] = cus * 8;        // strain: 256-thread workgroups
    b->grid[5] = cus * 8;        // update
    b->grid[1] = b->grid[2] = 0;                       // fused 2D kernel: one workgroup per tile
    b->grid[3] = b->grid[4] = cus * 16;                // 3D face: one-wave workgroups
    // the whole table image (zeros included) is written before any kernel reads it, so a
    // reused scratch needs no clearing; the read-back array is written by k_states first
    gks_status r = batch_upload(b);
    if (r != GKS_OK) { delete b; return r; }
    *out = b;
    return GKS_OK;
}

static gks_status batch_args_ok(const gks_handle* hs, int32_t count, int32_t capacity)
{
    if ((!hs && count) || count < 0 || capacity < 1 || count > capacity)
        return fail_h(nullptr, GKS_ERR_ARG, "bad batch arguments");
    for (int i = 0; i < count; ++i)
        if (!hs[i] || hs[i]->broken) return fail_h(nullptr, GKS_ERR_ARG, "member handle is NULL or broken");
    return GKS_OK;
}

gks_status gks_batch_create(const gks_handle* hs, int32_t count, int32_t capacity, void* dev_workspace, size_t bytes,
                            void* hip_stream, gks_batch* out)
{
    if (!out || !dev_workspace) return fail_h(nullptr, GKS_ERR_ARG, "bad batch arguments");
    gks_status r = batch_args_ok(hs, count, capacity);
    if (r != GKS_OK) return r;
    if (bytes < batch_bytes(capacity)) return fail_h(nullptr, GKS_ERR_NOMEM, "batch workspace too small");
    if (((uintptr_t)dev_workspace) & 255) return fail_h(nullptr, GKS_ERR_ARG, "workspace must be 256-byte aligned");
    return batch_make(hs, count, capacity, dev_workspace, hip_stream, -1, out);
}

gks_status gks_batch_create_static(const gks_handle* hs, int32_t count, int32_t capacity, void* hip_stream,
                                   gks_batch* out)
{
    if (!out) return fail_h(nullptr, GKS_ERR_ARG, "out is NULL");
    gks_status r = batch_args_ok(hs, count, capacity);
    if (r != GKS_OK) return r;
    if (capacity > GKS_BATCH_STATIC_CAPACITY)
        return fail_h(nullptr, GKS_ERR_ARG, "capacity exceeds GKS_BATCH_STATIC_CAPACITY (256) members");
    int dev = -1;
    void* ptr = nullptr;
    r = claim_static(&dev, &ptr);
    if (r != GKS_OK) return r;
    r = batch_make(hs, count, capacity, ptr, hip_stream, dev, out);
    if (r != GKS_OK) release_static(dev);
    return r;
}

gks_status gks_batch_set_members(gks_batch b, const gks_handle* hs, int32_t count)
{
    if (!b || count < 0 || count > b->cap || (!hs && count)) return fail_h(nullptr, GKS_ERR_ARG, "bad member list");
    for (int i = 0; i < count; ++i)
        if (!hs[i] || hs[i]->broken) return fail_h(nullptr, GKS_ERR_ARG, "member handle is NULL or broken");
    b->members.assign(hs, hs + count);
    for (int i = 0; i < count; ++i) hs[i]->pristine = false;
    return batch_upload(b);
}

// Grid of a launch kind: the persistent size set by gks_batch_set_launch, or (0) one
// workgroup per tile of the current table (rounded up to a multiple of the 8 XCDs).  The kernels walk the table with a grid-stride
// loop, so any grid covers any membership (a captured graph keeps its grid).
static int batch_grid(gks_batch b, int kind)
{
    if (b->grid[kind] > 0) return b->grid[kind];
    TabView tv(b->host_tab.data(), b->cap);
    // the strain launch also carries one end-of-step work item per member
    const int tiles = kind == 0 ? tv.hdr->total_cell + tv.hdr->count
                                : (kind == 5 ? tv.hdr->total_cell : tv.hdr->total_face[kind - 1]);
    return round8(tiles > 0 ? tiles : 1);
}

// One batch step: the frozen-form strain pass, which also ends every member's previous
// step, and the transported form's if any member transports k and omega; the face kernel
// of each (class, variant) pair present (walking its class's tiles, passing the other
// variants' tiles, at the class's tile size);
// the 3D update of each form present.
static void batch_launch(gks_batch b, const Present& present)
{
    const void* tab = b->tab;
    hipLaunchKernelGGL(k_strain<false>, dim3(batch_grid(b, 0)), dim3(CELL_TILE), 0, b->stream, tab, b->cap, 0, 1);
    if (present.strain[1])
        hipLaunchKernelGGL(k_strain<true>, dim3(batch_grid(b, 0)), dim3(CELL_TILE), 0, b->stream, tab, b->cap, 0, 0);
    for (int c = 0; c < NCLS; ++c)
        for (int v = 0; v < 32; ++v)
            if (present.face.test(c * 32 + v)) {
                hipLaunchKernelGGL(face_kernel(c, v, c < 2 ? b->shape2[c] : 0), dim3(batch_grid(b, 1 + c)),
                                   dim3(face_block(c, v)), 0, b->stream, tab, b->cap, c);
            }
    if (present.update[0])   // 3D members update in their own launch
        hipLaunchKernelGGL(k_update<false>, dim3(batch_grid(b, 5)), dim3(CELL_TILE), 0, b->stream, tab, b->cap);
    if (present.update[1])
        hipLaunchKernelGGL(k_update<true>, dim3(batch_grid(b, 5)), dim3(CELL_TILE), 0, b->stream, tab, b->cap);
}

gks_status gks_batch_step(gks_batch b, int32_t nsteps)
{
    MarkerRange marker("gks_batch_step");
    if (!b || nsteps < 0) return fail_h(nullptr, GKS_ERR_ARG, "bad batch step");
    // whole replays of the captured graph, then the remaining steps launched directly
    const int replays = b->captured ? nsteps / b->graph_steps : 0;
    for (int i = 0; i < replays; ++i)
        if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return fail_h(nullptr, GKS_ERR_DEVICE, "graph launch failed");
    for (int i = replays * (b->captured ? b->graph_steps : 0); i < nsteps; ++i) batch_launch(b, b->present);
    // end of the last step (outside the captured step graph)
    if (nsteps > 0)
        hipLaunchKernelGGL(k_finish, dim3(b->cap), dim3(CELL_TILE), 0, b->stream, (const void*)b->tab, b->cap, 0);
    if (hipGetLastError() != hipSuccess) return fail_h(nullptr, GKS_ERR_DEVICE, "batch launch failed");
    return GKS_OK;
}

gks_status gks_batch_capture(gks_batch b) { return gks_batch_capture_steps(b, 1); }

gks_status gks_batch_capture_steps(gks_batch b, int32_t steps)
{
    MarkerRange marker("gks_batch_capture_steps");
    if (!b || steps < 1 || steps > 1024) return fail_h(nullptr, GKS_ERR_ARG, "NULL batch or steps outside 1..1024");
    if (b->captured) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->captured = false;
    }
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail_h(nullptr, GKS_ERR_DEVICE, "begin capture failed");
    for (int i = 0; i < steps; ++i) batch_launch(b, b->present);
    if (hipStreamEndCapture(b->stream, &b->graph) != hipSuccess)
        return fail_h(nullptr, GKS_ERR_DEVICE, "end capture failed");
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(b->graph);
        return fail_h(nullptr, GKS_ERR_DEVICE, "graph instantiate failed");
    }
    b->captured = true;
    b->graph_steps = steps;
    return GKS_OK;
}

gks_status gks_batch_set_launch(gks_batch b, int32_t kind, int32_t grid, int32_t tile)
{
    if (!b || kind < 0 || kind > 5 || grid < 0) return fail_h(nullptr, GKS_ERR_ARG, "bad launch shape");
    // kinds 1, 2: the fused 2D kernel's tile shape (GKS_TILE2_*, 256 meaning the default
    // 16 x 15); kinds 3, 4: 0, 256 (the fused 3D kernel's fixed tile) or FACE_TILE (the 3D face
    // kernel of the options outside k_tile3); other kinds: 0
    const bool two = kind == 1 || kind == 2;
    const bool ok_tile = tile == 0 || (two && (tile == GKS_TILE2_32X7 || tile == GKS_TILE2_8X28 || tile == T2_THREADS)) ||
                         (kind >= 3 && kind <= 4 && (tile == T2_THREADS || tile == FACE_TILE));
    if (!ok_tile) return fail_h(nullptr, GKS_ERR_ARG, "unsupported tile size");
    b->grid[kind] = grid;
    if (b->captured) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->captured = false;
    }
    if (two) {
        const int shape = tile == T2_THREADS ? 0 : tile;
        if (b->shape2[kind - 1] != shape) {
            b->shape2[kind - 1] = shape;
            return batch_upload(b);     // the class's tile counts change
        }
    }
    return GKS_OK;
}

gks_status gks_batch_status(gks_batch b, int64_t* steps, double* res, double* res_first, double* t,
                            int32_t* state)
{
    if (!b) return fail_h(nullptr, GKS_ERR_ARG, "NULL batch");
    std::vector<State> sts(b->members.size());
    if (!sts.empty()) {
        // one gather launch and one copy for the whole batch, after the queued steps
        hipLaunchKernelGGL(k_states, dim3(1), dim3(64), 0, b->stream, (const void*)b->tab, b->cap, batch_states(b));
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(sts.data(), batch_states(b), sizeof(State) * sts.size(), hipMemcpyDeviceToHost,
                           b->stream) != hipSuccess)
            return fail_h(nullptr, GKS_ERR_DEVICE, "state read failed");
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail_h(nullptr, GKS_ERR_DEVICE, "sync failed");
    for (size_t i = 0; i < sts.size(); ++i) {
        if (steps) steps[i] = sts[i].steps;
        if (res) for (int m = 0; m < 5; ++m) res[5 * i + m] = sts[i].res[m];
        if (res_first) for (int m = 0; m < 5; ++m) res_first[5 * i + m] = sts[i].res_first[m];
        if (t) t[i] = sts[i].t;
        if (state) state[i] = sts[i].err ? 2 : (sts[i].active ? 0 : 1);
        if (sts[i].err) b->members[i]->broken = true;
    }
    return GKS_OK;
}

gks_status gks_batch_destroy(gks_batch b)
{
    if (!b) return GKS_OK;
    (void)hipStreamSynchronize(b->stream);
    if (b->captured) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
    }
    if (b->static_dev >= 0) release_static(b->static_dev);
    delete b;
    return GKS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------
// operation count of one face on the host
// ------------------------------------------------------------------------------------
namespace gks {
struct CR {
    double v;
    static thread_local double n;
    CR() : v(0) {}
    CR(double x) : v(x) {}
    CR(int x) : v(x) {}
    explicit operator double() const { return v; }
};
thread_local double CR::n = 0;
inline CR operator+(CR a, CR b) { CR::n += 1; return CR(a.v + b.v); }
inline CR operator-(CR a, CR b) { CR::n += 1; return CR(a.v - b.v); }
inline CR operator*(CR a, CR b) { CR::n += 1; return CR(a.v * b.v); }
inline CR operator/(CR a, CR b) { CR::n += 1; return CR(a.v / b.v); }
inline CR operator-(CR a) { return CR(-a.v); }
inline bool operator<(CR a, CR b) { return a.v < b.v; }
inline bool operator>(CR a, CR b) { return a.v > b.v; }
inline bool operator>=(CR a, CR b) { return a.v >= b.v; }
inline bool operator<=(CR a, CR b) { return a.v <= b.v; }
inline CR g_exp(CR a) { CR::n += 1; return CR(exp(a.v)); }
inline CR g_abs(CR a) { return CR(fabs(a.v)); }
inline CR g_min(CR a, CR b) { return CR(fmin(a.v, b.v)); }     // a comparison, not counted
inline CR g_copysign(CR a, CR b) { return CR(copysign(a.v, b.v)); }
inline CR g_rcp(CR a) { CR::n += 1; return CR(1.0 / a.v); }
inline CR g_rsqrt(CR a) { CR::n += 2; return CR(1.0 / sqrt(a.v)); }   // a square root and a division
// the erfc evaluation counts as one operation, as a library erfc call would
inline CR erfc_e(CR ax, CR e) { CR::n += 1; return CR(erfc(ax.v) + 0.0 * e.v); }

template <int D, int MODE = 0, int RK = 0>
static double count_face()
{
    constexpr int NV = D + 2;
    // a representative interior face: distinct left/right states, nonzero slopes, tau ~ dt/3
    // (six stencil cells: the outer two feed the WENO5 values only)
    const double prim[6][5] = {{0.97, 0.32, -0.11, 0.06, 0.88}, {1.00, 0.30, -0.10, 0.05, 0.90},
                               {1.10, 0.25, -0.05, 0.02, 1.00}, {0.95, 0.35, -0.12, 0.04, 0.85},
                               {1.05, 0.28, -0.08, 0.03, 0.95}, {1.02, 0.31, -0.09, 0.04, 0.93}};
    const double gamma = 1.4, h = 0.01;
    CR Wx[6][NV];
    for (int o = 0; o < 6; ++o) {
        const double rho = prim[o][0], p = prim[o][4];
        double ke = 0.0;
        Wx[o][0] = CR(rho);
        for (int d = 0; d < D; ++d) { Wx[o][1 + d] = CR(rho * prim[o][1 + d]); ke += rho * prim[o][1 + d] * prim[o][1 + d]; }
        Wx[o][D + 1] = CR(p / (gamma - 1.0) + 0.5 * ke);
    }
    FaceGeo<CR> geo;
    for (int q = 0; q < 3; ++q) geo.icd[q] = CR(1.0 / h);
    geo.dl = geo.dr = CR(0.5 * h);
    geo.idl = geo.idr = CR(2.0 / h);
    CR::n = 0;
    FaceIn<D, CR> in;
    const CR(*Wc)[NV] = Wx + 1;
    reconstruct<D, CR, RK>(Wc, geo, in);
    in.kf = CR(1e-3);
    in.wf = CR(10.0);
    in.Sf = CR(5.0);
    in.dt = CR(3e-3);
    for (int t = 0; t < D - 1; ++t)              // tangential gradients (multi-dimensional mode)
        for (int m = 0; m < NV; ++m) {
            in.tl[t][m] = CR(0.3 * (m + 1) * (t + 1));
            in.tr[t][m] = CR(-0.2 * (m + 2) * (t + 1));
        }
    const double b = 2.0 / (gamma - 1.0);
    GasC gas{1e-3, 0.1, b, 2.0 / b, 1.0 / b, 1.0 / 0.09, 1.0 / 0.72 - 1.0};
    CR F[NV];
    face_flux<CR, D, CR, MODE>(in, gas, F);
    return CR::n;
}

// operations of the rho k / rho omega fluxes of one face (transported solves)
static double count_kw_face()
{
    CR Fk, Fw;
    CR::n = 0;
    kw_face_t<CR>(CR(1e-3), CR(0.2), CR(1e-3), CR(2e-3), CR(5.0), CR(6.0), CR(2e-4), CR(3e-4), CR(100.0), CR(1e-3),
                  Fk, Fw);
    return CR::n;
}
}  // namespace gks

extern "C" gks_status gks_face_flops(int32_t dim, int32_t precision, double* flops)
{
    if (!flops || (dim != 2 && dim != 3) || (precision != GKS_FP64 && precision != GKS_FP32_FLUX))
        return fail_h(nullptr, GKS_ERR_ARG, "bad arguments");
    *flops = dim == 2 ? gks::count_face<2>() : gks::count_face<3>();
    return GKS_OK;
}

extern "C" gks_status gks_face_flops_multid(int32_t dim, double* flops)
{
    if (!flops || (dim != 2 && dim != 3)) return fail_h(nullptr, GKS_ERR_ARG, "bad arguments");
    *flops = dim == 2 ? gks::count_face<2, gks::FLUX_MULTID>() : gks::count_face<3, gks::FLUX_MULTID>();
    return GKS_OK;
}

extern "C" gks_status gks_face_flops_recon(int32_t dim, int32_t recon, double* flops)
{
    if (!flops || (dim != 2 && dim != 3) ||
        (recon != GKS_RECON_MUSCL2 && recon != GKS_RECON_MUSCL3 && recon != GKS_RECON_WENO5))
        return fail_h(nullptr, GKS_ERR_ARG, "bad arguments");
    if (recon == GKS_RECON_MUSCL2) *flops = dim == 2 ? gks::count_face<2>() : gks::count_face<3>();
    else if (recon == GKS_RECON_MUSCL3) *flops = dim == 2 ? gks::count_face<2, 0, 1>() : gks::count_face<3, 0, 1>();
    else *flops = dim == 2 ? gks::count_face<2, 0, 2>() : gks::count_face<3, 0, 2>();
    return GKS_OK;
}

extern "C" gks_status gks_kw_face_flops(double* flops)
{
    if (!flops) return fail_h(nullptr, GKS_ERR_ARG, "flops is NULL");
    *flops = gks::count_kw_face();
    return GKS_OK;
}
