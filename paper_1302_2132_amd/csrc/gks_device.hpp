// gks_device.hpp -- device-side data layout shared by the kernels and the host code of
// libgks: per-solve descriptor, per-solve step state, and the tile table that lets one
// set of persistent kernels advance any mix of solves.
#pragma once
#include <stdint.h>

namespace gks {

constexpr int CELL_TILE = 256;   // cells per tile of the strain/update kernels (= block size)
constexpr int FACE_TILE = 64;    // default faces per tile of the face kernel (= block size)
constexpr int NCLS = 4;          // face-kernel classes: (dim 2|3) x (FP64|FP32 flux)
constexpr int PSTRIDE = 6;       // per-tile partials: nv residual sums (slots 0..4), CFL rate max (slot 5)

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_DIRICHLET = 2, BC_PROFILE = 3, BC_OUTFLOW = 4 };

// Step state of one solve.  The update kernel writes the new state into W[parity ^ 1] and
// records it in `fresh` with `pending` set; the end of the step (residual, time, next dt,
// parity flip, clearing `pending`) then runs either folded into the next step's strain
// launch or as a trailing launch.  The strain pass reads W[fresh], which the end of the
// step does not touch, so the two can share one launch without a race.
struct alignas(64) State {
    double dt;          // step size of the step about to run
    double t;           // time reached
    double t_after;     // time at the end of the step about to run (t_end when clipped)
    double dt_last;     // size of the last completed step
    double res[5];      // residual of the last completed step
    double res_first[5];
    int parity;         // W[parity] is the current state
    int err;            // bit 0: non-physical state met
    int active;         // 1 while stepping
    int fresh;          // W[fresh] is the newest state (== parity unless a step end is pending)
    int pending;        // 1 between an update and the end of its step
    long long steps;
};

// Device descriptor of one solve.  Extended metric arrays are offset so that index i of
// axis d (i from -2) reads xf[d][i], xc[d][i], dx[d][i].
// With k-omega transport (kw = 1) the state holds nv + 2 components, rho k and rho omega
// after the flow variables; k and om then hold k and omega of the state a step starts
// from (written by its strain pass), Qk and Qw the explicit sources of that state, nt its
// rho k / omega.
struct Inst {
    int dim, nv, precision, cls;
    int kw;                    // 1: k and omega are transported, else frozen inputs
    int variant;               // the solve's face-kernel variant (bits of its options)
    int n[3];
    int ntan[3];               // cells in a boundary plane of axis d
    int ncells;                // < 2^29 (validated), so cell and face indices fit in int
    int nface[3];              // faces normal to axis d
    int bc[3][2];
    double gamma, prandtl, mu, c_a, c_mu, cfl, t_end, b;
    double two_over_b, inv_b, inv_cmu, pfix;   // 2/b, 1/b, 1/C_mu, 1/Pr - 1
    double* W[2];
    double* k;
    double* om;
    double* S;
    double* Qk;                // transport only: sources of rho k and rho omega per cell,
    double* Qw;
    double* nt;                // and the eddy viscosity rho k / omega of the diffusive fluxes
    void* F[3];                // 3D face fluxes per axis: [nv (+2)][nface[d]], FP64 (2D: none)
    const double* xf[3];
    const double* xc[3];
    const double* dx[3];
    const double* idx[3];      // 1/dx[i], i from -2 to n+1
    const double* ic2[3];      // 1/(xc[i+1] - xc[i-1]), i from 0 to n-1 (central differences)
    const double* icd[3];      // 1/(xc[i+1] - xc[i]), i from -2 to n
    const double* fgeo[3];     // per face f in [0, n]: xf-xc[f-1], xc[f]-xf, and their inverses
    const double* bcd[3][2];
    double* part;              // per-tile partials [max(ntile_cell, nstep_part)][PSTRIDE]
    State* st;
    int ntile_cell;
    int nstep_part;            // partial slots written by a step: fused 2D tiles, else update tiles
    int ntile_face[3];
    int ntile_face_all;
    int face_tile;             // faces per face-kernel tile in the table holding this copy
    int shape2;                // 2D: tile shape code of the fused kernel in the table holding this copy
    int fused3;                // 3D step in one fused tile kernel (k_tile3): no face fluxes in HBM
    int seg3, nseg3;           // planes per z-run of a fused 3D tile, runs per tile column
    long long max_steps;       // > 0: deactivate after this many steps
    double res_tol;            // > 0: deactivate once max_m res_m / res_first_m <= res_tol (steps >= 2)
};

// Tile table header; arrays follow at offsets computed by TabView.
struct TabHdr {
    int count;
    int total_cell;
    int ncls[NCLS];
    int total_face[NCLS];
};

__host__ __device__ constexpr size_t tab_align(size_t x) { return (x + 255) & ~size_t(255); }

struct TabView {
    TabHdr* hdr;
    Inst* inst;          // [cap]
    int* cell_prefix;    // [cap + 1]
    int* cls_member;     // [NCLS][cap]
    int* cls_prefix;     // [NCLS][cap + 1]
    __host__ __device__ TabView(void* base, int cap)
    {
        char* p = (char*)base;
        hdr = (TabHdr*)p;
        size_t off = tab_align(sizeof(TabHdr));
        inst = (Inst*)(p + off);
        off = tab_align(off + sizeof(Inst) * (size_t)cap);
        cell_prefix = (int*)(p + off);
        off += sizeof(int) * (size_t)(cap + 1);
        cls_member = (int*)(p + off);
        off += sizeof(int) * (size_t)NCLS * cap;
        cls_prefix = (int*)(p + off);
    }
    __host__ __device__ static constexpr size_t bytes(int cap)
    {
        size_t off = tab_align(sizeof(TabHdr));
        off = tab_align(off + sizeof(Inst) * (size_t)cap);
        off += sizeof(int) * (size_t)(cap + 1);
        off += sizeof(int) * (size_t)NCLS * cap;
        off += sizeof(int) * (size_t)NCLS * (cap + 1);
        return tab_align(off);
    }
};

}  // namespace gks
