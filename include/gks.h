/*
 * gks.h -- C ABI of the MI355X gas-kinetic flux/update library (libgks.so).
 *
 * The library advances the compressible Navier-Stokes equations with the turbulent
 * gas-kinetic scheme of M. Righi, "A gas-kinetic scheme for the simulation of
 * compressible turbulent flows" (arXiv:1302.2132): at every cell face a BGK (Xu-type)
 * flux built from the Kogan integral solution (Eqs. integralbgk, resultingf, fluxesf),
 * with a relaxation time made of a laminar part, the k-omega turbulent part and an
 * artificial part (Eqs. relaxation time, taua, tautchenadjusted), followed by the
 * conservative finite-volume update on a stretched Cartesian grid (section
 * "Implementation of the turbulent gas-kinetic scheme in a finite-volume solver").
 * k and omega are frozen inputs, or (turb_transport = 1) advanced with the flow by the
 * transport equations of the 2006 k-omega model (coefficients beta* = 0.09,
 * beta = 0.0708, alpha = 13/25, sigma* = 3/5, sigma = 1/2, sigma_do = 1/8): rho k and
 * rho omega are convected by each face's time-integrated gas-kinetic mass flux (upwind
 * k, omega), diffused with mu + sigma (mean of the two cells' rho k/omega), take the
 * model's production and cross-diffusion explicitly and its dissipation point-implicitly.
 *
 * Conventions used by every entry point
 *  - Cells are stored structure-of-arrays, x fastest: field m of cell (i, j, k) is at
 *    m * ncells + (k * ny + j) * nx + i.  Conservative variables are
 *    (rho, rho U, rho V, [rho W], rho E), nvar = dim + 2.  A solve with turb_transport
 *    stores nvar + 2 fields on the device, rho k and rho omega last.
 *  - Pointers named dev_* are device (HBM) pointers; all other pointers are host memory.
 *    The library copies every host input it needs during the call that receives it.
 *  - The caller owns device memory: it passes a workspace of the size the library asks
 *    for (a torch uint8 CUDA tensor works), and the library never allocates device
 *    memory itself.  The workspace must stay allocated until gks_destroy.
 *  - Every call returns a gks_status.  Asynchronous device errors (a non-positive
 *    density or pressure, a non-finite value) are raised by the kernels into a
 *    device-side flag and reported by the next synchronising call (gks_residual,
 *    gks_fields, gks_destroy) as GKS_ERR_NONPHYSICAL; after that only gks_fields and
 *    gks_destroy are accepted on the handle.
 *  - One handle belongs to one HIP stream; handles are independent of each other.
 */
#ifndef GKS_H
#define GKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GKS_OK = 0,
    GKS_ERR_ARG = 1,          /* invalid argument or configuration */
    GKS_ERR_NONPHYSICAL = 2,  /* rho <= 0, p <= 0 or non-finite state met */
    GKS_ERR_NOMEM = 3,        /* workspace too small */
    GKS_ERR_DEVICE = 4,       /* a HIP call failed */
    GKS_ERR_STATE = 5         /* call not allowed in the handle's current state */
} gks_status;

/* Boundary conditions per axis side.  Two ghost layers are synthesised on the fly:
 *  PERIODIC  wrap-around (both sides of the axis must be periodic);
 *  WALL      no-slip adiabatic wall: mirror image with every momentum component negated;
 *  DIRICHLET fixed state, bc_data = nvar conservative values;
 *  PROFILE   fixed state per boundary cell, bc_data = nvar x ntan values (field-major),
 *            ntan = product of the other axes' cell counts, tangential index with the
 *            lower axis fastest; ghost cells beyond the tangential range use the nearest;
 *  OUTFLOW   zeroth-order extrapolation (copy of the boundary cell).
 * k, omega and the strain rate of a ghost cell are those of its interior image
 * (wrapped for PERIODIC, mirrored for WALL, nearest boundary cell otherwise). */
enum { GKS_BC_PERIODIC = 0, GKS_BC_WALL = 1, GKS_BC_DIRICHLET = 2, GKS_BC_PROFILE = 3, GKS_BC_OUTFLOW = 4 };

/* Arithmetic of the flux evaluation.  FP32_FLUX evaluates the non-equilibrium part of the
 * flux in FP32: the slopes of the initial and equilibrium distributions (Eqs. initialf0,
 * eqlgform), the time coefficients A and Abar, and their time-weighted moment
 * contractions (the gam1, gam2, gam4, gam5 terms of Eq. fluxesf).  Everything of the size
 * of the pressure flux p dt stays FP64: the half-space moments of the two sides, the
 * interface state W0 (Eq. intermediatestate), the time weights, the Euler flux of W0 over
 * gam0 and the collisionless flux of the two sides over gam3, and the heat-flux
 * correction; so do the reconstruction, primitive recovery, the face fluxes as stored, the
 * conservative update and the time-step/residual reductions.  FP32 rounding therefore
 * scales with the viscous and slope terms, not with p dt. */
enum { GKS_FP64 = 0, GKS_FP32_FLUX = 1 };

/* Degree of rarefaction in the time weights of the flux.
 *  DT      eps = tau/dt (Eqs. resultingf4, epsilonkepsilon): the exact time integral of the
 *          Kogan solution over the step;
 *  TAUHAT  eps = tau/tau_hat (Eqs. tautautilde, tautilde, epsilonkomega): tau_hat =
 *          rho/|D rho|, D rho = U0 d_x rho - d_x (rho U) the interface material derivative
 *          along the normal (mean of the one-sided gradients through the interface state).
 *          The exponential time factors decay with tau_e = dt tau/tau_hat; the
 *          Chapman-Enskog terms keep the physical tau.  eps -> 0 gives the Navier-Stokes
 *          limit f_c (1 + Abar dt/2) (Eq. hydroturbolimit). */
enum { GKS_EPS_DT = 0, GKS_EPS_TAUHAT = 1 };

/* Reconstruction of the face values (section "Implementation ...": second- and
 * third-order TVD/MUSCL with the minmod limiter, and fifth-order WENO).  All use
 * conservative variables; the gradients that set the initial distribution's slopes are
 * the minmod of the two one-sided slopes on centre-to-centre distances in every scheme.
 *  MUSCL2  face values from the minmod gradients (second order);
 *  MUSCL3  face values from the limited kappa-scheme with kappa = 1/3: the slope towards a
 *          face is (1/3) minmod(s_away, 4 s_toward) + (2/3) minmod(s_toward, 4 s_away)
 *          (third-order face values on uniform grids, no new extrema);
 *  WENO5   face values by Jiang and Shu's fifth-order WENO (three-cell candidates of the
 *          five cells upwind-biased to each side, smoothness-indicator weights with
 *          eps = 1e-6) in index space, the cell widths not entering; it reads three cells
 *          on each side of a face, so it needs three ghost layers and at least three cells
 *          per axis.
 * Each combines with turb_transport and either eps_mode; MUSCL3 and WENO5 not with multi_d. */
enum { GKS_RECON_MUSCL2 = 0, GKS_RECON_MUSCL3 = 1, GKS_RECON_WENO5 = 2 };

/* Multi-dimensional expansion (multi_d = 1; section "Implementation ...": the distribution
 * expanded along all axes rather than only along the face normal).  The initial
 * distribution of each side and the equilibrium also carry tangential slopes b:
 *  - b of each side from the tangential gradients of its cell (minmod of the one-sided
 *    differences along each tangential axis on centre distances, from the ghost-filled
 *    states; a cell beyond a boundary takes its ghost neighbours, corner ghosts being
 *    filled axis by axis: the later axis' rule on the earlier axis' ghost);
 *  - b of the interface state from the mean of the two cells' tangential gradients;
 *  - A from <psi (a u + b.v_t + A)> = 0 and Abar from the time-integrated compatibility
 *    condition with the b terms; in the flux b.v_t enters beside a u.
 * Continuous linear data then give the Navier-Stokes flux with the full velocity-gradient
 * tensor.  It combines with turb_transport and either eps_mode (with GKS_EPS_TAUHAT the
 * rarefaction measure keeps its normal-direction form), not with MUSCL3 or WENO5. */

/* Fields for gks_fields. CONS: conservative state (nvar x ncells). PRIM: rho, U, V, [W],
 * p (nvar x ncells). STRAIN: strain-rate magnitude sqrt(2 S_ab S_ab) (ncells). TURB: k
 * then omega (2 x ncells): those of the current state when transported (computed on the
 * device from rho k, rho omega), the frozen inputs otherwise. EPS: eps_hat = tau/tau_hat of
 * each face at the current state and step, the largest over the cell's faces (ncells; in
 * either eps_mode, as the "turbulent Knudsen number" diagnostic). TAU: the relaxation time
 * tau = mu/p0 + tau_a + the k-omega part (Eqs. relaxation time, taua, tautchenadjusted) of
 * each face at the current state and step, the largest over the cell's faces (ncells).
 * TURB_CONS: rho k then rho omega of the current state (2 x ncells; turb_transport only,
 * else GKS_ERR_ARG), the transported variables as stored, for a checkpoint. */
enum { GKS_FIELD_CONS = 0, GKS_FIELD_PRIM = 1, GKS_FIELD_STRAIN = 2, GKS_FIELD_TURB = 3, GKS_FIELD_EPS = 4,
       GKS_FIELD_TAU = 5, GKS_FIELD_TURB_CONS = 6 };

typedef struct {
    int32_t dim;                  /* 2 or 3 */
    int64_t n[3];                 /* cells per axis (>= 2 each); n[2] ignored in 2D */
    const double* xf[3];          /* host: n[d]+1 increasing face coordinates per axis */
    int32_t bc[3][2];             /* GKS_BC_* for [axis][low, high] */
    const double* bc_data[3][2];  /* host: DIRICHLET / PROFILE data, else NULL */
    double gamma;                 /* ratio of specific heats, 1 < gamma <= 1 + 2/dim */
    double prandtl;               /* Prandtl number of the heat-flux correction */
    double mu;                    /* constant laminar viscosity (tau_lam = mu / p) */
    double c_a;                   /* artificial relaxation coefficient of Eq. taua (>= 0) */
    double c_mu;                  /* C_mu of the k-omega relaxation time (0.09) */
    double cfl;                   /* CFL number of the global time step */
    double t_end;                 /* > 0: clip the last step to land on t_end, then stop */
    int32_t precision;            /* GKS_FP64 or GKS_FP32_FLUX */
    int64_t max_steps;            /* > 0: the solve stops (on the device) after this many steps */
    int32_t turb_transport;       /* 1: transport k and omega with the flow; 0: frozen inputs */
    int32_t eps_mode;             /* GKS_EPS_DT or GKS_EPS_TAUHAT */
    int32_t recon;                /* GKS_RECON_MUSCL2, GKS_RECON_MUSCL3 or GKS_RECON_WENO5 */
    int32_t multi_d;              /* 1: multi-dimensional expansion (with GKS_RECON_MUSCL2;
                                     combines with turb_transport and either eps_mode) */
    double res_tol;               /* > 0: the solve stops (on the device) at the end of the first
                                     step n >= 2 with max_m res_m / res_first_m <= res_tol over
                                     the flow fields whose first-step residual is > 0 (the
                                     residual-fall criterion of a converging solve); 0: never */
} gks_config;

typedef struct gks_ctx* gks_handle;

/* Device workspace needed by one solve (state double buffer, frozen fields, face fluxes
 * of 3D solves with WENO5 or the multi-dimensional expansion, metrics, reduction partials).  This is the HBM footprint used for admission.  Pure host
 * arithmetic on cfg (no device call); GKS_ERR_ARG for a bad config. */
gks_status gks_workspace_bytes(const gks_config* cfg, size_t* bytes);

/* Set up a solve of the finite-volume scheme (section "Implementation of the turbulent
 * gas-kinetic scheme in a finite-volume solver") from a cell-averaged state W, the
 * turbulence fields k and omega that enter the relaxation time (Eq. tautchenadjusted) and
 * the gas constants of cfg.  Validate cfg and the initial state, copy W (nvar x ncells), k
 * and omega (ncells) from the host into dev_workspace (256-byte aligned,
 * >= gks_workspace_bytes), and compute the first CFL step on `hip_stream` (a hipStream_t;
 * NULL = default stream).  The handle (*out) is the library's; free it with gks_destroy.  With
 * turb_transport the initial rho k = rho * k and rho omega = rho * omega.  Returns
 * GKS_ERR_ARG for a bad config, k < 0, omega <= 0; GKS_ERR_NONPHYSICAL for rho <= 0 or
 * p <= 0; GKS_ERR_NOMEM if bytes is too small. */
gks_status gks_init(const gks_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
                    const double* W, const double* k, const double* omega, gks_handle* out);

/* Enqueue nsteps explicit steps (asynchronous; no host synchronisation).  Each step: CFL
 * time step from the current state, strain rate (the eta of Eq. tautchenadjusted), every
 * face flux (the time integral of Eq. resultingf over the step, Eq. fluxesf, with the
 * relaxation time of Eqs. relaxation time, taua, tautchenadjusted and the Prandtl
 * correction of the heat flux), conservative update of the cell averages by the fluxes'
 * differences (section "Implementation ..."), residual and next time step, all on the
 * device.  nsteps >= 0; a solve that reached t_end, max_steps or res_tol takes no more
 * steps (the call still succeeds).  GKS_ERR_STATE after a reported error.  With turb_transport the strain pass
 * also computes k, omega and the k-omega sources, the flux pass the fluxes of rho k and
 * rho omega through every face, and the update advances them; a step whose rho k < 0 or rho omega <= 0 is
 * non-physical. */
gks_status gks_step(gks_handle h, int32_t nsteps);

/* Synchronise and report the last step: res[nvar] = sqrt(mean(((W^{n+1}-W^n)/dt)^2)) per
 * flow field (rho k and rho omega excluded), res_first[nvar] the same for the first step of
 * the solve (for convergence ratios), the step dt_last, the time t and the number of steps
 * done.  The paper drives its steady solves to convergence without defining the residual;
 * this is the usual RMS of the time derivative of the conservative variables.  Any pointer
 * may be NULL; the arrays are the caller's.  Returns a pending device error
 * (GKS_ERR_NONPHYSICAL) after filling what it can. */
gks_status gks_residual(gks_handle h, double* res, double* res_first, double* dt_last, double* t,
                        int64_t* steps_done);

/* Synchronise and copy a field (GKS_FIELD_*, sizes as listed there) into host_out, which
 * the caller owns and sizes.  EPS and TAU evaluate every face of the current state at the
 * next step's dt with the solve's own options (Eqs. epsilonkomega, tautchenadjusted),
 * using the older state buffer as scratch, so they leave the state and later steps
 * unchanged.  GKS_ERR_ARG for an unknown field. */
gks_status gks_fields(gks_handle h, int32_t which, double* host_out);

/* Checkpoint/resume.  A solve is saved by gks_fields(CONS) (and TURB_CONS with
 * turb_transport) plus what gks_residual reports; it is restored by gks_init from the
 * saved CONS state (with the solve's k and omega, or any valid pair with transport)
 * followed by gks_resume with the saved values.  gks_resume sets the time, the step count
 * (counted towards max_steps), the last and first-step residuals (res_first drives
 * res_tol) and, with turb_transport, overwrites rho k and rho omega with turb_cons
 * (2 x ncells, host; NULL keeps rho k = rho * k of gks_init); then it recomputes the next
 * CFL step, clipped to t_end, by the arithmetic that ends every step.  The resumed solve
 * continues exactly as the saved one would have: stepping n, saving, resuming and stepping
 * m gives the state, residuals, time and step count of n + m steps, bitwise.  Only on a
 * handle that has taken no step and joined no batch (else GKS_ERR_STATE); res/res_first
 * (nvar each) may be NULL (zeros).  GKS_ERR_ARG for negative or non-finite values or
 * turb_cons without turb_transport; GKS_ERR_NONPHYSICAL (handle then in the error state)
 * when the restored state is not physical. */
gks_status gks_resume(gks_handle h, const double* res, const double* res_first, double dt_last, double t,
                      int64_t steps_done, const double* turb_cons);

/* Device pointer of the current conservative state (nvar x ncells, FP64; nvar + 2 with
 * turb_transport), inside the caller's workspace.  Valid until the next gks_step; the
 * caller may read it on the handle's stream (or after synchronising). */
gks_status gks_state_device_ptr(gks_handle h, const double** dev_W);

/* Synchronise and release the handle (the caller frees the workspace). */
gks_status gks_destroy(gks_handle h);

/* Per-kernel timing for benchmarks.  While enabled, gks_step launches each kernel with a
 * pair of HIP events on the handle's stream that the runtime stamps with that launch's
 * own start and end (no extra packets between launches).  A step is two launches: strain
 * (which also ends the previous step) and the fused tile kernel, which computes the faces
 * and updates (timed as face); a 3D step with transport, WENO5 or the multi-dimensional
 * expansion is three: strain, face and update.  A call
 * adds one trailing end-of-step launch (finish).  gks_kernel_times synchronises and writes the summed
 * milliseconds of each launch kind since timing was enabled (ms[0..3] = strain, face,
 * update, finish) and the number of steps timed; enabling again resets. */
gks_status gks_set_timing(gks_handle h, int32_t enable);
gks_status gks_kernel_times(gks_handle h, double* ms /*[4]*/, int64_t* steps_timed);

/* Text of the last error on the handle (or of the last failed handle-less call if NULL). */
const char* gks_last_error(gks_handle h);

/* Algorithmic FP operation count of one face flux of the given dimension and precision:
 * +, -, *, / and sqrt count 1, a fused multiply-add 2, each exp/erfc/expm1 call 1.
 * Counted by running the flux code on the host with a counting number type. */
gks_status gks_face_flops(int32_t dim, int32_t precision, double* flops);

/* The same count for the fluxes of rho k and rho omega that a transported solve adds to
 * every face (upwind convection by the mass flux plus diffusion with the mean eddy
 * viscosity; the mass flux itself is part of gks_face_flops). */
gks_status gks_kw_face_flops(double* flops);

/* The same count for the flux with the multi-dimensional expansion (multi_d). */
gks_status gks_face_flops_multid(int32_t dim, double* flops);

/* The same count (FP64) with the face values of the given reconstruction (GKS_RECON_*);
 * GKS_RECON_MUSCL2 gives gks_face_flops. */
gks_status gks_face_flops_recon(int32_t dim, int32_t recon, double* flops);

/* ---------------------------------------------------------------------------------- */
/* Batched form: many independent solves (any mix of sizes, dims, precisions) advanced  */
/* by persistent kernels that walk one device tile table per step.                       */
/* ---------------------------------------------------------------------------------- */
/* The paper runs one solve at a time; the batch advances many solves of the same scheme
 * (the step of gks_step, with each solve's own options) together, each member's result
 * being that of its solve stepped alone.  A gks_batch handle is the library's; free it
 * with gks_batch_destroy (the members stay the caller's). */
typedef struct gks_batch_ctx* gks_batch;

/* Device workspace of a batch able to hold up to `capacity` solves: its tile table and a
 * read-back buffer of `capacity` step states. */
gks_status gks_batch_workspace_bytes(int32_t capacity, size_t* bytes);

/* Create a batch over `count` initialised handles (all on the same device).  Batch work
 * runs on `hip_stream`, which must not be the legacy null stream if the batch is to be
 * captured as a graph.  Creation (and gks_batch_set_members) waits for the members' own
 * streams; afterwards every per-handle call on a member first waits for the batch stream.
 * The table lives in dev_workspace.  Handles stay owned by the caller and must outlive
 * the batch.  Members may carry any options (transport, eps_mode, reconstruction,
 * multi_d): a step launches the face kernel of each (dimension, precision, options) group
 * present, and the transported form's strain and 3D update passes when a member transports
 * k and omega; each member's result equals its solve stepped alone, bitwise. */
gks_status gks_batch_create(const gks_handle* hs, int32_t count, int32_t capacity,
                            void* dev_workspace, size_t bytes, void* hip_stream, gks_batch* out);

/* Replace the member list (admission/retirement).  The device table is rewritten in
 * place, so a captured step graph stays valid. */
gks_status gks_batch_set_members(gks_batch b, const gks_handle* hs, int32_t count);

/* Enqueue nsteps steps of every member (members that reached t_end or raised an error
 * are skipped on the device).  When a graph is captured (gks_batch_capture) the steps
 * replay it. */
gks_status gks_batch_step(gks_batch b, int32_t nsteps);

/* Capture one step of the batch as a HIP graph; later gks_batch_step calls replay it. */
gks_status gks_batch_capture(gks_batch b);

/* Capture `steps` (1..1024) consecutive steps as one HIP graph: gks_batch_step(n) then
 * replays it n / steps times and launches the remaining n % steps steps directly.  Every
 * step reads its parity, time step and activity from the device, so the replays are
 * identical launches and each member's result is the same as with one-step graphs or none
 * (bitwise).  Invalidated like a one-step graph by set_launch and by membership changes
 * that need kernels the graph lacks. */
gks_status gks_batch_capture_steps(gks_batch b, int32_t steps);

/* Launch shape of the batch kernels: kind 0 = strain, 1 = fused 2D tile kernel (FP64),
 * 2 = fused 2D tile kernel (FP32 flux), 3 = 3D face-class kernels (FP64), 4 = the same in
 * FP32 flux, 5 = update (3D solves outside the fused kernel).  grid = number of persistent
 * workgroups walking the tile table (0 = one per tile).  tile: for kinds 1 and 2 the cell
 * tile of the plain scheme's fused 2D kernel, GKS_TILE2_16X15 (0, also 256),
 * GKS_TILE2_32X7 or GKS_TILE2_8X28 (solves with options keep 16 x 15); for kinds 3 and 4
 * 0, 256 (the fused 3D column of 16 x 15 cells marching along z) or 64 (faces per
 * workgroup of the 3D face kernel of solves with transport, WENO5 or the
 * multi-dimensional expansion); 0 for the other kinds.  Anything else is GKS_ERR_ARG.
 * Results do not depend on the launch shape: the state bitwise, the residual up to the
 * rounding of its per-tile partial sums.  Invalidates a captured graph. */
enum { GKS_TILE2_16X15 = 0, GKS_TILE2_32X7 = 1, GKS_TILE2_8X28 = 2 };
gks_status gks_batch_set_launch(gks_batch b, int32_t kind, int32_t grid, int32_t tile);

/* Synchronise; copy per-member steps done, residual of the last step and of the first
 * step (5 slots per member each), time and status (0 running, 1 done by t_end, max_steps
 * or res_tol, 2 error) into host arrays (any NULL).  The states are gathered on the
 * device after the queued steps and read back in one copy. */
gks_status gks_batch_status(gks_batch b, int64_t* steps, double* res, double* res_first, double* t,
                            int32_t* state);

gks_status gks_batch_destroy(gks_batch b);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gks_batch_create without a workspace.
 * The batch's scratch -- its tile table and the read-back array of its members' step
 * states -- lives in a static device array of the library (one per device, ~0.2 MB,
 * held by each device the library runs on until the process ends), sized for up to
 * GKS_BATCH_STATIC_CAPACITY members.  The members' own workspaces are still the caller's.
 * The call allocates nothing (no hipMalloc, no allocating library routine); it fills the
 * table with one host-to-device copy on `hip_stream` and waits for it.
 * Limits and errors: capacity > GKS_BATCH_STATIC_CAPACITY -> GKS_ERR_ARG; at most one
 * such batch exists per device at a time: a second call on a device whose array serves a
 * live batch returns GKS_ERR_STATE until gks_batch_destroy of the first releases it.  The
 * array keeps the last batch's contents; every batch rewrites all of it that it reads.
 * Calls on one such batch from several threads at once race, as for any batch.  The
 * batch is then used with every gks_batch_* call like one made by gks_batch_create. */
enum { GKS_BATCH_STATIC_CAPACITY = 256 };
gks_status gks_batch_create_static(const gks_handle* hs, int32_t count, int32_t capacity, void* hip_stream,
                                   gks_batch* out);

#ifdef __cplusplus
}
#endif
#endif /* GKS_H */
