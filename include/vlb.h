/*
 * vlb.h -- C ABI of the MI355X coupled viscoelastic lattice Boltzmann library.
 *
 * One time step couples (Yu, Chen, Wang, Yuan, Shu, arXiv:2508.16997):
 *   - a D2Q9 two-relaxation-time regularized hydrodynamic lattice with a third-order
 *     Hermite equilibrium, the Galilean correction G_i, the first-order Hermite body
 *     force F_i and the local viscoelastic source T_i (Sec. 3.1);
 *   - three D2Q9 two-relaxation-time regularized convection-diffusion lattices for the
 *     conformation components A_xx, A_xy, A_yy with the Oldroyd-B constitutive source,
 *     the auxiliary term G~_i (incompressible form), the source term F~_i and its
 *     backward time difference (Sec. 2.2-2.3, 3.2);
 *   - conservative non-equilibrium bounce-back (CNEBB) for every conformation lattice
 *     at solid walls (Sec. 3.3), half-way or linearly interpolated bounce-back (or
 *     wet-node non-equilibrium bounce-back walls) for the hydrodynamic lattice, and open
 *     inlet / outlet columns whose ghost populations are set by non-equilibrium
 *     extrapolation from the adjacent fluid column (inlet: the prescribed velocity and
 *     conformation profile; outlet: rho = 1 with zero-gradient u and A; the channel set-up
 *     of Sec. 4.3).
 *
 * Conventions
 *   - Every call returns an int status: VLB_OK (0) or a negative VLB_E_* code; a
 *     thread-local detail string is available from vlb_last_error_detail().  No C++
 *     exception crosses this interface.  Invalid arguments are rejected before any
 *     device work is enqueued.
 *   - Memory: the library never allocates or frees device memory.  The caller owns
 *     the workspace (size from vlb_workspace_bytes) and every array it passes.  Host
 *     arrays given to the library are copied before the call returns.
 *   - Device arrays of fields are row-major [ny][nx] (x fastest), in the simulation's
 *     precision (float for VLB_FP32, double for VLB_FP64), unless stated otherwise.
 *   - Streams: all device work is enqueued on the HIP stream given to vlb_bind
 *     (hipStream_t passed as void*; 0 is the null stream).  Calls that return data
 *     to the host (vlb_monitors, vlb_load_state) synchronize that stream.
 *   - Threads: a vlb_sim must not be used from two host threads at once.
 */
#ifndef VLB_H
#define VLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VLB_OK = 0,
    VLB_E_INVALID_ARG = -1, /* bad size, mode, parameter (tau <= 1/2, lambda <= 0) */
    VLB_E_WORKSPACE = -2,   /* workspace missing, too small or misaligned            */
    VLB_E_HIP = -3,         /* a HIP runtime call failed (detail string has it)      */
    VLB_E_NONFINITE = -4,   /* NaN/Inf detected by the monitors: numerical breakdown */
    VLB_E_STATE = -5,       /* call out of order (e.g. step before bind/init)        */
    VLB_E_UNSUPPORTED = -6  /* feature not available for this configuration          */
};

enum { VLB_FP32 = 0, VLB_FP64 = 1 };
/* Boundary kind of an axis.  VLB_OPEN (x only): inlet ghost column at x = -1 and outlet
 * ghost column at x = nx, filled by non-equilibrium extrapolation from the first / last
 * column (inlet: the prescribed profile of vlb_set_inlet; outlet: rho = 1, zero-gradient
 * u and A).  VLB_WALL: no-slip wall half a spacing outside the first and last rows
 * (columns), half-way bounce-back for f.  VLB_WET (y only): wet-node walls -- rows 0 and
 * ny - 1 are wall nodes with u = 0 (channel height ny - 1), f rebuilt there by
 * non-equilibrium bounce-back (Zou-He closure with the half-force momentum; the wall
 * setting of the paper's channel flows, Sec. 4.2-4.3), CNEBB for the conformation
 * lattices at the wall nodes, one-sided second-order wall-normal differences; needs
 * ny >= 5 and fluid nodes on rows 0-2 and ny-3..ny-1. */
enum { VLB_PERIODIC = 0, VLB_WALL = 1, VLB_OPEN = 2, VLB_WET = 3 };
/* Node classes returned by vlb_geometry. */
enum { VLB_NODE_FLUID = 0, VLB_NODE_SOLID = 1, VLB_NODE_BOUNDARY = 2 };
/* Parameter flags. */
enum {
    VLB_FLAG_NO_SOURCE = 1,   /* constitutive source S forced to 0 (conservation checks)     */
    VLB_FLAG_CURVED_YLW = 2,  /* curved (circle) links of f: the paper's cylinder scheme YLW
                                 (Sec. 4.3) instead of linear interpolated bounce-back -- the
                                 unified interpolation of Yu, Mei, Luo and Shyy (2003),
                                 [(1 - q) f_o(x + e_i) + q f_o(x) + q f_i(x)] / (1 + q) for the
                                 unknown f_i(x) with o opposite to i (half-way without a fluid
                                 x + e_i), and the rest population restoring the node's mass
                                 (known populations plus those that left toward the wall), the
                                 conservation CNEBB shares with it (Sec. 3.3).  Flat walls
                                 (q = 1/2) stay half-way.  Not differentiable by the adjoint. */
    VLB_FLAG_OPEN_NEBB = 4    /* VLB_OPEN x only: the hydrodynamic open ends of
                                 the paper's cylinder (Sec. 4.3) as wet boundary nodes -- the
                                 first and last columns rebuild the populations from beyond the
                                 inlet / outlet by non-equilibrium bounce-back (Zou-He) for the
                                 inlet velocity (u_in(y), 0) and for density 1 with u_y = 0,
                                 with the half-force shift; the conformation lattices keep the
                                 extrapolation ghosts.  With VLB_WET y the corner nodes take
                                 the open-end rule first, then the wall rule.
                                 VLB_E_UNSUPPORTED off VLB_OPEN x. */
};

typedef struct vlb_sim vlb_sim;

/* Grid description.  A node is solid if solid_mask[y*nx + x] != 0 or if
 * (x - xc)^2 + (y - yc)^2 <= R^2 for one of the circles (evaluated in double without
 * fused multiply-add; exact for half-integer centres and radii).  Links that end in a
 * circle carry the wall fraction q of the exact circle; every other wall link has
 * q = 1/2. */
typedef struct {
    int nx, ny;               /* 1 <= nx, ny; (nx + 129)(ny + 2) < 2^31 / 64 (padded
                                 plane of at most 33.5 M slots); at least 2 nodes along
                                 a periodic or open axis, ny >= 5 with VLB_WET       */
    int xmode, ymode;         /* VLB_PERIODIC / VLB_WALL / VLB_OPEN (xmode only) /
                                 VLB_WET (ymode only)                                 */
    int precision;            /* VLB_FP32 or VLB_FP64                                  */
    const uint8_t* solid_mask;/* host, ny*nx, nullable                                 */
    const double* circles;    /* host, 3 per circle (xc, yc, R), nullable              */
    int ncircles;
} vlb_grid;

/* Constitutive closures (Sec. 2.2: the model function F(A) enters the conformation
 * equation as the relaxation term -(1/lambda) F and the Kramers relation as the stress
 * (eta_p / lambda) F).  The paper's runs use Oldroyd-B, F = A - I.  The others, in
 * conformation form with the 2-D trace tr A (2 at rest), relaxation function F_r and
 * stress function F_s:
 *   VLB_GIESEKUS  model_param = alpha in [0, 1]:  F_r = (A - I) + alpha (A - I)^2,  F_s = A - I
 *   VLB_LPTT      model_param = eps >= 0:   F_r = [1 + eps (tr A - 2)] (A - I),  F_s = A - I
 *   VLB_EPTT      model_param = eps >= 0:   F_r = exp[eps (tr A - 2)] (A - I),   F_s = A - I
 *   VLB_FENE_P    model_param = L^2 > 2:    F_r = F_s = f A - I, f = (L^2 - 2) / (L^2 - tr A) */
enum { VLB_OLDROYD_B = 0, VLB_GIESEKUS = 1, VLB_LPTT = 2, VLB_EPTT = 3, VLB_FENE_P = 4 };

/* Lattice-unit parameters (rho0 = 1).  The library derives the relaxation times of
 * Sec. 3.1-3.2: tau_s1 = nu_s / c_s^2 + 1/2, tau_s2 = Lambda_s / (tau_s1 - 1/2) + 1/2,
 * tau_p1 = kappa / c_s^2 + 1/2, tau_p2 = Lambda_p / (tau_p1 - 1/2) + 1/2, and the
 * polymer stress tau_ab = (eta_p / lambda) F_s(A)_ab of the chosen closure (zero
 * initialisation gives Oldroyd-B). */
typedef struct {
    double nu_s;      /* solvent kinematic viscosity, > 0                  */
    double eta_p;     /* polymer viscosity, >= 0                           */
    double lambda;    /* polymer relaxation time, > 0                      */
    double kappa;     /* centre-of-mass diffusion coefficient, > 0         */
    double Lambda_s;  /* hydrodynamic magic parameter, > 0                 */
    double Lambda_p;  /* conformation magic parameter, > 0                 */
    double Fx, Fy;    /* uniform body force (used until a force field is set) */
    int flags;        /* VLB_FLAG_*                                        */
    int model;        /* VLB_OLDROYD_B (0) ... VLB_FENE_P                  */
    double model_param; /* alpha, eps or L^2 (see above); ignored for Oldroyd-B */
} vlb_params;

typedef struct {
    double mass[4];     /* sum over fluid nodes of rho, A_xx, A_xy, A_yy (FP64 accumulation) */
    double residual;    /* max |u(now) - u(previous monitor call)| over fluid nodes           */
    double umax;        /* max |u| over fluid nodes                                          */
    int64_t step;       /* time step of the state                                            */
    int64_t nonfinite;  /* fluid nodes with a non-finite rho, u or A                         */
    int64_t spd_violations; /* fluid nodes with det(A) <= 0 or tr(A) <= 0                    */
} vlb_monitor;

/* ---- creation (host only, no device work) -------------------------------------- */

/* Builds the node classes and the boundary-link list on the host. */
int vlb_create(const vlb_grid* grid, vlb_sim** out);
void vlb_destroy(vlb_sim* sim);

/* Bytes of device workspace this simulation needs (populations, history, force,
 * geometry tables, monitors). */
int vlb_workspace_bytes(const vlb_sim* sim, size_t* bytes);

/* Node classes (host array of ny*nx, VLB_NODE_*) and the boundary-link list: one entry
 * per fluid node and direction d (1..8, D2Q9 order of the paper) whose neighbour
 * x + e_d is solid, as (node = y*nx + x, d, q), sorted by (node, d).  *nlinks receives
 * the total count; at most cap entries are written (cap = 0 and null arrays to query).
 * Host-only: usable without a device. */
int vlb_geometry(const vlb_sim* sim, uint8_t* node_class, int32_t* link_node,
                 int8_t* link_dir, double* link_q, int cap, int* nlinks);

/* ---- binding and set-up ------------------------------------------------------- */

/* Attaches a caller-owned device workspace (>= vlb_workspace_bytes, 256-byte aligned)
 * and the stream for all later work; uploads the geometry tables (async). */
int vlb_bind(vlb_sim* sim, void* workspace_dev, size_t bytes, void* hip_stream);

/* Validates and stores the parameters (tau_s1, tau_p1 > 1/2 follow from nu_s, kappa > 0). */
int vlb_set_params(vlb_sim* sim, const vlb_params* p);

/* Lattice-unit parameters from the dimensionless groups of Sec. 2.4-2.5 (rho0 = 1,
 * c_s^2 = 1/3): U_c = Ma c_s, nu_0 = U_c L_c / Re, nu_s = beta nu_0,
 * eta_p = (1 - beta) nu_0, lambda = Wi L_c / U_c, kappa = nu_s / Sc.  Fills *out
 * (force zero, flags 0) and, if uc is non-null, the characteristic speed U_c.
 * Host only.  Errors: VLB_E_INVALID_ARG for Re, Wi, Sc, Ma, L_c, Lambda_s, Lambda_p
 * <= 0 or beta outside (0, 1]. */
int vlb_params_from_groups(double Re, double Wi, double beta, double Sc, double Ma, double Lc,
                           double Lambda_s, double Lambda_p, vlb_params* out, double* uc);

/* Per-node body force F(x) of the hydrodynamic lattice (the forcing term F_i and the
 * half-force velocity shift of Sec. 3.1; the four-roll mill's force field of Sec. 4.1):
 * device arrays [ny][nx] in the simulation precision, copied into the workspace on the
 * stream, so the caller may free them once the stream has passed this call.  Both null:
 * back to the uniform force of vlb_params.  Errors: VLB_E_INVALID_ARG if exactly one is
 * null, VLB_E_STATE before vlb_bind, VLB_E_HIP. */
int vlb_set_force_field(vlb_sim* sim, const void* fx_dev, const void* fy_dev);

/* Inlet profile for VLB_OPEN x (the channel inlet of Sec. 4.3: a parabolic velocity and
 * the conformation of the steady channel solution, A_xy = lambda u', A_xx = 1 +
 * 2 (lambda u')^2, A_yy = 1): host arrays of ny doubles (u_x, A_xx, A_xy, A_yy, row y at
 * index y), copied before the call returns; u_y = 0 at the inlet.  The inlet ghost column
 * is filled each step by non-equilibrium extrapolation around this profile.  Errors:
 * VLB_E_INVALID_ARG (null array, non-finite value), VLB_E_UNSUPPORTED (x not VLB_OPEN). */
int vlb_set_inlet(vlb_sim* sim, const double* ux, const double* axx, const double* axy,
                  const double* ayy);

/* Equilibrium initial state (Sec. 4.2: populations at equilibrium, zero
 * non-equilibrium part): f = f^eq(rho, u), g = g^eq(A, u).  Device arrays [ny][nx] in
 * the simulation precision; a null array takes rho = 1, u = 0, A = I.  Resets the
 * step counter; the first step uses F~(t-1) = F~(t). */
int vlb_init_equilibrium(vlb_sim* sim, const void* rho, const void* ux, const void* uy,
                         const void* axx, const void* axy, const void* ayy);

/* ---- time stepping and read-out ----------------------------------------------- */

/* Advances nsteps coupled time steps (the coupled update of Sec. 3.1-3.3: streaming and
 * the boundary rules, the hydrodynamic and the three conformation collisions with their
 * source terms), async on the stream; nsteps = 0 does nothing.  Errors: VLB_E_STATE
 * (not bound, parameterised and initialised), VLB_E_INVALID_ARG (nsteps < 0), VLB_E_HIP.
 * A numerical breakdown is not detected here: vlb_monitors reports it. */
int vlb_step(vlb_sim* sim, int64_t nsteps);

/* Current step count (host-side, no synchronization). */
int vlb_get_step(const vlb_sim* sim, int64_t* step);

/* Macroscopic fields at the current time (the moments of Sec. 3.1 and 3.2): rho = sum
 * f_i, u = (sum e_i f_i + F/2) / rho, A_k = sum g^k_i.  Device arrays [ny][nx] in the
 * simulation precision, written on the stream; any may be null; solid nodes read 0.
 * Errors: VLB_E_STATE before vlb_init_equilibrium (or vlb_load_state), VLB_E_HIP. */
int vlb_read_fields(vlb_sim* sim, void* rho, void* ux, void* uy, void* axx, void* axy,
                    void* ayy);

/* History the next step will use: S(t-1) for the three components and u(t-1).
 * Device arrays as for vlb_read_fields. */
int vlb_read_history(vlb_sim* sim, void* sxx, void* sxy, void* syy, void* uxp, void* uyp);

/* Wavefront-reduced monitors: the total of rho and of each conformation component over
 * the fluid nodes (the quantities the CNEBB scheme of Sec. 3.3 conserves), the
 * velocity residual max |u(now) - u(previous call)| (divided by U_c and the call interval
 * it is the steady-state criterion of Sec. 4.1), the largest |u|, and the counts of
 * non-finite nodes and of nodes where A is not positive definite.  Synchronizes the
 * stream.  Returns VLB_E_NONFINITE when any fluid node is non-finite (the breakdown the
 * paper's stability studies record), with *out filled; VLB_E_STATE before
 * initialisation; VLB_E_HIP. */
int vlb_monitors(vlb_sim* sim, vlb_monitor* out);

/* Momentum-exchange force on a solid (Sec. 4.3): over the boundary links (fluid node
 * x_f, direction i with x_f + e_i solid) sum e_i (f_i^post(x_f, t) + f_opp(i)(x_f, t+1)),
 * with the post-collision values of the last step and the populations its boundary
 * rules return.  circle >= 0 (index into vlb_grid.circles) keeps the links into that
 * circle; circle < 0 keeps every solid link (walls, mask solids and circles).  Lattice
 * units (force per unit depth).  Deterministic (fixed-order reduction); synchronizes.
 * Errors: VLB_E_STATE before the first step, VLB_E_INVALID_ARG for a bad circle,
 * VLB_E_UNSUPPORTED for circle < 0 with wet-node walls (circles only there). */
int vlb_drag(vlb_sim* sim, int circle, double* fx, double* fy);

/* ---- checkpoint ------------------------------------------------------------------ */

/* Checkpoint of the full time-stepping state: the post-streaming populations of the four
 * lattices and the history the next step needs (S and u of the previous step, for the
 * time derivative of F~_i, Sec. 3.2), plus the step counter.
 * vlb_state_bytes: bytes of a saved state (a 256-byte header, then the state).
 * vlb_save_state: copies the state into a caller-owned device buffer of at least that
 *   size (async on the stream).  VLB_E_STATE before initialisation, VLB_E_WORKSPACE for a
 *   null or short buffer.
 * vlb_load_state: restores a state saved by a simulation of the same grid, precision and
 *   boundary kinds (checked from the header; else VLB_E_INVALID_ARG and nothing changes);
 *   synchronizes the stream to read the header.  VLB_E_STATE before vlb_set_params. */
int vlb_state_bytes(const vlb_sim* sim, size_t* bytes);
int vlb_save_state(vlb_sim* sim, void* dev, size_t bytes);
int vlb_load_state(vlb_sim* sim, const void* dev, size_t bytes);

/* ---- tuning ------------------------------------------------------------------------ */

/* Tile height of the step kernel (64 x ty nodes per workgroup, ty in {1, 2, 4, 8});
 * results are bit-identical for every choice. */
int vlb_set_tile(vlb_sim* sim, int ty);
/* Stores of the post-collision state: 0 = automatic (non-temporal once the two
 * population buffers exceed the last-level cache), 1 = cached, 2 = non-temporal. */
int vlb_set_store_mode(vlb_sim* sim, int mode);
/* Use hipGraph replay for runs of nsteps >= 2 * chunk (chunk 0 disables graphs). */
int vlb_set_graph_chunk(vlb_sim* sim, int chunk);
/* Launch schedule of the step kernel; results are bit-identical for every choice.
 * tile_order: 1 = XCD bands (consecutive workgroups go round-robin to the 8 XCDs and each
 * XCD sweeps one contiguous band of tile rows, sharing its halo rows in that XCD's L2),
 * 2 = row-major (the whole chip sweeps the grid together), 3 = column strips (each XCD
 * owns one eighth of the tile columns and all XCDs move down the rows together),
 * 0 = automatic (bands while the two population buffers fit the last-level cache,
 * row-major beyond).
 * waves: register budget of the single-precision step kernel, 3 or 4 waves per SIMD
 * (the kernel fits 4 without spilling; 3 leaves the compiler more registers), 0 =
 * automatic (4); double precision always runs at its natural allocation.
 * Errors: VLB_E_INVALID_ARG for other values. */
int vlb_set_schedule(vlb_sim* sim, int tile_order, int waves);

/* ---- adjoint ------------------------------------------------------------------------ */

/* Discrete adjoint of nsteps coupled steps (Sec. 3, Eqs. 31-51, differentiated step by
 * step in reverse order) for domains whose axes are periodic or VLB_WALL, with solid
 * masks and circles (the transposes of half-way and interpolated bounce-back, Sec. 3.3
 * and 4.3, of CNEBB, Sec. 3.3, and of the wall-aware velocity-gradient differences),
 * with any of the constitutive closures above.  The
 * differentiated quantities are the relaxation time lambda, the polymer viscosity
 * eta_p and the per-node body force F(x) (held fixed over the steps; with a uniform
 * force the gradient is still returned per node).  Memory: sqrt(N) checkpointing --
 * the forward pass saves the state every `stride` steps; the backward pass recomputes
 * each segment into `stride` state slots and sweeps it in reverse.  All memory is the
 * caller's 256-byte aligned device workspace of vlb_adjoint_workspace_bytes (it holds
 * ceil(nsteps / stride) + stride states of vlb_state_bytes each, plus adjoint buffers).
 *
 * vlb_adjoint_forward: from the current state, advances nsteps steps (exactly as
 *   vlb_step) and records checkpoints in the workspace.
 * vlb_adjoint_backward: after vlb_adjoint_forward (the simulation not stepped, reloaded
 *   or re-parameterised since), given dL/du of the velocity read out at the last step
 *   (device, [ny][nx], simulation precision), returns dL/dlambda and dL/deta_p (host)
 *   and dL/dF_x, dL/dF_y (device, [ny][nx], double; NULL to skip).  Synchronizes.
 *   Solid nodes get zero force gradients; their entries of dL/du are ignored.
 * vlb_adjoint: both, for the loss L = (1 / 2N) sum_x |u(x, T) - u*(x)|^2 over the N
 *   fluid nodes, with the target u* (device, [ny][nx], simulation precision; values at
 *   solid nodes are ignored); *loss gets L.
 * Errors: VLB_E_UNSUPPORTED (VLB_OPEN x or VLB_WET y), VLB_E_INVALID_ARG,
 * VLB_E_WORKSPACE, VLB_E_STATE (backward without a matching forward), VLB_E_HIP. */
int vlb_adjoint_workspace_bytes(const vlb_sim* sim, int64_t nsteps, int stride, size_t* bytes);
int vlb_adjoint_forward(vlb_sim* sim, int64_t nsteps, int stride, void* workspace_dev,
                        size_t bytes);
int vlb_adjoint_backward(vlb_sim* sim, const void* dL_dux_dev, const void* dL_duy_dev,
                         double* dL_dlambda, double* dL_detap, void* dL_dFx_dev,
                         void* dL_dFy_dev, void* workspace_dev, size_t bytes);
int vlb_adjoint(vlb_sim* sim, int64_t nsteps, int stride, const void* ux_target_dev,
                const void* uy_target_dev, double* loss, double* dL_dlambda, double* dL_detap,
                void* dL_dFx_dev, void* dL_dFy_dev, void* workspace_dev, size_t bytes);

/* ---- batches ----------------------------------------------------------------------- */

/* Many independent simulations of one precision (uneven sizes, parameters, boundary
 * kinds) advanced together: one step launch and one boundary launch per time step
 * cover every member's tiles (a concatenated, XCD-ordered tile list), replayed from a
 * hipGraph.  This is the batched form of the coupled step of Sec. 3 (Eqs. 31-51); each
 * member computes exactly what vlb_step computes for it, bit for bit.
 *
 * sims: n >= 1 handles, all bound, parameterised and initialised, of one precision, on
 * one stream and at the same step; the caller keeps them alive until the batch is
 * destroyed and may read them (vlb_read_fields, vlb_monitors, ...) between batch steps.
 * ty: tile height 1, 2, 4 or 8 for the batch's launches.  workspace_dev: device
 * memory of at least vlb_batch_workspace_bytes, 256-byte aligned, owned by the
 * caller, holding the work lists, member descriptors and the persistent form's work
 * counters.  A member's new parameters, force field or inlet are picked up at the next
 * vlb_batch_step.  Errors:
 * VLB_E_INVALID_ARG (null/mixed members, bad ty), VLB_E_STATE (member not ready,
 * steps differ, or a member was stepped or reloaded outside the batch),
 * VLB_E_WORKSPACE, VLB_E_HIP. */
typedef struct vlb_batch vlb_batch;
int vlb_batch_workspace_bytes(vlb_sim* const* sims, int n, int ty, size_t* bytes);
int vlb_batch_create(vlb_sim* const* sims, int n, int ty, void* workspace_dev, size_t bytes,
                     vlb_batch** out);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid it): vlb_batch_create without a workspace.  The
 * batch's work lists, member descriptors and persistent-form counters go into a static
 * scratch array of 16 MiB that the library holds on each device for the life of the
 * process (the batched 256-run workload needs about 2 MB at ty = 4, 6 MB at ty = 1).
 * The call allocates nothing; the members' device must be current.  One such batch per
 * device at a time: while it lives, a second call on that device fails with VLB_E_STATE
 * (vlb_batch_destroy releases the scratch; the contents are rewritten by the next
 * create).  Batches from vlb_batch_create are unaffected and may coexist with it.
 * Everything else -- members, results, stepping, graphs, the persistent form -- is as
 * for vlb_batch_create, bit for bit.  Errors: those of vlb_batch_create, and
 * VLB_E_WORKSPACE when the lists exceed the scratch (checked before any device work). */
int vlb_batch_create_noalloc(vlb_sim* const* sims, int n, int ty, vlb_batch** out);
/* Advances every member nsteps steps (async on the shared stream). */
int vlb_batch_step(vlb_batch* batch, int64_t nsteps);
/* vlb_read_fields of member `run` (0-based, in creation order). */
int vlb_batch_read_fields(vlb_batch* batch, int run, void* rho, void* ux, void* uy, void* axx,
                          void* axy, void* ayy);
/* hipGraph replay in chunks of 2 * chunk steps (0 disables). */
int vlb_batch_set_graph_chunk(vlb_batch* batch, int chunk);
/* vlb_set_schedule for the batch's launches (the members' own settings are not used;
 * automatic by the size of all members' state together).  The persistent form follows
 * the tile order and always runs three waves per SIMD.  Synchronizes the stream. */
int vlb_batch_set_schedule(vlb_batch* batch, int tile_order, int waves);
/* on = 1: persistent form -- one cooperative launch advances every member up to 256
 * steps (all tiles of a step, a grid-wide barrier, all boundary fills, a barrier, next
 * step).  The grid is as many workgroups as stay resident together; they draw tiles
 * from per-XCD queues (atomic counters in the batch workspace).  Results are
 * bit-identical to the per-step launches (on = 0, the default; also hipGraph-captured
 * when a graph chunk is set).  Errors: VLB_E_UNSUPPORTED without cooperative launch
 * support. */
int vlb_batch_set_persistent(vlb_batch* batch, int on);
void vlb_batch_destroy(vlb_batch* batch);

/* ---- errors ------------------------------------------------------------------------ */
const char* vlb_error_string(int status);
const char* vlb_last_error_detail(void);

#ifdef __cplusplus
}
#endif
#endif /* VLB_H */
