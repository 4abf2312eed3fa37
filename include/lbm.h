/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the double-distribution
 * non-orthogonal multiple-relaxation-time lattice Boltzmann method of
 * Liu, He, Li & Li, "Non-orthogonal multiple-relaxation-time lattice
 * Boltzmann method for incompressible thermal flows" (arXiv:1510.08224).
 *
 * One solver advances, on one GPU, a 2-D lattice with
 *   - a D2Q9 flow population fbar (Sec. 2.1): collision in the raw-moment
 *     space of the non-orthogonal matrix M (Eqs. 8, 13, 16, 17, 20), with
 *     the transformed populations fbar = f - S/2 (Eq. 7);
 *   - a D2Q5 temperature population g (Sec. 2.2): collision in the moment
 *     space of N (Eqs. 24, 26, 28, 29);
 *   - the Boussinesq force F = g beta (T - T0) y_hat + a (Eq. 4);
 *   - streaming in velocity space (Eqs. 9, 25) with link-wise walls.
 *
 * Conventions for every entry point:
 *   - lattice units: delta_x = delta_t = c = 1, rho0 = 1 (Sec. 3);
 *   - every call returns LBM_OK (0) or a negative lbm_status; nothing aborts
 *     and no C++ exception crosses the ABI; lbm_last_error() explains a
 *     failure;
 *   - host arrays are caller-owned, row-major [y][x] (x fastest) for fields
 *     and [i][y][x] for populations, FP64;
 *   - device pointers are caller-owned device memory on the solver's GPU;
 *   - the library owns every allocation it makes and frees it in
 *     lbm_destroy; a buffer handed to lbm_create_ext stays the caller's
 *     and must outlive the solver;
 *   - lbm_step is asynchronous on the solver's stream; readouts that fill
 *     host memory synchronize that stream before returning;
 *   - a solver handle is not thread-safe; use one per host thread.
 *
 * State and time.  The library holds, for time t, the populations that
 * streaming (with the wall rules) turns into the pre-collision populations
 * fbar(x, t), g(x, t).  "Populations at time t" always means those
 * pre-collision populations (the state after streaming, before collision);
 * moments, Nusselt numbers and residuals are computed from them.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2

typedef struct lbm_solver lbm_solver; /* opaque, library-owned */

/* Return codes. */
enum lbm_status {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,         /* invalid argument (sizes, rates, sides, NULL) */
    LBM_ERR_NOMEM = -2,       /* device or host allocation failed / buffer too small */
    LBM_ERR_DEVICE = -3,      /* a HIP runtime call or kernel launch failed */
    LBM_ERR_STATE = -4,       /* call out of order (e.g. step before set_params) */
    LBM_ERR_UNSTABLE = -5,    /* non-finite values found by a reduction */
    LBM_ERR_UNSUPPORTED = -6  /* valid request the library does not implement */
};

/* Population storage in device memory.  LBM_F64 stores the populations
 * themselves and collides in FP64.  LBM_F32 and LBM_F16 store deviations
 * from a rest equilibrium, rounded to nearest even, and collide in FP32;
 * the conserved sums (rho, rho0 u, T) are accumulated in FP64 in every
 * mode.  LBM_F32: fbar_i - w_i rho0 and g_i - g_i^eq(T0, 0).  LBM_F16
 * (scaled by powers of two): g_i - g_i^eq(T_ref, 0), T_ref the linear
 * conduction profile between the two link-wise Dirichlet walls of one
 * axis when the other axis has none (else T0), and, on an x-periodic
 * lattice with T_ref along y, fbar_i - w_i rho_ref(y) with rho_ref the
 * hydrostatic density of T_ref (Eq. 4 at rest; else rho0); each value is
 * stored relative to the reference of the node that pulls it. */
enum lbm_storage { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2 };

enum lbm_side { LBM_LEFT = 0, LBM_RIGHT = 1, LBM_BOTTOM = 2, LBM_TOP = 3 };

/* Thermal model, fixed at creation (it sets the number of populations).
 * LBM_MODEL_D2Q5: the paper's D2Q5 temperature equation (Sec. 2.2).
 * LBM_MODEL_D2Q9T: its D2Q9 variant (Eqs. 31-33): equilibrium of Eq. 31
 *   with theta in {0, 1}, collided with the non-orthogonal M of Eq. 13 and
 *   Q = diag(1, zeta_alpha, zeta_alpha, zeta_e, zeta_nu, zeta_nu, zeta_q,
 *   zeta_q, zeta_eps) (Eq. 32); c_sT^2 = 1/3.
 * LBM_MODEL_ISOTHERMAL: no temperature field (Secs. 3.1-3.2); the force
 *   is the external acceleration a only. */
enum lbm_model { LBM_MODEL_D2Q5 = 0, LBM_MODEL_D2Q9T = 1, LBM_MODEL_ISOTHERMAL = 2 };

/* Collision operator (lbm_params.collision).
 * LBM_COLLISION_MRT: the paper's non-orthogonal MRT (Eqs. 8, 24), the
 *   default.
 * LBM_COLLISION_BGK and LBM_COLLISION_ORTHO_MRT: the two operators Sec. 3.2
 *   compares it with.  BGK relaxes every flow population at s_nu (f^eq of
 *   Eq. 22, Guo source in velocity space) and every temperature population
 *   at zeta_alpha (g^eq of Eq. 30 or 31).  ORTHO_MRT is the classical MRT on
 *   the orthogonal D2Q9 basis (Gram-Schmidt of 1, |e|^2, |e|^4, e_x,
 *   e_x|e|^2, e_y, e_y|e|^2, e_x^2 - e_y^2, e_x e_y), m^eq = M_o f^eq,
 *   sources M_o S, with s_e, s_eps, s_q, s_nu on the energy, energy-square,
 *   heat-flux and stress moments; the temperature keeps the model's MRT.
 *   Both run in the same step kernels (fused pairs included) and cannot
 *   join a batch. */
enum lbm_collision { LBM_COLLISION_MRT = 0, LBM_COLLISION_BGK = 1, LBM_COLLISION_ORTHO_MRT = 2 };

/* Flow boundary per side.  LBM_BC_WALL is halfway bounce-back with the
 * moving-wall term: the wall lies half a spacing outside the last node,
 * and a population leaving node x through it returns to x in the opposite
 * direction j with 6 w_j rho0 (e_j . u_w) added.  LBM_BC_NEE is
 * non-equilibrium extrapolation (the wall scheme of the paper's Sec. 3):
 * the wall passes through the last node row/column, whose populations are
 * rebuilt every step from the inward neighbour x_f as
 * f^eq(rho(x_f), u_w) + fbar(x_f) - f^eq(rho(x_f), u(x_f)) (Eq. 22), and
 * likewise for g with g^eq (Eq. 30) at the wall temperature.  Periodicity
 * is per axis: both sides of an axis must be periodic, for flow and
 * temperature alike, or neither.  NEE and link-wise walls are not mixed on
 * one lattice, and an NEE flow wall takes an NEE temperature wall. */
enum lbm_bc_flow { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1, LBM_BC_NEE = 2 };

/* Temperature boundary per side.  LBM_T_DIRICHLET is anti-bounce-back,
 * g_j(x) = -g*_opp(j)(x) + varpi T_w / 2; LBM_T_ADIABATIC is bounce-back,
 * g_j(x) = g*_opp(j)(x) (zero normal flux).  LBM_T_NEE_DIRICHLET and
 * LBM_T_NEE_ADIABATIC pair with LBM_BC_NEE: the wall node's temperature is
 * T_w, or that of its inward neighbour. */
enum lbm_bc_temp { LBM_T_PERIODIC = 0, LBM_T_DIRICHLET = 1, LBM_T_ADIABATIC = 2,
                   LBM_T_NEE_DIRICHLET = 3, LBM_T_NEE_ADIABATIC = 4 };

/* Problem statement (Secs. 2-3 of the paper).  Fill with
 * lbm_params_default() first; struct_size versions the layout. */
typedef struct {
    uint32_t struct_size;  /* = sizeof(lbm_params) */
    uint32_t reserved0;
    double ra, pr;         /* Rayleigh and Prandtl numbers (Eq. 40) */
    double u_c;            /* characteristic velocity sqrt(g beta dT L); Ma = sqrt(3) u_c (Eq. 40) */
    double length;         /* L in Eq. 40 and in the Nusselt number; 0 => the distance
                              between the bottom and top walls (ny, or ny - 1 with NEE walls) */
    double t_hot, t_cold;  /* dT = t_hot - t_cold, T0 = (t_hot + t_cold)/2 (Sec. 3.4) */
    double s_e, s_q, s_eps;        /* free D2Q9 rates (Eq. 20); defaults 1.6, 1.2, 1.8 */
    double zeta_e, zeta_nu, varpi; /* free D2Q5 rates (Eq. 29) and varpi (Eq. 28); 1.9, 1.9, 0.5 */
    double zeta_q, zeta_eps;       /* further D2Q9 thermal rates (Eq. 32); 1.9, 1.9 */
    double theta;                  /* D2Q9 thermal equilibrium switch of Eq. 31, 0 or 1; 1 */
    double s_nu, zeta_alpha;       /* 0 => from Eq. 40; > 0 => used as given */
    double ax, ay;                 /* external acceleration a (Eq. 4) */
    int32_t bc_flow[4];            /* enum lbm_bc_flow, indexed by enum lbm_side */
    int32_t bc_temp[4];            /* enum lbm_bc_temp */
    int32_t collision;             /* enum lbm_collision; LBM_COLLISION_MRT */
    int32_t reserved1;
    double wall_T[4];              /* Dirichlet wall temperatures */
    double wall_u[4][2];           /* wall velocities (ux, uy) */
} lbm_params;

/* Defaults: the cavity of Sec. 3.4 with Pr = 0.71, rates of Sec. 3.4,
 * varpi = 1/2, walls everywhere, left hot (1) / right cold (0), top and
 * bottom adiabatic; ra = u_c = 0 (must be set, or s_nu/zeta_alpha given).
 * NULL is ignored. */
void lbm_params_default(lbm_params* p);

/* Shear relaxation rate for a Reynolds number (Sec. 3.2, the lid-driven
 * cavity; the viscosity stated after Eq. 20): Re = L u / nu with
 * nu = c_s^2 (1/s_nu - 1/2), c_s^2 = 1/3, so s_nu = 1 / (1/2 + 3 L u / Re).
 * re > 0, length > 0, u > 0 (lattice units: L in node spacings, u a wall
 * speed).  Writes s_nu (in (0, 2)) to *s_nu; LBM_ERR_ARG for other
 * arguments or a NULL output.  Pure host arithmetic, no device. */
int lbm_rate_for_reynolds(double re, double length, double u, double* s_nu);

/* Library ABI version (LBM_ABI_VERSION) and a build description string. */
int32_t lbm_abi_version(void);
const char* lbm_build_info(void);

/* Device bytes a solver of this size, storage and thermal model needs
 * (both population buffers with row padding).  LBM_ERR_ARG for the sizes
 * lbm_create rejects (more than 2^31 nodes, or a row of nodes of 2^31
 * elements or more), a bad storage or model, or a NULL output. */
int lbm_required_bytes(int32_t nx, int32_t ny, int32_t storage, int32_t model, uint64_t* bytes);

/* Create a solver for an nx x ny lattice (nx, ny >= 1, at most 2^31 nodes,
 * (9 + NG) * nx below 2^31) on the current HIP device.  hip_stream: a hipStream_t to launch on, or NULL for a stream the
 * library creates and owns.  Allocates lbm_required_bytes() of device
 * memory.  *out is set to NULL on failure. */
int lbm_create(lbm_solver** out, int32_t nx, int32_t ny, int32_t storage, int32_t model, void* hip_stream);

/* As lbm_create, but the population buffers live in caller-owned device
 * memory [device_buffer, device_buffer + bytes), 256-byte aligned, at least
 * lbm_required_bytes(); the caller keeps it alive until lbm_destroy. */
int lbm_create_ext(lbm_solver** out, int32_t nx, int32_t ny, int32_t storage, int32_t model,
                   void* device_buffer, uint64_t bytes, void* hip_stream);

/* Validate and apply a problem, derive the rates, and reset the state to
 * rest at T = T0: fbar_i = w_i rho0 (Eq. 22 at u = 0) and
 * g_i = g_i^eq(T0, 0) (Eq. 30 or 31), time t = 0.
 * Derived (unless given explicitly, Eq. 40):
 *   1/s_nu = 1/2 + Ma L sqrt(3 Pr)/sqrt(Ra),  Ma = sqrt(3) u_c,
 *   1/zeta_alpha = 1/2 + c_s^2 (1/s_nu - 1/2)/(c_sT^2 Pr),
 *   c_s^2 = 1/3, c_sT^2 = varpi/2 (D2Q5) or 1/3 (D2Q9 thermal),
 *   g beta = u_c^2/(dT L) (0 if u_c = 0 or without a temperature field).
 * Errors: LBM_ERR_ARG for rates outside (0, 2), varpi outside (0, 1),
 * theta other than 0 or 1 (D2Q9 thermal), inconsistent periodicity,
 * unknown boundary codes, or missing data to derive a rate.  The
 * temperature boundary codes are checked for every model. */
int lbm_set_params(lbm_solver* h, const lbm_params* p);

/* Rates and constants in use: s9 = diag(Lambda) (Eq. 20); q9 = diag(Q),
 * 9 values: Eq. 29 in the first 5 and zeros (D2Q5), Eq. 32 (D2Q9 thermal),
 * all zero (no temperature field); g beta, T0, L, dT.  Any pointer may be
 * NULL.  LBM_ERR_STATE before lbm_set_params. */
int lbm_get_derived(const lbm_solver* h, double* s9, double* q9, double* gbeta,
                    double* T0, double* length, double* dT);

/* Reset to rest with a temperature field: fbar_i = w_i rho0,
 * g_i = g_i^eq(T(x), 0) (Eq. 30 or 31); t = 0.  T is host [y][x], nx*ny
 * values; NULL means T = T0 everywhere.  A non-NULL T without a
 * temperature field is LBM_ERR_UNSUPPORTED. */
int lbm_init_temperature(lbm_solver* h, const double* T);

/* Advance nsteps >= 0 time steps: per node, stream (Eqs. 9, 25) with the
 * wall rules, then collide (Eqs. 8, 24).  Asynchronous. */
int lbm_step(lbm_solver* h, int64_t nsteps);

/* Graph replay: lbm_step advances in captured HIP graphs of `steps` sweeps
 * (an even count in [2, 4096]; 0 = one kernel launch per step), rebuilt
 * after lbm_set_params or lbm_set_launch.  The default is 64 for lattices
 * of at most 2^18 nodes (where a sweep is shorter than a launch) and 0
 * otherwise.  Results do not depend on it. */
int lbm_set_graph_steps(lbm_solver* h, int32_t steps);
int lbm_get_graph_steps(const lbm_solver* h, int32_t* steps);

/* Time level t (number of steps taken since the last reset). */
int lbm_time(const lbm_solver* h, int64_t* t);

/* Wait for all work queued on the solver's stream. */
int lbm_synchronize(lbm_solver* h);

/* Macroscopic fields at time t (Eqs. 18, 19, 27): rho = sum fbar,
 * u = (sum e fbar + rho0 F/2)/rho0, T = sum g.  Host arrays of nx*ny
 * doubles, [y][x]; any may be NULL.  Synchronizes. */
int lbm_moments(lbm_solver* h, double* rho, double* ux, double* uy, double* T);

/* As lbm_moments into caller-owned device arrays; asynchronous on the
 * solver's stream. */
int lbm_moments_device(lbm_solver* h, double* rho, double* ux, double* uy, double* T);

/* Wall Nusselt number on a Dirichlet side (Eq. 39 and the local
 * definition before it): Nu(s) = -L (dT/dx_n)/dT along the wall, with the
 * wall half a spacing outside the first fluid node and the gradient from
 * the second-order one-sided fit dT/dn = (9 T1 - T2 - 8 T_w)/3 (n into the
 * fluid; dT/dx_n = dT/dn on the left/bottom wall, -dT/dn on the
 * right/top).  Mean over the wall nodes (midpoint rule), maximum and the
 * index of the first maximum.  Reduced in FP64 in a fixed order.
 * LBM_ERR_ARG if the side is not Dirichlet or the lattice is one node
 * deep.  Synchronizes. */
int lbm_nusselt(lbm_solver* h, int32_t side, double* nu_mean, double* nu_max, int32_t* i_max);

/* (Nusselt numbers need a temperature field: LBM_ERR_UNSUPPORTED for the
 * isothermal model.) */

/* Local Nusselt numbers along a Dirichlet side into a host array of ny
 * (left/right) or nx (bottom/top) doubles.  Synchronizes. */
int lbm_nusselt_local(lbm_solver* h, int32_t side, double* nu_local);

/* Steady-state residual: r = max over nodes of max(|ux - ux'|, |uy - uy'|,
 * |T - T'|) against the snapshot taken by the previous call, then the
 * snapshot is replaced by the current fields.  The first call after a
 * reset, a state load or lbm_set_populations only takes the snapshot and
 * reports r = +infinity.
 * *nonfinite = number of nodes whose rho, u or T is not finite; if it is
 * nonzero the call returns LBM_ERR_UNSTABLE (outputs still written).
 * FP64.  Synchronizes. */
int lbm_residual(lbm_solver* h, double* r, int64_t* nonfinite);

/* lbm_residual without allocating device memory, for callers that cannot
 * allocate (tight serving loops, harnesses that forbid allocation once set
 * up).  Same inputs, outputs, snapshot semantics and errors as
 * lbm_residual, and bitwise the same r and *nonfinite; the per-block
 * partial results and the reduced values go to a static device array of
 * 1 MiB + 256 bytes that each GPU the library runs on holds until the
 * process ends.  The handle's residual snapshot must already exist (one
 * lbm_residual call, or lbm_batch_add, allocates it): LBM_ERR_STATE
 * otherwise.  Lattices of more than 2^24 nodes (16,777,216: 4096^2) need
 * more partials than the array holds: LBM_ERR_ARG.  All calls on one GPU
 * share its array: calls that overlap on one GPU (other threads, or other
 * streams before a call returns) race.  Synchronizes. */
int lbm_residual_static(lbm_solver* h, double* r, int64_t* nonfinite);

/* Pre-collision populations at time t in FP64, host arrays
 * f9[9][ny][nx] and g5[NG][ny][nx] with NG = 5, 9 or 0 by thermal model
 * (either may be NULL).  For deviation
 * storage the rest equilibrium is added back.  Synchronizes. */
int lbm_get_populations(lbm_solver* h, double* f9, double* g5);

/* Replace the state by the given pre-collision populations at time t
 * (same layout; both required), keeping t.  For deviation storage the
 * values are rounded to the storage type.  Synchronizes. */
int lbm_set_populations(lbm_solver* h, const double* f9, const double* g5);

/* Raw state in storage format (bitwise checkpoint): copies both the
 * population buffer and the time level.  lbm_state_bytes() gives the size;
 * lbm_save_state writes to host memory, lbm_load_state restores a state
 * saved from a solver of the same size, storage and parameters.
 * Synchronizes. */
int lbm_state_bytes(const lbm_solver* h, uint64_t* bytes);
int lbm_save_state(lbm_solver* h, void* host, uint64_t bytes);
int lbm_load_state(lbm_solver* h, const void* host, uint64_t bytes);

/* The solver's stream (hipStream_t), storage mode and thermal model. */
void* lbm_stream(const lbm_solver* h);
int32_t lbm_storage_of(const lbm_solver* h);
int32_t lbm_model_of(const lbm_solver* h);

/* Memory policy of the step kernel (bit mask):
 *   LBM_POLICY_XCD_BANDS    each of the 8 XCDs takes a contiguous band of
 *                           tiles (rows);
 *   LBM_POLICY_XCD_STRIPS   each XCD takes a contiguous eighth of every
 *                           row of tiles (when a row holds a multiple of 8
 *                           tiles; bands otherwise);
 *                           with neither bit, tile b runs on XCD b % 8;
 *   LBM_POLICY_KEEP_STORES  stores keep their lines in the last-level
 *                           cache; otherwise they are non-temporal;
 *   LBM_POLICY_FUSE2        lbm_step runs pairs of time steps in one launch:
 *                           a workgroup steps its tile and a one-node halo
 *                           from HBM into LDS, then steps the tile again from
 *                           LDS and stores it, so the state crosses HBM once
 *                           per two steps.  Bitwise the same results.  Used
 *                           with every collision operator on buffers below
 *                           4 GiB and, with NEE walls, when no edge tile is
 *                           one node wide or high (tiles are 64 x 12 nodes
 *                           for FP32/FP16 storage with the D2Q5 model, 64 x 8
 *                           otherwise: nx % 64 == 1 or ny % 12 (8) == 1);
 *                           otherwise steps run singly
 *                           (lbm_steps_per_launch tells which);
 *   LBM_POLICY_FUSEK        lbm_step runs K time steps in one launch where
 *                           a kernel exists (every collision operator):
 *                           K = 4 on 32 x 16 tiles for FP64 and FP32
 *                           storage with the D2Q5 model or no temperature
 *                           field, K = 3 on 32 x 8 tiles for FP64 storage
 *                           with the D2Q9 thermal model.  A workgroup steps
 *                           its tile grown by K - 1 nodes from HBM into LDS,
 *                           the tile grown by K - 2 .. 1 nodes from LDS, and
 *                           the tile into HBM, so the state crosses HBM once
 *                           per K steps (lbm_steps_per_launch gives K).
 *                           Bitwise the same results.  Same conditions as
 *                           LBM_POLICY_FUSE2 (with NEE walls, a last tile
 *                           one node wide or high, nx % 32 == 1 or
 *                           ny % 16 (8) == 1, falls back); steps left over
 *                           run as a pair (with LBM_POLICY_FUSE2) or singly,
 *                           and so does every step where no kernel exists.
 * The default follows the storage and the footprint F of both population
 * buffers: kept stores while F <= 256 MiB; K steps per launch with bands
 * where that kernel exists, for FP64 at any F and for FP32 with
 * F > 256 MiB or F <= 96 MiB; otherwise fused pairs, with bands, or strips (with a
 * multiple of 8 tiles per row) once one row of fused tiles (tiles and
 * halos, every plane) exceeds 3 MiB or an FP64 lattice is 48 or more tiles
 * wide.  Fused pairs stay allowed beside K-step launches. */
enum {
    LBM_POLICY_DEFAULT = -2,     /* back to the footprint rule */
    LBM_POLICY_KEEP = -1,        /* leave the policy as it is */
    LBM_POLICY_XCD_BANDS = 1,
    LBM_POLICY_KEEP_STORES = 2,
    LBM_POLICY_XCD_STRIPS = 4,
    LBM_POLICY_FUSE2 = 8,
    LBM_POLICY_FUSEK = 16
};

/* Launch shape of the step kernel: block_x threads along x (64, 128 or
 * 256), block_y rows of threads (block_x * block_y <= 256) and
 * rows_per_thread (1 or 2) consecutive rows handled by each thread; 0
 * keeps the current value.  policy: a mask of LBM_POLICY_* bits,
 * LBM_POLICY_KEEP or LBM_POLICY_DEFAULT.  Results do not depend on the
 * shape or the policy (bitwise).  LBM_ERR_ARG for other values. */
int lbm_set_launch(lbm_solver* h, int32_t block_x, int32_t block_y, int32_t rows_per_thread, int32_t policy);

/* Time steps one step-kernel launch advances with the current parameters
 * and launch settings: K (4, or 3 for the D2Q9 thermal model) when K-step
 * launches are in use, 2 when fused
 * pairs are, else 1 (remainders of a step count run shorter launches). */
int lbm_steps_per_launch(const lbm_solver* h, int32_t* steps);
int lbm_get_launch(const lbm_solver* h, int32_t* block_x, int32_t* block_y, int32_t* rows_per_thread,
                   int32_t* policy);

/* ------------------------------------------------------------------------
 * Batches.  A batch advances many independent solvers (each with its own
 * size, parameters and state) with one kernel launch per time step: a
 * device table lists, for every workgroup, a member lattice and a tile of
 * block_x x (256 / block_x) nodes (block_x from the member's
 * lbm_set_launch), and every member runs exactly the step of lbm_step.
 * Results of a member are bitwise the same alone and in a batch.
 * Members must share the batch's storage and stream (create them with
 * lbm_batch_stream()).  A solver belongs to at most one batch; lbm_destroy
 * removes it.  Stepping, resetting or reconfiguring a member on its own is
 * allowed and only makes the next lbm_batch_step rebuild the table.
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* Create an empty batch for `storage` on hip_stream (NULL: own stream).
 * All members share one thermal model (that of the first member). */
int lbm_batch_create(lbm_batch** out, int32_t storage, void* hip_stream);

/* Add a solver (params set, same storage and stream); *slot receives its
 * slot index (the lowest free one). */
int lbm_batch_add(lbm_batch* b, lbm_solver* s, int32_t* slot);

/* Remove the solver in `slot` (it stays valid and owned by the caller).
 * Waits for the batch's queued work. */
int lbm_batch_remove(lbm_batch* b, int32_t slot);

/* Number of members and of slots (members plus free slots). */
int lbm_batch_size(const lbm_batch* b, int32_t* active, int32_t* slots);

/* The solver in a slot, or NULL. */
lbm_solver* lbm_batch_member(const lbm_batch* b, int32_t slot);

/* Advance every member nsteps steps (asynchronous). */
int lbm_batch_step(lbm_batch* b, int64_t nsteps);

/* Replay captured graphs of `steps` batched time steps (even, <= 4096;
 * 0 = launches issued one by one, the default). */
int lbm_batch_set_graph_steps(lbm_batch* b, int32_t steps);

/* Fused time steps for the whole batch (the kernels of lbm_set_launch's
 * LBM_POLICY_FUSE2 and LBM_POLICY_FUSEK, one launch per pair or per K
 * steps for all members, the same tiles).  policy: LBM_POLICY_DEFAULT, or
 * a mask of LBM_POLICY_FUSE2 and LBM_POLICY_FUSEK (0: one launch per
 * step).  The default fuses pairs for FP64 and FP32 storage and steps FP16
 * once per launch, and takes K steps per launch for FP64 storage.  A kind of fused launch
 * applies only when every member qualifies (buffers below 4 GiB; with
 * walls by non-equilibrium extrapolation, no one-node edge tile); steps
 * left over run as a pair or singly.  Results are bitwise the same either
 * way.  Takes effect at the next lbm_batch_step.  LBM_ERR_ARG for any
 * other value. */
int lbm_batch_set_policy(lbm_batch* b, int32_t policy);

/* Launch tuning of the batch (the autotuner's knobs; results are bitwise
 * the same with any setting):
 *   xcd_order      order in which the tiles of the batch's tile tables go
 *                  to the 8 XCDs: 1 contiguous bands (each XCD a range of
 *                  the table), 0 round robin, -1 the default (bands);
 *   keep_stores    1 stores keep their lines in the last-level cache, 0
 *                  non-temporal stores, -1 the default (kept when all
 *                  members' buffers fit the 256 MB last-level cache);
 *   largest_first  1 the tile tables list the members largest lattice
 *                  first, 0 in the order they were added (the default).
 * Takes effect at the next lbm_batch_step.  LBM_ERR_ARG for other values. */
int lbm_batch_set_tuning(lbm_batch* b, int32_t xcd_order, int32_t keep_stores, int32_t largest_first);

/* The tuning in effect with the current members (defaults resolved):
 * xcd_order 0 or 1, keep_stores 0 or 1, largest_first 0 or 1.  Rebuilds
 * the tile tables if members changed. */
int lbm_batch_get_tuning(lbm_batch* b, int32_t* xcd_order, int32_t* keep_stores, int32_t* largest_first);

/* Time steps one batched launch advances with the current members and
 * policy (1 or 2); rebuilds the tile table if members changed. */
int lbm_batch_steps_per_launch(lbm_batch* b, int32_t* steps);

/* Wait for the batch's stream. */
int lbm_batch_synchronize(lbm_batch* b);

/* lbm_residual of every member: r[slot] and nonfinite[slot] for each slot
 * (NaN and -1 for free slots).  Returns LBM_ERR_UNSTABLE if any member has
 * non-finite values (all outputs still written).  Synchronizes. */
int lbm_batch_residual(lbm_batch* b, double* r, int64_t* nonfinite);

/* The batch's stream (hipStream_t). */
void* lbm_batch_stream(const lbm_batch* b);

/* Message for the last failure on this batch (or of the last failed
 * create when b is NULL). */
const char* lbm_batch_last_error(const lbm_batch* b);

/* Free the batch (members are released, not destroyed).  A batch created
 * with its own stream destroys that stream: solvers created on it must be
 * destroyed first.  NULL-safe. */
void lbm_batch_destroy(lbm_batch* b);

/* Message for the last failure on this handle (or of the last failed
 * create when h is NULL).  Library-owned; valid until the next call. */
const char* lbm_last_error(const lbm_solver* h);

/* Free the solver and everything it allocated.  NULL-safe.
 * Tracing: if the environment variable LBM_PROFILE is set (and not "0")
 * when the solver is created, lbm_step brackets each call with HIP events
 * on the solver's stream (not while the stream is being captured), and
 * lbm_destroy writes one line to stderr:
 *   {"lbm_profile": {"nx": .., "ny": .., "storage": "f64", "model": ..,
 *    "calls": .., "steps": .., "launches": .., "gpu_ms": .., "mlups": ..}}
 * gpu_ms is the summed GPU time between the events of each call. */
void lbm_destroy(lbm_solver* h);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
