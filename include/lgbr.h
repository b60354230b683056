/*
 * lgbr.h -- C ABI of the MI355X hybrid LAD-GBR right-hand-side library (liblgbr.so).
 *
 * Method: arxiv 2511.18042 (Kumar, Saini, Vadlamani, Chamarthi), "Assessment of
 * gradient-based reconstruction and artificial diffusivity methods in simulating
 * high-speed compressible flows".  The library evaluates the per-Runge-Kutta-stage
 * right-hand side of the compressible Navier-Stokes equations in generalised
 * curvilinear coordinates (Sec. 2.1, Eq. eq:3.1.1 and Eq. tauij) in three forms:
 *   - C-GBR  (Sec. 2.3): centralised gradient-based reconstruction of the
 *     characteristic primitives from explicit sixth-order (MEG6) or compact
 *     fourth-order (MIG4) gradients, MP5 limiting with the wave-appropriate Omega
 *     sensor, curvilinear HLLC fluxes;
 *   - LAD    (Sec. 2.2, Sec. 5): fourth-order explicit central differences (LAD-E4)
 *     with localized artificial shear / bulk viscosity and conductivity, or the
 *     stand-alone sixth-order compact form LAD-C6 with its implicit filter (Sec. 3,
 *     Alg. 1);
 *   - hybrid (Alg. 3, Sec. 5): a troubled-cell flag selects the C-GBR interface flux,
 *     the LAD flux elsewhere (per-cell form), or C-GBR for the whole field when any
 *     interior cell is troubled (the paper's global form);
 * and advances it with the third-order TVD (SSP) Runge-Kutta scheme.
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers owned by the caller; the library never
 *    frees them and never keeps them beyond the call, except where stated (batches).
 *  - Node layout: a field is stored on the ghost-padded node grid of one problem,
 *    i fastest: index = i + N0 * (j + N1 * k) with N_d = n_d + 2 * 5 for the active
 *    directions d < ndim and N_d = 1 for inactive ones.  Nodes are cell centres.
 *    A stack of fields is field-major: field q at [q * N0 N1 N2 + index].
 *  - Q is the physical conserved state (rho, rho u, rho v, rho w, E), FP64, [5][N].
 *    Its ghost layers are rewritten by every call (boundary images), except on
 *    boundaries marked LG_BC_FIXED, whose ghost values the caller owns.
 *  - dQdt receives dQ/dt = -J sum_l (F_{l,i+1/2} - F_{l,i-1/2}) on interior nodes,
 *    FP64, [5][N]; its ghost entries are not written.
 *  - Work is enqueued on the context's HIP stream; no call synchronises the host
 *    except lg_poll_status and lg_create / lg_destroy / lg_batch_create.
 *  - Errors: invalid arguments return LG_EINVAL before anything is enqueued; HIP
 *    launch or allocation failures return LG_EHIP / LG_ENOMEM.  Non-physical states
 *    (rho <= 0, p <= 0 or not finite after an RK stage, the paper's "abrupt
 *    divergence" of Sec. 3.4) are counted on the device and reported by
 *    lg_poll_status as LG_ENONPHYS.
 */
#ifndef LGBR_H
#define LGBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LG_OK = 0,
  LG_EINVAL = -1,
  LG_ENOMEM = -2,
  LG_EHIP = -3,
  LG_ENONPHYS = -4,
  LG_EUNSUPPORTED = -5
} lg_status;

/* boundary conditions (the per-case boundary treatments of Sec. 3) */
enum {
  LG_BC_PERIODIC = 0,          /* periodic images                                      */
  LG_BC_TRANSMISSIVE = 1,      /* zeroth-order extrapolation of every variable        */
  LG_BC_REFLECTIVE = 2,        /* mirror, normal momentum negated (inviscid wall)      */
  LG_BC_NOSLIP_ADIABATIC = 3,  /* mirror, all momentum negated (no-slip adiabatic wall)*/
  LG_BC_FIXED = 4,             /* ghosts owned by the caller (inflow at the IC state)  */
  LG_BC_NOSLIP_ISOTHERMAL = 5  /* no-slip wall held at wall_T (Sec. 4, M2.9 ramp): mirror
                                  with velocity negated, pressure even, temperature odd
                                  about wall_T, density from the equation of state     */
};
enum { LG_GRAD_E6 = 0, LG_GRAD_C4 = 1 };          /* MEG6 / MIG4 gradients (Sec. 2.3)   */
enum { LG_FP64 = 0, LG_MIXED = 1 };               /* FP64 everywhere / FP32 bulk math   */
enum { LG_HYB_PERCELL = 0, LG_HYB_GLOBAL = 1 };   /* hybrid selection (Sec. 5, Alg. 3)   */
enum { LG_SCHEME_CGBR = 0, LG_SCHEME_LAD = 1, LG_SCHEME_HYBRID = 2 };
enum { LG_LAD_E4 = 0, LG_LAD_C6 = 1 };            /* central scheme of LG_SCHEME_LAD        */
enum { LG_RK3 = 0, LG_RK4 = 1 };                  /* time integrator (lg_opts.time_scheme)  */

typedef struct {
  int ndim;            /* 1, 2 or 3 active directions                                 */
  int n[3];            /* interior nodes per direction; 1 for inactive directions     */
  int ng;              /* ghost layers per active direction; must be 5               */
  int bc[3][2];        /* LG_BC_* for the low / high side of every active direction   */
  int curvilinear;     /* 0: Cartesian, spacings h; 1: node metrics + coordinates    */
  double h[3];         /* Cartesian node spacings (unused when curvilinear)          */
  double wall_T[3][2]; /* wall temperature (T_ref = 1) of LG_BC_NOSLIP_ISOTHERMAL
                          faces, > 0; ignored on other faces                        */
} lg_grid;

typedef struct {       /* non-dimensional gas model (Sec. 2.1)                        */
  double gamma;        /* ratio of specific heats                                     */
  double Re;           /* Reynolds number: mu_hat = mu / Re                           */
  double Pr;           /* Prandtl number                                              */
  double Mref;         /* reference Mach number: p = rho T / (gamma Mref^2)           */
  double suth;         /* Sutherland constant S / T_ref                               */
  int viscous;         /* 0: inviscid (no physical viscosity or conduction)           */
} lg_gas;

typedef struct {
  int grad;            /* LG_GRAD_E6 or LG_GRAD_C4                                     */
  int precision;       /* LG_FP64 or LG_MIXED (FP32 reconstruction, limiter, sensor,
                          HLLC and LAD; FP64 state, RK combination, compact solves and
                          flux differences)                                           */
  double cfl;          /* CFL number of the time step (Sec. 3: 0.2)                   */
  double omega_thr;    /* Omega sensor threshold (Sec. 2.3: 0.01)                     */
  double mp_eps;       /* MP criterion threshold (Sec. 2.3: 1e-20)                    */
  double mp_alpha;     /* MP5 alpha (4)                                               */
  double C_mu, C_beta, C_kappa;  /* LAD constants (Sec. 2.2: 0.002, 1.75, 0.01; the
                          paper's runs use C_mu = 0)                                   */
  int hybrid_mode;     /* LG_HYB_PERCELL or LG_HYB_GLOBAL                              */
  double rho_thr;      /* troubled if rho < rho_thr (Sec. 5; negative: never)         */
  double p_thr;        /* troubled if p < p_thr (Sec. 5; negative: never)             */
  int dilate;          /* troubled-flag dilation radius of the per-cell hybrid (3)    */
  int seg;             /* nodes per lane in the strided sweeps (0: default)           */
  int lad_scheme;      /* LG_LAD_E4 (the hybrid's LAD, Sec. 5) or LG_LAD_C6 (the
                          stand-alone LAD scheme of Sec. 3: compact sixth-order
                          gradients and interface fluxes; LG_SCHEME_LAD only)          */
  double filter_alpha; /* alpha_f of the tenth-order implicit filter (Sec. 2.1) that
                          follows the last RK stage wherever that stage ran the LAD-based
                          solver (Alg. 1 FILTER_CALLS, also in the hybrid's LAD phases,
                          Alg. 3): LG_SCHEME_LAD with LAD-E4 or LAD-C6, and hybrid stages
                          that ran LAD; 0 <= alpha_f <= 0.5, 0.5 = no filter          */
  int filter_every_stage; /* 0: filter after the last stage (Alg. 1); 1: after every
                          stage of rk3_step that ran LAD (an alternative reading)      */
  int time_scheme;     /* LG_RK3: SSP-RK3 (Sec. 2.3, every scheme); LG_RK4: the classic
                          four-stage RK4 (Sec. 2.1 names RK4,4 for the LAD solver; LAD-C6
                          filters in its fourth stage, Sec. 5), LG_SCHEME_LAD steps only:
                          rk3_step and batches refuse other schemes (LG_EUNSUPPORTED)    */
} lg_opts;

typedef struct lg_ctx lg_ctx;
typedef struct lg_batch lg_batch;

/* Optional allocator for workspaces (e.g. a framework's caching allocator).
 * alloc(bytes, user) returns device memory or NULL; free_(ptr, user) releases it.
 * Passing NULL functions restores hipMalloc / hipFree.  Affects later lg_create calls. */
lg_status lg_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* user);

/* Create a context for one grid.  node_metrics: device [10][N] FP64 metrics
 * (xi_x, xi_y, xi_z, eta_x, .., zeta_z)/J and J (Sec. 2.1), required when
 * grid->curvilinear, else NULL.  coords: device [3][N] FP64 node coordinates, required
 * when curvilinear (LAD length scales, Sec. 2.2), else NULL.  Both must stay valid for
 * the life of the context.  stream: a hipStream_t (NULL = default stream).
 * Allocates the context's workspace. */
lg_status lg_create(lg_ctx** ctx, const lg_grid* grid, const double* node_metrics, const double* coords,
                    const lg_gas* gas, const lg_opts* opts, void* stream);
void lg_destroy(lg_ctx* ctx);
size_t lg_workspace_bytes(const lg_ctx* ctx);

/* 1 if the context stores one plane of node metrics and LAD grid factors because they do
 * not vary along zeta (a 2D section extruded spanwise, detected at lg_create to 1e-12 of
 * the plane's values), 0 if it stores them at every node, -1 for a null context. */
int lg_metrics_planar(const lg_ctx* ctx);

/* Conservative node metrics from node coordinates (Sec. 2.1; fourth-order central
 * differences as the outer operator so that the discrete metric identities hold).
 * coords [3][N] -> node_metrics [10][N]; values are defined on nodes at least two
 * nodes inside the padded grid.  Allocates and frees a temporary [9][N] buffer. */
lg_status lg_metrics_from_coords(const lg_grid* grid, const double* coords, double* node_metrics,
                                 void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): lg_metrics_from_coords with the same arguments,
 * results and stream ordering, but its [9][N] scratch of inner derivatives lives in a
 * static device array of 9 * LG_NOALLOC_MAX_NODES doubles (72 MiB) that every GPU the
 * library runs on holds from library load until the process ends.  No allocation, no
 * host synchronisation.  Grids whose padded node count N exceeds LG_NOALLOC_MAX_NODES
 * return LG_EUNSUPPORTED before anything is enqueued.  The scratch is shared by every call
 * on a GPU and keeps the last call's contents (each call writes all it reads): calls that
 * overlap on one GPU (different streams, or different host threads without ordering) race;
 * calls ordered on one stream do not.  The stream must belong to the current device. */
#define LG_NOALLOC_MAX_NODES (1LL << 20)
lg_status lg_metrics_from_coords_noalloc(const lg_grid* grid, const double* coords, double* node_metrics,
                                         void* stream);

/* dQdt = C-GBR right-hand side of Q (Sec. 2.3, Alg. 2). */
lg_status cgbr_rhs(lg_ctx* ctx, double* Q, double* dQdt);
/* dQdt = LAD right-hand side of Q (Sec. 2.2, Alg. 1 without the filter): LAD-E4, or
 * LAD-C6 on a context created with lad_scheme = LG_LAD_C6. */
lg_status lad_rhs(lg_ctx* ctx, double* Q, double* dQdt);
/* FILTER_CALLS of Alg. 1: the implicit low-pass filter (Sec. 2.1; Gaitonde-Visbal,
 * tenth order, alpha_f = opts->filter_alpha) of the whole field
 *   alpha_f phi^_{i-1} + phi^_i + alpha_f phi^_{i+1} = sum_{k=0}^{5} a_k/2 (phi_{i+k} + phi_{i-k})
 * applied to the conserved state Q in place along xi, eta, zeta in turn.  Before each
 * direction the ghost layers of that direction are refilled with the boundary images;
 * bounded lines filter their interior nodes with the ghost values as known neighbours,
 * periodic lines are cyclic.  Interior nodes and the ghosts of FIXED faces hold the
 * result; other ghosts hold images of intermediate fields.  rk3_step calls it after the
 * third stage of LG_SCHEME_LAD steps, and in the hybrid's LAD phases (see rk3_step);
 * lg_rk3_stage does not.  LG_EUNSUPPORTED unless alpha_f < 0.5. */
lg_status lad_filter(lg_ctx* ctx, double* Q);
/* dQdt = hybrid right-hand side of Q (Alg. 3, Sec. 5).  flags_in (nullable, uint8 [N])
 * replaces the troubled-cell criterion; flags_out (nullable, uint8 [N]) receives the
 * troubled flags that were used.  LG_EUNSUPPORTED on LG_LAD_C6 contexts (the hybrid's
 * LAD is LAD-E4). */
lg_status hybrid_rhs(lg_ctx* ctx, double* Q, double* dQdt, const uint8_t* flags_in, uint8_t* flags_out);

/* One time step of scheme LG_SCHEME_* on Q in place: the three-stage SSP-RK3 of Sec. 2.3,
 * or the classic four-stage RK4 of Sec. 2.1 when time_scheme = LG_RK4 (LG_SCHEME_LAD only;
 * the filter then follows the fourth stage).  The step size is
 * dt = cfl / max_i sum_l (|xi_l . u| + c |xi_l|) from Q, clipped so that t does not
 * pass t_end; t_inout is a device double that is advanced by dt.  dt stays on the
 * device (no host synchronisation).  Unless filter_alpha = 0.5 the step ends with the
 * implicit filter where its third stage ran the LAD-based solver (Alg. 1; Alg. 3 runs that
 * solver in the hybrid's LAD phases): LG_SCHEME_LAD filters the whole field; under the
 * global hybrid switch the field is filtered when the third stage found no troubled
 * interior node and left alone when it ran C-GBR (Alg. 2 has no filter); under the
 * per-cell switch the lines are filtered whole and the nodes in the dilated troubled set
 * keep their unfiltered values.  In the hybrid, a node whose filtered density or pressure
 * is not positive (or not finite) keeps its unfiltered state.  The decision is taken on the
 * device from the stage's troubled-cell reduction.  With filter_every_stage the same
 * follows every stage. */
lg_status rk3_step(lg_ctx* ctx, int scheme, double* Q, double t_end, double* t_inout);

/* One RK3 stage from given states (for per-stage checks):
 * Us <- a Un + b (Us + dt L(Us)) on interior nodes, with (a, b) = (0, 1), (3/4, 1/4),
 * (1/3, 2/3) for stage 0, 1, 2; ghosts of Us <- ghosts of Un. */
lg_status lg_rk3_stage(lg_ctx* ctx, int scheme, int stage, const double* Un, double* Us, double dt);

/* dt_out (device double) = cfl / max spectral radius of Q (no clipping). */
lg_status lg_compute_dt(lg_ctx* ctx, const double* Q, double* dt_out);

/* Batch of independent problems advanced together: every kernel of a step is one
 * launch over all problems, and nsteps RK3 steps are captured into one HIP graph.
 * All contexts must share ndim, precision, gradient kind, hybrid mode, viscosity and
 * stream.  Q[i] / t[i] are device pointers (state and time of problem i) that must stay
 * valid for the life of the batch; t_end[i] are the end times. */
lg_status lg_batch_create(lg_batch** batch, lg_ctx* const* ctxs, double* const* Q, double* const* t,
                          const double* t_end, int n, int nsteps, int scheme);
lg_status lg_batch_run(lg_batch* batch);      /* one graph launch = nsteps RK3 steps     */
void lg_batch_destroy(lg_batch* batch);

/* Per-launch timing for measurement: while enabled, every launch of the selected kernel
 * class (LG_KC_*, or -1 for all classes) issued through this context is bracketed by a
 * pair of HIP events on the context's stream, up to max_launches launches.  lg_prof_stop
 * synchronises the stream and returns, per class, the summed event time in ms and the
 * number of timed launches (arrays of LG_KC_COUNT entries); it also releases the events.
 * lg_prof_stop_launches does the same and also writes the duration (ms) and class of each
 * timed launch, in issue order, into each_ms / each_class (host arrays of cap entries;
 * *n_out = the number written, at most cap).  A launch that the device-side switch turned
 * into an immediate return is timed like any other; the per-launch durations tell the two
 * apart.  Both return LG_EINVAL when timing was not started. */
enum {
  LG_KC_BC = 0, LG_KC_PRIM, LG_KC_FLAGS, LG_KC_GRAD_E6, LG_KC_GRAD_C4, LG_KC_SENSOR, LG_KC_VISC,
  LG_KC_LAD_NODE, LG_KC_LAD_RAW, LG_KC_GAUSS, LG_KC_LAD_FLUX, LG_KC_SWEEP_X, LG_KC_SWEEP_Y,
  LG_KC_SWEEP_Z, LG_KC_COMBINE, LG_KC_DT, LG_KC_BC_SCALAR, LG_KC_LAD_SWEEP, LG_KC_C6_FACES, LG_KC_FILTER,
  LG_KC_GBR_ITEMS, LG_KC_HYB_ASSEMBLE, LG_KC_FILTER_GUARD, LG_KC_COUNT
};
lg_status lg_prof_start(lg_ctx* ctx, int kernel_class, int max_launches);
lg_status lg_prof_stop(lg_ctx* ctx, double* ms, int* launches);
lg_status lg_prof_stop_launches(lg_ctx* ctx, double* ms, int* launches, float* each_ms, int* each_class, int cap,
                                int* n_out);

/* Launch-shape tuning (no effect on results): seg = nodes per lane of the strided
 * interface sweeps (0 = built-in heuristic, else 2..64); pcr_blocks = persistent
 * workgroups of the PCR line solves (0 = built-in, else 256..65536); zc = planes per
 * chunk of the z-marching stencil kernels (0 = built-in, else 1..1024).  Applies to later
 * calls on the context and to batches created afterwards.  lg_get_tuning reports the
 * values in effect (heuristic values resolved for the context's grid). */
lg_status lg_set_tuning(lg_ctx* ctx, int seg, int pcr_blocks, int zc);
lg_status lg_get_tuning(const lg_ctx* ctx, int* seg, int* pcr_blocks, int* zc);
/* Tile shapes (no effect on results): zm_width = columns along xi of the tiles of the
 * z-marching stencil kernels, which hold 256 columns (32 x 8, 64 x 4 or 128 x 2; 0 restores
 * 64); line_batch = most lines per LDS line tile of the compact solves (1..16; 0 = as many as
 * fit the tile).  Other values return LG_EINVAL.  Applies to later calls on the context and
 * to batches created afterwards; lg_get_tile_shape reports the values in effect. */
lg_status lg_set_tile_shape(lg_ctx* ctx, int zm_width, int line_batch);
lg_status lg_get_tile_shape(const lg_ctx* ctx, int* zm_width, int* line_batch);
/* Line-solve kernels of the compact schemes (no effect on results beyond rounding): bit
 * 3 s + d of mask allows LDS line tiles (all five variables of a few lines in one
 * workgroup) for system s (0 = LAD-C6 gradients, 1 = LAD-C6 interface fluxes, 2 = implicit
 * filter, 3 = MIG4 gradients outside per-cell hybrid stages) along direction d.  Where
 * allowed, tiles are used for the contiguous direction and for strided directions with
 * fewer than 32768 lines (bit 12 set: for strided directions whatever their line count);
 * other lines are solved by PCR per (line, variable) or one lane per line.  Along xi the
 * implicit filter on bounded lines of 128 to 2048 unknowns, the MIG4 gradients (outside the
 * listed lines of per-cell stages) and the LAD-C6 gradients on bounded lines of 130 to 2050
 * nodes, and the LAD-C6 interface fluxes on bounded lines of 129 to 2049 nodes of 2D and 3D
 * grids use the partition method (one wave per line and variable: segment solves joined
 * through their end unknowns) unless bit 13 is set.  Along eta and zeta, lines that are not
 * in tiles are solved in register segments of at most 64 unknowns joined the same way (64
 * lines and one variable per workgroup) unless bit 14 is set: the filter and the MIG4
 * gradients on lines of 16 to 512 unknowns, the LAD-C6 interface fluxes on lines of 16 to
 * 256 faces and the LAD-C6 gradients on periodic lines of 16 to 256 nodes; one lane per
 * line otherwise.  mask in
 * [0, 32767]; -1 restores the default (4095: tiles allowed, bits 12 to 14 clear).
 * lg_get_line_tiles returns the mask in effect (-1 for a null context).  Applies to later
 * calls and to batches created afterwards. */
lg_status lg_set_line_tiles(lg_ctx* ctx, int mask);
int lg_get_line_tiles(const lg_ctx* ctx);
/* Code forms of the LAD kernels and the primitive conversion.  By default the FP32 kernels
 * read fields by 32-bit offsets from a scalar base and convert primitives two nodes per
 * lane, and the LAD coefficient kernel (FP32), node-flux kernel (FP64) and the C-GBR
 * direction sweeps (viscous problems) take a form compiled for 3D curvilinear grids whose
 * metrics are planar along zeta; the kernels fall back by themselves to 64-bit addressing,
 * one node per lane and the general form for fields of 2^32 bytes or more, odd node
 * counts, unaligned state, other grids or inviscid problems.  generic
 * is a bit mask that forces fallbacks so that tests can compare the forms: bit 0 the
 * addressing and node pairs (results bitwise equal), bit 1 the general geometry (FP64
 * bitwise equal; FP32 equal to rounding, the compiler fusing and ordering the arithmetic of
 * the two forms differently); 0 restores the defaults.  Applies to later calls on the
 * context, not to batches.  LG_EINVAL for a null context or generic outside [0, 3]. */
lg_status lg_set_generic_access(lg_ctx* ctx, int generic);

/* Synchronises the context's stream and reads its non-physical node count since the
 * last poll (then resets it).  Returns LG_ENONPHYS when the count is non-zero. */
lg_status lg_poll_status(lg_ctx* ctx, int* nonphys_count);
/* Digital-filter inflow turbulence (Sec. 4: the 3D cases' inflow, with per-component integral
 * length scales in two wall-normal zones and the strong Reynolds analogy for temperature
 * and density).  One generator per context writes the FIXED ghost layers of the low-xi
 * face; each update:
 *   1. filters a plane of standard normal numbers (supplied by the caller, rnd, device,
 *      [3][ny + 2 pad][nz], pad = the largest filter support along eta, see
 *      lg_df_random_count) along zeta (periodic) and eta with the coefficients
 *      b_i = exp(-pi |i| / n) / norm, |i| <= ceil(2 n), n = length scale / spacing (eta:
 *      the row's spacing and zone, inner where y <= y_lim);
 *   2. correlates it in time: psi <- psi exp(-pi dt / 2T) + new sqrt(1 - exp(-pi dt / T)),
 *      T = Ix / U_ref (first update: psi = new);
 *   3. forms u' = a11 psi_u, v' = a21 psi_u + a22 psi_v, w' = a33 psi_w (a: Cholesky
 *      factor of R11, R21, R22, R33), T'/T = -(gamma - 1) M_sra^2 U u' / (U_ref^2 T) (the
 *      strong Reynolds analogy at the local mean Mach number; T in units of the
 *      reference temperature), rho = rho_mean (1 - T'/T), p unchanged, and writes
 *      (rho, U + u', V + v', w', p) as
 *      conserved values into every ghost layer of the low-xi face (interior eta, zeta).
 * The context needs ndim >= 2 and LG_BC_FIXED on the low-xi face; ny = n[1], nz = n[2]
 * (1 in 2D).  Profile arrays are host memory, copied at creation. */
typedef struct {
  int ny, nz;              /* inflow plane: interior eta rows and zeta columns           */
  const double* dy;        /* [ny] row spacings along eta (> 0)                          */
  const double* y;         /* [ny] wall distance of each row (zone selection)           */
  double dz;               /* spanwise spacing (> 0; unused in 2D)                       */
  double y_lim;            /* inner zone: y <= y_lim                                     */
  double Iy[3][2];         /* eta length scales of u, v, w: inner, outer (> 0)           */
  double Iz[3], Ix[3];     /* zeta and streamwise length scales of u, v, w (> 0)         */
  double U_ref;            /* Taylor convection velocity and analogy velocity (> 0)      */
  const double* mean;      /* [4][ny] mean rho (> 0), U, V, T                           */
  const double* rey;       /* [4][ny] Reynolds stresses R11, R21, R22, R33 (R_ii >= 0)  */
  double M_sra;            /* reference Mach number of the strong Reynolds analogy        */
  double p;                /* inflow pressure (> 0)                                      */
} lg_df_spec;
typedef struct lg_df lg_df;
lg_status lg_df_create(lg_ctx* ctx, const lg_df_spec* spec, lg_df** out);
/* doubles of rnd one update consumes: 3 (ny + 2 pad) nz */
lg_status lg_df_random_count(const lg_df* df, long long* count);
/* One update on the context's stream; dt < 0 takes the context's device time step (the
 * last step's), else dt; first != 0 starts the time correlation.  Q: the state whose
 * inflow ghosts are written (device). */
lg_status lg_df_update(lg_df* df, const double* rnd, double* Q, double dt, int first);
void lg_df_destroy(lg_df* df);

/* Switching record of the hybrid (Sec. 5: the share of the run spent on each scheme):
 * every hybrid stage of the context (hybrid_rhs, rk3_step, lg_rk3_stage, batches) counts
 * one, and one more in *troubled_stages when a node was troubled at its start (global
 * switch: the stage ran on C-GBR; per-cell switch: some interfaces did).  Synchronises
 * the context's stream; reset != 0 zeroes both counters after reading.  Counters wrap
 * after 2^32 stages. */
lg_status lg_switch_stats(lg_ctx* ctx, int* hybrid_stages, int* troubled_stages, int reset);

const char* lg_strerror(lg_status s);

#ifdef __cplusplus
}
#endif

#endif /* LGBR_H */
