/*
 * esdg.h -- C ABI of the MI355X (gfx950) flux-differencing DGSEM library.
 *
 * The library evaluates and integrates the method-of-lines semi-discretisation
 * du/dt = RHS(u) of the compressible Euler equations with the entropy-stable /
 * kinetic-energy-preserving flux-differencing LGL-DGSEM of Ranocha et al.,
 * "Efficient implementation of modern entropy stable and kinetic energy
 * preserving discontinuous Galerkin methods for conservation laws":
 *
 *   du_i/dt = -(1/J_i) [ sum_n sum_k D~_{i_n k} f_vol(u_i, u_k, (Ja^n_i + Ja^n_k)/2)
 *                        + sum_n (+-) f_surf(u_L, u_R, n_face) / w_end ]
 *
 * with D~ = 2D - M^-1 B the skew-symmetric flux-differencing operator
 * (Sec. 2.1, optimised flux-differencing form; Sec. 2.2, skew-symmetry),
 * directional two-point fluxes in the direction of the averaged contravariant
 * vectors (Sec. 2.3, rearranged curvilinear volume term) and the volume fluxes
 * of Shima et al. and Ranocha (Sec. 3.2) with the log means of Algorithms 2
 * and 3 (Sec. 3.1).  Meshes are periodic tensor-product boxes of hexahedra
 * (3D) or quadrilaterals (2D), affine or smoothly warped.
 *
 * Conventions shared by every entry point:
 *   - all floating-point values crossing the ABI are FP64, whatever the
 *     internal precision;
 *   - state layout (host or device): u[elem][var][node], variables
 *     (rho, rho v_1 .. rho v_d, rho e), node index x-fastest
 *     (i + N j + N^2 k, N = p+1), element index x-fastest
 *     (ex + nx ey + nx ny ez);
 *   - caller-owned pointers are never retained or freed by the library; host
 *     pointers are only read or written during the call; device pointers are
 *     read or written by work enqueued on the handle's stream, so the caller
 *     keeps them valid (and unmodified, for inputs) until that work is done,
 *     in stream order;
 *   - every call returns an esdg_status; ESDG_OK == 0; on failure a message
 *     is available from esdg_last_error();
 *   - a handle is not thread-safe; distinct handles on distinct streams may
 *     be used concurrently;
 *   - device work is enqueued on the handle's stream (a hipStream_t, NULL =
 *     the default stream); calls that return host data synchronise it.
 */
#ifndef ESDG_H
#define ESDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esdg_problem esdg_problem;

typedef enum {
  ESDG_OK = 0,
  ESDG_EINVAL = -1,        /* invalid argument or descriptor */
  ESDG_ENOMEM = -2,        /* device allocation failed */
  ESDG_EDEVICE = -3,       /* HIP runtime error (launch, copy, no device) */
  ESDG_ENONPHYSICAL = -4,  /* a kernel met rho <= 0, p <= 0 or a non-finite state */
  ESDG_ESTATE = -5         /* call needs a state: esdg_set_state was not called */
} esdg_status;

/* two-point fluxes (Sec. 3.2 and the local Lax-Friedrichs surface flux) */
typedef enum {
  ESDG_FLUX_RANOCHA = 0,  /* entropy conservative, KEP, PEP; log means of Algs. 2-3 */
  ESDG_FLUX_SHIMA = 1,    /* kinetic-energy and pressure-equilibrium preserving */
  ESDG_FLUX_LLF = 2,      /* surface only: central flux minus lam/2 [u],
                             lam = max(|v-.n|,|v+.n|) + max(c-,c+)|n| */
  ESDG_FLUX_CENTRAL = 3   /* (f(u-)+f(u+)).n/2; reduces to the strong form */
} esdg_flux;

typedef enum { ESDG_FP64 = 0, ESDG_FP32 = 1 } esdg_precision;
typedef enum { ESDG_HOST = 0, ESDG_DEVICE = 1 } esdg_where;

typedef struct {
  int32_t dim;              /* 2 or 3 */
  int32_t p;                /* polynomial degree, 1 <= p <= ESDG_PMAX */
  int32_t n[3];             /* elements per direction (n[2] ignored in 2D) */
  double lo[3], hi[3];      /* periodic box */
  double warp;              /* 0: affine; else x_m = xh_m + warp*prod_j sin(pi s_j),
                               s_j = 2(xh_j-lo_j)/(hi_j-lo_j) - 1 */
  const double *coords;     /* optional host node coordinates [elem][dim][node]
                               of a periodic conforming mesh with the box's
                               connectivity; overrides warp; NULL = none */
  double gamma;             /* ratio of specific heats, > 1 */
  int32_t volume_flux;      /* esdg_flux: RANOCHA, SHIMA or CENTRAL */
  int32_t surface_flux;     /* esdg_flux: any */
  int32_t precision;        /* esdg_precision of the internal state and fluxes */
  void *stream;             /* hipStream_t for all device work; NULL = default */
  int32_t nodes;            /* esdg_nodes: LGL (flux-differencing DGSEM, Sec. 2) or
                               GAUSS (Legendre-Gauss collocation with entropy
                               projection, Sec. 6; affine meshes only: warp = 0,
                               coords = NULL) */
  int32_t pad;
} esdg_mesh_desc;

/* Nodes of the element: Legendre-Gauss-Lobatto (the volume nodes include the
 * element boundary) or Legendre-Gauss collocation in the hybridised form of
 * Sec. 6: du/dt = -[M^-1 [I; R]^T f_h + M^-1 R^T B f*] with
 * f_h = sum_n 2 Q_h,n o F(u~, u~) over the volume nodes and the face points,
 * Q_h the hybridised SBP operator and u~ = [u; u(R w(u))] the entropy
 * projection (face states from the interpolated entropy variables).  The state
 * layout is the same; node coordinates are the Gauss points. */
typedef enum { ESDG_NODES_LGL = 0, ESDG_NODES_GAUSS = 1 } esdg_nodes;

#define ESDG_PMAX 7

/* Build the operators (LGL nodes, weights, D, D~), node coordinates, metric
 * terms (2D cross-product form, 3D conservative curl form; Sec. 2.3), one
 * normal per face and the device buffers of a problem.  Not part of the
 * timed right-hand side.  *out receives a handle owned by the caller
 * (release with esdg_destroy). */
esdg_status esdg_init_mesh(const esdg_mesh_desc *desc, esdg_problem **out);

/* Release the handle and every device buffer it owns.  NULL-safe. */
void esdg_destroy(esdg_problem *prob);

/* Sizes: elements, nodes per element ((p+1)^dim), conserved variables (dim+2). */
esdg_status esdg_sizes(const esdg_problem *prob, int64_t *n_elem, int32_t *nodes_per_elem,
                       int32_t *n_var);

/* Replace the stream used for all later device work (hipStream_t; NULL = default). */
esdg_status esdg_set_stream(esdg_problem *prob, void *stream);

/* Node coordinates [elem][dim][node] into a host buffer (FP64). */
esdg_status esdg_get_coords(const esdg_problem *prob, double *x);

/* 1/J per node, [elem][node] (node x-fastest), into a caller-owned host
 * buffer of n_elem * nodes_per_elem doubles, J = det(dx/dxi) from the
 * collocation derivatives of the node coordinates (Sec. 2.3, metric terms).
 * Curved meshes: the values the kernels scale the right-hand side with (in
 * FP32 mode the FP32 values they read, widened).  Affine meshes: the box's
 * exact constant 1/J = prod_n 2/h_n in FP64 (the kernels apply it as the
 * per-direction factors 2/h_n of the contravariant vectors and never read
 * 1/J itself).  For host quadratures sum_i J_i W_i f_i (W the LGL weights
 * of esdg_operators, tensor products per element).  Synchronous (a strided
 * device-to-host copy on the problem's stream); ESDG_EINVAL for a NULL
 * argument, ESDG_EDEVICE if the copy fails, ESDG_ENOMEM if host memory for
 * the FP32 staging runs out. */
esdg_status esdg_get_inv_jacobian(esdg_problem *prob, double *inv_j);

/* Set / read the conserved state u[elem][var][node]: the nodal values of
 * the conserved variables (rho, rho v, rho e) of the compressible Euler
 * equations (Sec. 3) that the semi-discretisation du/dt = RHS(u) of Sec. 2
 * advances.  FP64, host or device memory as `where` says (device pointers
 * on the handle's device); in FP32 mode set rounds to FP32 on the device and
 * get widens.  Host calls synchronise the stream.  ESDG_EINVAL for a NULL
 * pointer; esdg_get_state before any esdg_set_state gives ESDG_ESTATE. */
esdg_status esdg_set_state(esdg_problem *prob, const double *u, int32_t where);
esdg_status esdg_get_state(esdg_problem *prob, double *u, int32_t where);

/* rhs!: du = RHS(current state) (Sec. 2.1 optimised flux-differencing form).
 * du has the state layout, FP64, host or device memory. */
esdg_status esdg_rhs(esdg_problem *prob, double *du, int32_t where);

/* step!: advance the state by nsteps steps of an explicit Runge-Kutta
 * method, the time integration of the semi-discretisation (Sec. 4.1: the
 * paper's runs use explicit low-storage Runge-Kutta schemes): the problem's
 * integrator (esdg_set_integrator), classical RK4 (Butcher a = 1/2, 1/2, 1;
 * b = 1/6, 1/3, 1/3, 1/6) in low-storage form (state, accumulator and two
 * alternating stage buffers), or the five-stage 2N-storage scheme; each
 * stage one fused launch (surface flux + volume term + lifting + stage
 * update).  dt > 0: fixed step; dt <= 0: the CFL step of esdg_max_dt,
 * recomputed at the start of every step on the device.  The problem's time
 * (device, FP64) advances by each step's dt.  t_inout (may be NULL): on
 * entry the time to start from, on return the time reached (this
 * synchronises the stream).  ESDG_ENONPHYSICAL, with nothing enqueued, if an
 * earlier kernel met a non-physical state (the flag is cleared by reporting
 * it); with t_inout also if this call's own kernels met one.  ESDG_EINVAL for
 * nsteps < 0 or dt <= 0 with cfl <= 0; ESDG_ESTATE before esdg_set_state. */
esdg_status esdg_step(esdg_problem *prob, double dt, int32_t nsteps, double cfl,
                      double *t_inout);

/* Time integrators of esdg_step (and of a batch's members). */
typedef enum {
  ESDG_RK4 = 0,  /* classical four-stage RK4 (default) */
  ESDG_CK45 = 1  /* five-stage, fourth-order 2N-storage RK of Carpenter and Kennedy,
                    du <- A_i du + dt RHS(u), u <- u + B_i du (the scheme of the
                    paper's FLUXO runs, Sec. 4.1); R holds du */
} esdg_integrator;

/* Select / read the integrator of later esdg_step calls (ESDG_EINVAL for an
 * unknown one).  A batch records its members' integrators when created. */
esdg_status esdg_set_integrator(esdg_problem *prob, int32_t integrator);
esdg_status esdg_get_integrator(const esdg_problem *prob, int32_t *integrator);

/* The problem's time (0 after esdg_init_mesh); esdg_get_time synchronises. */
esdg_status esdg_set_time(esdg_problem *prob, double t);
esdg_status esdg_get_time(esdg_problem *prob, double *t);

/* The reductions below synchronise the stream, write their result and then
 * return ESDG_ENONPHYSICAL if any kernel so far met a non-physical state
 * (rho <= 0, p <= 0 or non-finite; the flag is cleared by reporting it).
 * ESDG_EINVAL for a NULL output, ESDG_ESTATE before esdg_set_state. */

/* entropy_rate: dS/dt = sum_i J_i W_i w(u_i) . RHS_i with the entropy
 * U = -rho s/(gamma-1), s = ln p - gamma ln rho (Sec. 2 entropy definitions);
 * FP64 fixed-order reduction on the device.  Zero to round-off for the
 * Ranocha flux in volume and surface on periodic meshes. */
esdg_status esdg_entropy_rate(esdg_problem *prob, double *dSdt);

/* totals[v] = sum_i J_i W_i u_{i,v}, the discrete integrals of the conserved
 * variables that the semi-discretisation keeps constant on periodic meshes
 * (Sec. 2, conservation); FP64, fixed order; dim+2 entries. */
esdg_status esdg_totals(esdg_problem *prob, double *totals);

/* Allocation-free variant of esdg_totals, for callers that cannot allocate
 * device memory or wait for the device: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The same sums, bit for
 * bit (same kernels and block partition), written as dim+2 doubles to
 * `totals_dev`, a caller-owned DEVICE pointer, in stream order on the
 * handle's stream; the call returns without waiting for them.  Allocates
 * nothing: the block partial sums go to a library-owned static device array
 * of 16,384 doubles (128 KiB per GPU, held until the process ends), which
 * every call on that GPU shares, so calls that overlap on one GPU (other
 * handles, other streams or threads) race and must be serialised by the
 * caller.  A problem needs red_blocks x (dim+2) <= 16,384 partials, which
 * every valid problem meets (at most 2,048 blocks); larger needs return
 * ESDG_EINVAL.  ESDG_ESTATE before set_state; ESDG_ENONPHYSICAL if a
 * kernel has flagged a non-physical state (the flag is read from
 * host-mapped memory, without a wait). */
esdg_status esdg_totals_noalloc(esdg_problem *prob, double *totals_dev);

/* CFL step size of the current state, the same formula esdg_step uses:
 * dt = cfl*2/((p+1) max_i sum_n (|v_i.Ja^n_i| + c_i |Ja^n_i|)/J_i), c the
 * speed of sound.  The paper's runs control the step size by a CFL
 * condition (Sec. 4.1) without stating the formula; this is the library's
 * reading of it.  FP64 maximum on the device; ESDG_EINVAL for cfl <= 0. */
esdg_status esdg_max_dt(esdg_problem *prob, double cfl, double *dt);

/* Wait for the handle's stream and report deferred device errors
 * (ESDG_ENONPHYSICAL if any kernel saw a non-physical state; the flag is
 * cleared by reporting it).  The flag lives in host-mapped memory, so
 * esdg_step can report it without waiting. */
esdg_status esdg_sync(esdg_problem *prob);

/* Per-kernel timing with hipEvents on the handle's stream: while enabled,
 * every launch of the listed kernels is bracketed by an event pair.
 * esdg_timing_read returns the summed duration (ms) and launch count since
 * the last reset, synchronising the stream.  STAGE is the fused
 * right-hand-side / RK-stage kernel, REDUCE the FP64 reductions, PROJECT the
 * entropy projection of Gauss problems, FACE the face kernel of the
 * once-per-face mode (esdg_set_face_flux_mode). */
typedef enum {
  ESDG_KERNEL_STAGE = 1,
  ESDG_KERNEL_REDUCE = 2,
  ESDG_KERNEL_PROJECT = 3,
  ESDG_KERNEL_FACE = 4
} esdg_kernel;
esdg_status esdg_timing_enable(esdg_problem *prob, int32_t enable);
esdg_status esdg_timing_read(esdg_problem *prob, int32_t kernel, double *total_ms,
                             int64_t *launches);
esdg_status esdg_timing_reset(esdg_problem *prob);

/* Tile variants of the fused stage kernel (workgroup shapes: elements per
 * workgroup and lanes per direction).  Variants 0-2 give one lane to each
 * line of an element (one wave per direction; the fewest elements filling
 * whole waves; twice the default); variant 3 gives one lane to each node,
 * which sweeps its partners along every direction (each pair evaluated from
 * both ends, fewer registers per lane); variant 4 (3D) gives one lane to
 * each node and has the lanes of a line evaluate each pair once, handing
 * the flux to the partner lane (one wave per z-plane of the element at
 * p = 7, and at p = 6 for FP64 curved meshes; lines of one direction packed
 * into waves otherwise).  Variants 0-3 compute bit-identical
 * results; variant 4 adds each node's terms in another order (the same
 * values up to rounding).  The variant in use is chosen per (dim, p, volume
 * flux, mesh kind, precision, node kind) in a process-wide table; until
 * changed, for 3D LGL problems: variant 0 up to p = 3, variant 3 at p = 4,
 * at p = 5 variant 4 except on curved FP32 meshes (3), variant 4 at p = 6
 * and 7.  2D and Gauss
 * problems have variant 0 only.
 *   esdg_autotune: times every variant on the problem's current state (reps
 *     right-hand-side launches each, written to internal scratch; the state
 *     is unchanged), stores the fastest in the table and returns it in *best
 *     and the time per launch of each variant in us_per_variant
 *     [ESDG_TILE_VARIANTS] (either may be NULL; -1 for a missing variant).
 *     Synchronises the stream.
 *   esdg_set_tile_variant: store a variant for the problem's parameters.
 *   esdg_get_tile_variant: the variant in use and its elements per workgroup. */
#define ESDG_TILE_VARIANTS 5
esdg_status esdg_autotune(esdg_problem *prob, int32_t reps, int32_t *best, double *us_per_variant);
esdg_status esdg_set_tile_variant(esdg_problem *prob, int32_t variant);
esdg_status esdg_get_tile_variant(const esdg_problem *prob, int32_t *variant, int32_t *elems_per_block);

/* Where the surface fluxes are evaluated (Sec. 2.4 names evaluating them
 * once per face and handing them to both elements as the usual efficient
 * organisation on CPUs).
 *   ESDG_FACES_FUSED (default): the stage kernel evaluates f* at every face
 *     node of each element it updates, so every face is evaluated by both of
 *     its elements, from the same inputs in the same order (the left
 *     element's trace, the right one's, the left element's + face normal).
 *   ESDG_FACES_ONCE: before every stage launch a face kernel evaluates f* once
 *     per face node, for the + face of every element in every direction, into
 *     a device buffer of E dim nv nf reals of the problem's precision (E nf
 *     faces per direction), and the stage kernel reads it.  Bitwise the same
 *     results as the fused mode; on MI355X slower at every measured size (the
 *     face pass moves more data than the flux arithmetic it saves).
 * 3D LGL problems only, with a stage kernel built for it: tile variants 3
 * and 4, and the line tiles (0-2) up to p = 4 (in the line tiles above and
 * in 2D the extra branch costs registers).  ESDG_EINVAL for an unknown mode,
 * a 2D or Legendre-Gauss problem (which evaluates face fluxes per element),
 * a tile variant in use without that build; in ONCE mode
 * esdg_set_tile_variant refuses such a variant, esdg_autotune skips it, and
 * a step finding one in the process-wide table fails.  Switching to ONCE
 * allocates the buffer (ESDG_ENOMEM if that fails); switching back
 * synchronises the handle's stream and frees it.  Batches evaluate faces
 * fused: esdg_batch_create rejects a member in ONCE mode (ESDG_EINVAL). */
#define ESDG_FACES_FUSED 0
#define ESDG_FACES_ONCE 1
esdg_status esdg_set_face_flux_mode(esdg_problem *prob, int32_t mode);
esdg_status esdg_get_face_flux_mode(const esdg_problem *prob, int32_t *mode);

/* Device memory (bytes) esdg_init_mesh would allocate for the descriptor:
 * five state-sized arrays (state, two stage states, accumulator, RHS), an
 * FP64 staging array in FP32 mode, metrics and face normals on curved
 * meshes, and small scalars.  No device call. */
esdg_status esdg_footprint(const esdg_mesh_desc *desc, int64_t *bytes);

/* ---- batches: several problems advanced together ------------------------
 * A batch groups problems by (dim, p, volume and surface flux, mesh kind,
 * precision, node kind, gamma); each RK stage is one launch per group (two
 * for Gauss groups: projection, then stage) over the
 * element tiles of all its problems.  Every problem computes exactly what it
 * computes alone (same kernels, same per-element arithmetic): states, times
 * and CFL steps are bit-identical to esdg_step on the problem by itself.
 * The batch references the problems (it does not own them): they must stay
 * alive, on one device, and keep their state set while the batch exists.
 *   t_end: optional per-problem end times (NULL: none); a step of problem i
 *     never passes t_end[i] (dt = min(dt, t_end[i] - t)), so a problem that
 *     has reached its end time takes steps of dt = 0 (no change).
 *   stream: hipStream_t of the batch's work; NULL: the batch creates a
 *     non-blocking stream of its own.  Work already enqueued on a member's
 *     stream is ordered before the batch's work, and the batch's work before
 *     later work on the members' streams.
 *   flags: ESDG_BATCH_GRAPHS replays each step as a captured HIP graph;
 *     ESDG_BATCH_CONCURRENT lets the groups of a stage run on concurrent
 *     streams. */
typedef struct esdg_batch esdg_batch;
#define ESDG_BATCH_GRAPHS 1
#define ESDG_BATCH_CONCURRENT 2
esdg_status esdg_batch_create(esdg_problem *const *probs, int32_t count, const double *t_end, void *stream,
                              int32_t flags, esdg_batch **out);
void esdg_batch_destroy(esdg_batch *batch);

/* nsteps steps of every member as in esdg_step (dt > 0 fixed, else CFL
 * with each member's own dt).  ESDG_ENONPHYSICAL, with nothing enqueued,
 * while a member's non-physical flag is raised (esdg_batch_sync names the
 * member and clears its flag). */
esdg_status esdg_batch_step(esdg_batch *batch, double dt, int32_t nsteps, double cfl);

/* Right-hand side of every member's state; du[i] (FP64, state layout, host or
 * device as `where` says) receives member i's; du or du[i] may be NULL (the
 * result then stays in the member's internal buffer). */
esdg_status esdg_batch_rhs(esdg_batch *batch, double *const *du, int32_t where);

/* Current time of every member into t[count] (host); synchronises. */
esdg_status esdg_batch_times(esdg_batch *batch, double *t);

/* Wait for the batch's work; ESDG_ENONPHYSICAL with *bad (may be NULL) the
 * first member whose kernels met a non-physical state (its flag is cleared,
 * so a further call reports the next one), else *bad = -1. */
esdg_status esdg_batch_sync(esdg_batch *batch, int32_t *bad);

/* Tune the tile variant of every 3D LGL group on its own launch: each variant
 * is timed over reps right-hand-side launches of all the group's tiles (after
 * one untimed launch; written to the members' internal RHS buffers, states
 * unchanged) and the fastest is stored in the process-wide table for the
 * group's parameters, as esdg_set_tile_variant does.  Synchronises the batch's
 * and the members' streams; ESDG_EINVAL for reps < 1, ESDG_ESTATE if a member
 * has no state. */
esdg_status esdg_batch_autotune(esdg_batch *batch, int32_t reps);

/* Groups (launches per stage) and total element tiles of the batch. */
esdg_status esdg_batch_info(esdg_batch *batch, int32_t *groups, int64_t *tiles);

/* Whole-step timing: while enabled every esdg_batch_step step is bracketed by
 * an event pair on the batch stream; read returns the summed ms and the
 * number of steps since the last read, and resets. */
esdg_status esdg_batch_timing_enable(esdg_batch *batch, int32_t enable);
esdg_status esdg_batch_timing_read(esdg_batch *batch, double *total_ms, int64_t *steps);

const char *esdg_batch_last_error(const esdg_batch *batch);

/* ---- serving: a continuous-batching loop over time-integration jobs -----
 * Jobs (a mesh, an initial state, a start and an end time) are queued by
 * esdg_server_submit and admitted in arrival order while the device memory
 * of the admitted and unfetched jobs (esdg_footprint) stays within
 * hbm_budget and at most max_active jobs are being stepped.  Each
 * esdg_server_tick enqueues steps_per_tick CFL steps of every admitted job as
 * one batch (a job that reaches t_end stops there), admits what fits while
 * the device works (geometry and state upload of new jobs), then retires
 * the jobs that have reached their end time.  A retired job's final state
 * stays on the device until esdg_server_fetch.  Each job's result is
 * bit-identical to the same job served alone.  Host-side calls on one
 * server are not thread-safe. */
typedef struct esdg_server esdg_server;
typedef struct {
  int64_t hbm_budget;      /* bytes for admitted jobs; 0: 90% of the free device memory */
  int32_t max_active;      /* admitted jobs at most; 0: no limit */
  int32_t steps_per_tick;  /* RK steps per tick, >= 1 */
  int32_t flags;           /* ESDG_BATCH_* for the batch of admitted jobs */
  int32_t pad;
  double cfl;              /* CFL number of every job's steps, > 0 */
} esdg_server_config;

typedef struct {
  esdg_mesh_desc mesh;  /* the stream field is ignored */
  const double *u0;     /* initial state (host, FP64, state layout); copied by submit */
  double t0, t_end;     /* start and end time, t_end > t0 */
} esdg_job_desc;

typedef enum {
  ESDG_JOB_QUEUED = 0,
  ESDG_JOB_ACTIVE = 1,
  ESDG_JOB_DONE = 2,     /* reached t_end; state ready for esdg_server_fetch */
  ESDG_JOB_FAILED = 3    /* non-physical state or device error; see esdg_server_last_error */
} esdg_job_status;

esdg_status esdg_server_create(const esdg_server_config *cfg, esdg_server **out);
void esdg_server_destroy(esdg_server *server);
/* Queue a job; ESDG_EINVAL if its footprint exceeds the whole budget. */
esdg_status esdg_server_submit(esdg_server *server, const esdg_job_desc *job, int64_t *job_id);
/* One tick (see above); the counts after it (any may be NULL). */
esdg_status esdg_server_tick(esdg_server *server, int32_t *finished, int32_t *active, int32_t *queued);
/* Status, current time and RK steps taken (including dt = 0 steps after
 * t_end within the last tick) of a job (any output may be NULL). */
esdg_status esdg_server_job(esdg_server *server, int64_t job_id, int32_t *status, double *t, int64_t *steps);
/* Jobs that finished (DONE or FAILED) in the last tick: up to max ids, *n of them. */
esdg_status esdg_server_finished(esdg_server *server, int64_t *ids, int32_t max, int32_t *n);
/* Copy a DONE job's final state to u (host, FP64; may be NULL) and release
 * the job (also releases a FAILED job). */
esdg_status esdg_server_fetch(esdg_server *server, int64_t job_id, double *u);
/* Device memory held by admitted and finished-but-unfetched jobs. */
esdg_status esdg_server_memory(esdg_server *server, int64_t *used, int64_t *budget);
const char *esdg_server_last_error(const esdg_server *server);
/* The server's admission rule as a pure host function (no device access):
 * of n_queued jobs in arrival order with device footprints queued_bytes,
 * how many are admitted now, given used bytes of admitted and unfetched
 * jobs, the budget, the number of active jobs and the cap max_active
 * (0: none).  Admission keeps arrival order: it stops at the first job that
 * does not fit.  ESDG_EINVAL on negative sizes or a NULL output. */
esdg_status esdg_server_plan(const int64_t *queued_bytes, int32_t n_queued, int64_t used, int64_t budget,
                             int32_t active, int32_t max_active, int32_t *n_admit);

/* Last error message of the handle (or of the calling thread if prob is NULL). */
const char *esdg_last_error(const esdg_problem *prob);

/* The 1D operators the library uses for degree p (host computation, no device
 * needed): LGL nodes x[p+1] and weights w[p+1] (Sec. 2, LGL-DGSEM example),
 * the derivative matrix D and the flux-differencing operator
 * D~ = 2D - M^-1 B (Sec. 2.1), both (p+1)x(p+1) row-major.  Any output
 * pointer may be NULL.  ESDG_EINVAL if p is out of [1, ESDG_PMAX]. */
esdg_status esdg_operators(int32_t p, double *x, double *w, double *D, double *Dt);

/* Library version string. */
const char *esdg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ESDG_H */
