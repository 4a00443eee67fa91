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
 *   - caller-owned pointers are only read or written during the call and are
 *     never retained or freed by the library;
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
} esdg_mesh_desc;

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

/* Set / read the conserved state u[elem][var][node] (FP64, host or device
 * memory as `where` says; device pointers must be on the handle's device). */
esdg_status esdg_set_state(esdg_problem *prob, const double *u, int32_t where);
esdg_status esdg_get_state(esdg_problem *prob, double *u, int32_t where);

/* rhs!: du = RHS(current state) (Sec. 2.1 optimised flux-differencing form).
 * du has the state layout, FP64, host or device memory. */
esdg_status esdg_rhs(esdg_problem *prob, double *du, int32_t where);

/* step!: advance the state by nsteps steps of classical RK4 (Butcher
 * a = 1/2, 1/2, 1; b = 1/6, 1/3, 1/3, 1/6) in low-storage form (state,
 * accumulator and two alternating stage buffers), each stage one fused
 * launch (surface flux + volume term + lifting + stage update).  dt > 0: fixed step; dt <= 0:
 * dt = cfl*2/((p+1) max_i sum_n (|v.Ja^n|+c|Ja^n|)/J_i) recomputed at the start
 * of every step on the device.  *t_inout (may be NULL) is advanced by the
 * total time; in CFL mode this synchronises the stream. */
esdg_status esdg_step(esdg_problem *prob, double dt, int32_t nsteps, double cfl,
                      double *t_inout);

/* entropy_rate: dS/dt = sum_i J_i W_i w(u_i) . RHS_i with the entropy
 * U = -rho s/(gamma-1), s = ln p - gamma ln rho (Sec. 2 entropy definitions);
 * FP64 fixed-order reduction on the device.  Zero to round-off for the
 * Ranocha flux in volume and surface on periodic meshes. */
esdg_status esdg_entropy_rate(esdg_problem *prob, double *dSdt);

/* totals[v] = sum_i J_i W_i u_{i,v} (FP64, fixed order); totals has dim+2 entries. */
esdg_status esdg_totals(esdg_problem *prob, double *totals);

/* CFL step size of the current state (same formula as esdg_step). */
esdg_status esdg_max_dt(esdg_problem *prob, double cfl, double *dt);

/* Wait for the handle's stream and report deferred device errors
 * (ESDG_ENONPHYSICAL if any kernel saw a non-physical state; the flag is
 * cleared by reporting it). */
esdg_status esdg_sync(esdg_problem *prob);

/* Per-kernel timing with hipEvents on the handle's stream: while enabled,
 * every launch of the listed kernels is bracketed by an event pair.
 * esdg_timing_read returns the summed duration (ms) and launch count since
 * the last reset, synchronising the stream.  STAGE is the fused
 * right-hand-side / RK-stage kernel, REDUCE the FP64 reductions. */
typedef enum { ESDG_KERNEL_STAGE = 1, ESDG_KERNEL_REDUCE = 2 } esdg_kernel;
esdg_status esdg_timing_enable(esdg_problem *prob, int32_t enable);
esdg_status esdg_timing_read(esdg_problem *prob, int32_t kernel, double *total_ms,
                             int64_t *launches);
esdg_status esdg_timing_reset(esdg_problem *prob);

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
