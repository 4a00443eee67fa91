/*
 * esdg_oracle.c -- plain, slow, obviously-correct CPU oracle for the
 * flux-differencing LGL-DGSEM semi-discretisation of the compressible Euler
 * equations (Ranocha et al., "Efficient implementation of modern entropy
 * stable and kinetic energy preserving discontinuous Galerkin methods for
 * conservation laws").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file: only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the HIP library.
 *
 * Everything is FP64 and written as the paper's definitions, without the
 * optimisations the paper proposes:
 *   - the volume term is the flux-differencing sum with 2*D over ALL k
 *     (Sec. 2, flux-differencing form of the strong DG scheme), not the
 *     skew-symmetric D~ form of Sec. 2.1, and no i<k halving (Sec. 2.2);
 *   - the surface term is M^-1 R^T B (f_num - sum_j N_j R f^j) (same form),
 *     evaluated per element side, not once per face;
 *   - two-point fluxes take conservative variables and recompute primitive
 *     variables on every call (no precomputed primitives or logarithms,
 *     Sec. 7.1/7.2);
 *   - time stepping is the textbook classical RK4 with k-vectors.
 * OpenMP is used only across elements, which does not change any result.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   R1  D from the closed-form Legendre expression with the textbook diagonal
 *       D_00 = -p(p+1)/4, D_pp = p(p+1)/4, D_ii = 0 otherwise.
 *   R2  entropy U = -rho*s/(gamma-1), s = ln p - gamma ln rho.
 *   R3  log-mean cutoff: series iff u < 1e-4 (strict).
 *   R7  LLF: 0.5(f(u-)+f(u+)).n - 0.5*lam*(u+ - u-),
 *       lam = max(|v-.n|,|v+.n|) + max(c-,c+)*|n|.
 *   R8  curvilinear surface term uses the contravariant (non-unit) normal Ja^n.
 *   R9  one normal per face: the average of the two sides' Ja^n.
 *   R10 3D metrics in the conservative curl form; J = det(dx/dxi) from
 *       collocation derivatives.
 *   R14 warp: x_m = xhat_m + warp*prod_j sin(pi*s_j), s_j in [-1,1] the
 *       global box coordinate.
 *   R17 CFL: dt = cfl*2/((p+1)*max_i sum_n (|v.Ja^n| + c|Ja^n|)/J_i).
 *
 * Legendre-Gauss collocation (Sec. 6, hybridised form with the entropy
 * projection) is evaluated on affine meshes by assembling, for every line of
 * an element, the dense hybridised operator of the paper's formulation over
 * the line's volume nodes and its two face points and summing
 * 2 Q_h f(u~_a, u~_b) over all pairs of that combined set, with the face
 * states u~ = u(R w(u)) of the element and of its neighbour.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXN 16 /* at most degree 15 */

enum { ORC_RANOCHA = 0, ORC_SHIMA = 1, ORC_LLF = 2, ORC_CENTRAL = 3 };

typedef struct {
  int32_t dim, p, n[3];
  double lo[3], hi[3];
  double warp, gamma;
  int32_t vol_flux, surf_flux;
  int32_t nodes; /* 0: Legendre-Gauss-Lobatto, 1: Legendre-Gauss (affine only) */
} orc_desc;

typedef struct {
  orc_desc d;
  int N;        /* nodes per line */
  int nn;       /* nodes per element */
  int64_t ne;   /* elements */
  int nv;       /* conserved variables */
  double xi[ORC_MAXN], w[ORC_MAXN], D[ORC_MAXN * ORC_MAXN];
  double rL[ORC_MAXN], rR[ORC_MAXN]; /* Gauss: Lagrange basis at -1 and +1 */
  double *x;    /* [ne][dim][nn] physical node coordinates */
  double *Ja;   /* [ne][3][3][nn]: Ja[e][n][m][i] = (Ja)^n_m at node i */
  double *J;    /* [ne][nn] */
} orc_mesh;

/* threads the element loops use (OpenMP) */
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* ------------------------------------------------------------------------ */
/* 1D LGL operators (Sec. 2, LGL-DGSEM example; textbook closed forms)      */
/* ------------------------------------------------------------------------ */

/* Legendre P_p and its first two derivatives at x, by the three-term
 * recurrence, in long double. */
static void legendre(int p, long double x, long double *P, long double *dP,
                     long double *d2P) {
  long double p0 = 1.0L, p1 = x, dp0 = 0.0L, dp1 = 1.0L, d2p0 = 0.0L,
              d2p1 = 0.0L;
  if (p == 0) {
    *P = 1.0L; *dP = 0.0L; *d2P = 0.0L;
    return;
  }
  for (int k = 2; k <= p; ++k) {
    long double pk = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    long double dpk = dp0 + (2 * k - 1) * p1;           /* P'_k = P'_{k-2} + (2k-1)P_{k-1} */
    long double d2pk = d2p0 + (2 * k - 1) * dp1;
    p0 = p1; p1 = pk; dp0 = dp1; dp1 = dpk; d2p0 = d2p1; d2p1 = d2pk;
  }
  *P = p1; *dP = dp1; *d2P = d2p1;
}

/* LGL nodes xi (ascending), weights w and the nodal derivative matrix D
 * (row-major D[i*N+j]) for degree p.  Interior nodes are the roots of P'_p,
 * found by Newton's method from Chebyshev-Gauss-Lobatto guesses. */
int orc_lgl(int p, double *xi, double *w, double *D) {
  if (p < 1 || p >= ORC_MAXN) return -1;
  int N = p + 1;
  long double x[ORC_MAXN], Pp[ORC_MAXN];
  x[0] = -1.0L; x[p] = 1.0L;
  for (int i = 1; i < p; ++i) {
    long double t = -cosl(3.14159265358979323846264338327950288L * i / p);
    for (int it = 0; it < 100; ++it) {
      long double P, dP, d2P;
      legendre(p, t, &P, &dP, &d2P);
      long double dt = dP / d2P;
      t -= dt;
      if (fabsl(dt) < 1e-19L) break;
    }
    x[i] = t;
  }
  /* symmetrise exactly: x_{p-i} = -x_i */
  for (int i = 0; i < N / 2; ++i) {
    long double s = 0.5L * (x[p - i] - x[i]);
    x[i] = -s; x[p - i] = s;
  }
  if (N % 2 == 1) x[p / 2] = 0.0L;
  for (int i = 0; i < N; ++i) {
    long double P, dP, d2P;
    legendre(p, x[i], &P, &dP, &d2P);
    Pp[i] = P;
    xi[i] = (double)x[i];
    w[i] = (double)(2.0L / ((long double)p * (p + 1) * P * P));
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      long double v;
      if (i != j) v = Pp[i] / (Pp[j] * (x[i] - x[j]));
      else if (i == 0) v = -(long double)p * (p + 1) / 4.0L;
      else if (i == p) v = (long double)p * (p + 1) / 4.0L;
      else v = 0.0L;
      D[i * N + j] = (double)v;
    }
  return 0;
}

/* Legendre-Gauss nodes xi (roots of P_N, N = p+1, ascending), weights
 * 2/((1-x^2) P_N'(x)^2), the textbook collocation derivative matrix
 * D_ij = P_N'(x_i) / (P_N'(x_j) (x_i - x_j)), D_ii = x_i / (1 - x_i^2), and
 * the values rL, rR of the Lagrange basis at -1 and +1 (Sec. 6 operators
 * R: volume nodes -> face points). */
int orc_gauss(int p, double *xi, double *w, double *D, double *rL, double *rR) {
  if (p < 0 || p + 1 >= ORC_MAXN) return -1;
  const int N = p + 1;
  long double x[ORC_MAXN], dP[ORC_MAXN];
  for (int i = 0; i < N; ++i) {
    long double t = -cosl(3.14159265358979323846264338327950288L * (i + 0.5L) / N);
    for (int it = 0; it < 100; ++it) {
      long double P, d1, d2;
      legendre(N, t, &P, &d1, &d2);
      long double dt = P / d1;
      t -= dt;
      if (fabsl(dt) < 1e-19L) break;
    }
    x[i] = t;
  }
  for (int i = 0; i < N / 2; ++i) {
    long double s = 0.5L * (x[N - 1 - i] - x[i]);
    x[i] = -s; x[N - 1 - i] = s;
  }
  if (N % 2 == 1) x[N / 2] = 0.0L;
  for (int i = 0; i < N; ++i) {
    long double P, d1, d2;
    legendre(N, x[i], &P, &d1, &d2);
    dP[i] = d1;
    xi[i] = (double)x[i];
    w[i] = (double)(2.0L / ((1.0L - x[i] * x[i]) * d1 * d1));
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      long double v = (i != j) ? dP[i] / (dP[j] * (x[i] - x[j])) : x[i] / (1.0L - x[i] * x[i]);
      D[i * N + j] = (double)v;
    }
  for (int k = 0; k < N; ++k) {
    long double a = 1.0L, b = 1.0L;
    for (int j = 0; j < N; ++j) {
      if (j == k) continue;
      a *= (-1.0L - x[j]) / (x[k] - x[j]);
      b *= (1.0L - x[j]) / (x[k] - x[j]);
    }
    rL[k] = (double)a;
    rR[k] = (double)b;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Logarithmic means (Sec. 3.1, Algorithms 2 and 3)                         */
/* ------------------------------------------------------------------------ */

double orc_logmean(double am, double ap) {
  double u = (am * (am - 2.0 * ap) + ap * ap) / (am * (am + 2.0 * ap) + ap * ap);
  double eps = 1.0e-4;
  if (u < eps)
    return (am + ap) / (2.0 + u * (2.0 / 3.0 + u * (2.0 / 5.0 + u * (2.0 / 7.0))));
  return (ap - am) / log(ap / am);
}

double orc_inv_logmean(double am, double ap) {
  double u = (am * (am - 2.0 * ap) + ap * ap) / (am * (am + 2.0 * ap) + ap * ap);
  double eps = 1.0e-4;
  if (u < eps)
    return (2.0 + u * (2.0 / 3.0 + u * (2.0 / 5.0 + u * (2.0 / 7.0)))) / (am + ap);
  return log(ap / am) / (ap - am);
}

/* ------------------------------------------------------------------------ */
/* Compressible Euler (Sec. 3, ideal gas)                                   */
/* ------------------------------------------------------------------------ */

/* conservative u = (rho, rho v_1..rho v_d, rho e) -> rho, v[3], p */
static void primitives(int dim, double g, const double *u, double *rho,
                       double v[3], double *p) {
  double r = u[0];
  double kin = 0.0;
  v[0] = v[1] = v[2] = 0.0;
  for (int m = 0; m < dim; ++m) {
    v[m] = u[1 + m] / r;
    kin += u[1 + m] * v[m];
  }
  *rho = r;
  *p = (g - 1.0) * (u[dim + 1] - 0.5 * kin);
}

/* physical flux in direction n (not necessarily unit): sum_j n_j f^j(u) */
void orc_phys_flux(int dim, double g, const double *u, const double *n,
                   double *f) {
  double rho, v[3], p;
  primitives(dim, g, u, &rho, v, &p);
  double vn = 0.0;
  for (int m = 0; m < dim; ++m) vn += v[m] * n[m];
  f[0] = rho * vn;
  for (int m = 0; m < dim; ++m) f[1 + m] = rho * v[m] * vn + p * n[m];
  f[dim + 1] = (u[dim + 1] + p) * vn;
}

/* Directional two-point fluxes, arguments (u_-, u_+, n) in this order
 * (Sec. 3.2; Def. of numerical fluxes in Sec. 2). */
static void flux_shima(int dim, double g, const double *um, const double *up,
                       const double *n, double *f) {
  double rm, rp, vm[3], vp[3], pm, pp;
  primitives(dim, g, um, &rm, vm, &pm);
  primitives(dim, g, up, &rp, vp, &pp);
  double vnm = 0.0, vnp = 0.0, vv = 0.0;
  for (int m = 0; m < dim; ++m) {
    vnm += vm[m] * n[m];
    vnp += vp[m] * n[m];
    vv += vm[m] * vp[m];
  }
  double rho_avg = 0.5 * (rm + rp);
  double vn_avg = 0.5 * (vnm + vnp);
  double p_avg = 0.5 * (pm + pp);
  double frho = rho_avg * vn_avg;
  f[0] = frho;
  for (int m = 0; m < dim; ++m) f[1 + m] = frho * 0.5 * (vm[m] + vp[m]) + p_avg * n[m];
  /* ((v;v)) = (v+ . v- + v- . v+)/2 = v- . v+ ; ((p; v.n)) = (p+ vn- + p- vn+)/2 */
  f[dim + 1] = frho * vv / 2.0 + p_avg * vn_avg / (g - 1.0) +
               0.5 * (pp * vnm + pm * vnp);
}

static void flux_ranocha(int dim, double g, const double *um, const double *up,
                         const double *n, double *f) {
  double rm, rp, vm[3], vp[3], pm, pp;
  primitives(dim, g, um, &rm, vm, &pm);
  primitives(dim, g, up, &rp, vp, &pp);
  double vnm = 0.0, vnp = 0.0, vv = 0.0;
  for (int m = 0; m < dim; ++m) {
    vnm += vm[m] * n[m];
    vnp += vp[m] * n[m];
    vv += vm[m] * vp[m];
  }
  double rho_log = orc_logmean(rm, rp);
  double vn_avg = 0.5 * (vnm + vnp);
  double p_avg = 0.5 * (pm + pp);
  double frho = rho_log * vn_avg;
  /* 1/{{rho/p}}_log = p+ p- / {{rho- p+, rho+ p-}}_log  (Sec. 3.2) */
  double inv_rho_p_log = pp * pm * orc_inv_logmean(rm * pp, rp * pm);
  f[0] = frho;
  for (int m = 0; m < dim; ++m) f[1 + m] = frho * 0.5 * (vm[m] + vp[m]) + p_avg * n[m];
  f[dim + 1] = frho * vv / 2.0 + frho * inv_rho_p_log / (g - 1.0) +
               0.5 * (pp * vnm + pm * vnp);
}

static void flux_central(int dim, double g, const double *um, const double *up,
                         const double *n, double *f) {
  double fm[5], fp[5];
  orc_phys_flux(dim, g, um, n, fm);
  orc_phys_flux(dim, g, up, n, fp);
  for (int v = 0; v < dim + 2; ++v) f[v] = 0.5 * (fm[v] + fp[v]);
}

static void flux_llf(int dim, double g, const double *um, const double *up,
                     const double *n, double *f) {
  double rm, rp, vm[3], vp[3], pm, pp;
  primitives(dim, g, um, &rm, vm, &pm);
  primitives(dim, g, up, &rp, vp, &pp);
  double vnm = 0.0, vnp = 0.0, nn = 0.0;
  for (int m = 0; m < dim; ++m) {
    vnm += vm[m] * n[m];
    vnp += vp[m] * n[m];
    nn += n[m] * n[m];
  }
  double cm = sqrt(g * pm / rm), cp = sqrt(g * pp / rp);
  double lam = fmax(fabs(vnm), fabs(vnp)) + fmax(cm, cp) * sqrt(nn);
  double fc[5];
  flux_central(dim, g, um, up, n, fc);
  for (int v = 0; v < dim + 2; ++v) f[v] = fc[v] - 0.5 * lam * (up[v] - um[v]);
}

void orc_two_point(int kind, int dim, double g, const double *um,
                   const double *up, const double *n, double *f) {
  switch (kind) {
    case ORC_RANOCHA: flux_ranocha(dim, g, um, up, n, f); break;
    case ORC_SHIMA: flux_shima(dim, g, um, up, n, f); break;
    case ORC_LLF: flux_llf(dim, g, um, up, n, f); break;
    default: flux_central(dim, g, um, up, n, f); break;
  }
}

/* entropy variables for U = -rho s/(gamma-1), s = ln p - gamma ln rho (R2) */
void orc_entropy_vars(int dim, double g, const double *u, double *w) {
  double rho, v[3], p;
  primitives(dim, g, u, &rho, v, &p);
  double s = log(p) - g * log(rho);
  double v2 = 0.0;
  for (int m = 0; m < dim; ++m) v2 += v[m] * v[m];
  w[0] = (g - s) / (g - 1.0) - 0.5 * rho * v2 / p;
  for (int m = 0; m < dim; ++m) w[1 + m] = rho * v[m] / p;
  w[dim + 1] = -rho / p;
}

/* inverse of orc_entropy_vars: u(w) for the same entropy (R2).  With
 * beta = -w_E = rho/p: v = w_m/beta, s = gamma - (gamma-1)(w_0 + beta|v|^2/2),
 * ln p = (s + gamma ln beta)/(1 - gamma), rho = beta p. */
void orc_cons_from_entropy(int dim, double g, const double *w, double *u) {
  double beta = -w[dim + 1];
  double v[3] = {0.0, 0.0, 0.0}, v2 = 0.0;
  for (int m = 0; m < dim; ++m) {
    v[m] = w[1 + m] / beta;
    v2 += v[m] * v[m];
  }
  double s = g - (g - 1.0) * (w[0] + 0.5 * beta * v2);
  double p = exp((s + g * log(beta)) / (1.0 - g));
  double rho = beta * p;
  u[0] = rho;
  for (int m = 0; m < dim; ++m) u[1 + m] = rho * v[m];
  u[dim + 1] = p / (g - 1.0) + 0.5 * rho * v2;
}

/* entropy U and entropy flux in direction n: F.n = U (v.n) (R2) */
void orc_entropy(int dim, double g, const double *u, const double *n,
                 double *U, double *Fn) {
  double rho, v[3], p;
  primitives(dim, g, u, &rho, v, &p);
  double s = log(p) - g * log(rho);
  double vn = 0.0;
  for (int m = 0; m < dim; ++m) vn += v[m] * n[m];
  *U = -rho * s / (g - 1.0);
  *Fn = *U * vn;
}

/* ------------------------------------------------------------------------ */
/* Mesh: node coordinates and metric terms (Sec. 2.3)                        */
/* ------------------------------------------------------------------------ */

static int ipow(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

/* multi-index of node i (x fastest) */
static void node_index(int N, int dim, int i, int idx[3]) {
  idx[0] = i % N;
  idx[1] = dim > 1 ? (i / N) % N : 0;
  idx[2] = dim > 2 ? i / (N * N) : 0;
}

static int node_of(int N, int dim, const int idx[3]) {
  int i = idx[0];
  if (dim > 1) i += N * idx[1];
  if (dim > 2) i += N * N * idx[2];
  return i;
}

static void elem_index(const orc_desc *d, int64_t e, int ie[3]) {
  ie[0] = (int)(e % d->n[0]);
  ie[1] = d->dim > 1 ? (int)((e / d->n[0]) % d->n[1]) : 0;
  ie[2] = d->dim > 2 ? (int)(e / ((int64_t)d->n[0] * d->n[1])) : 0;
}

static int64_t elem_of(const orc_desc *d, const int ie[3]) {
  int64_t e = ie[0];
  if (d->dim > 1) e += (int64_t)d->n[0] * ie[1];
  if (d->dim > 2) e += (int64_t)d->n[0] * d->n[1] * ie[2];
  return e;
}

/* neighbour of element e in direction n, side s = +1 or -1 (periodic) */
static int64_t neighbour(const orc_desc *d, int64_t e, int n, int s) {
  int ie[3];
  elem_index(d, e, ie);
  ie[n] = (ie[n] + s + d->n[n]) % d->n[n];
  return elem_of(d, ie);
}

/* apply the reference derivative in direction dir to nodal field a -> b */
static void ref_deriv(const orc_mesh *m, int dir, const double *a, double *b) {
  int N = m->N, dim = m->d.dim;
  for (int i = 0; i < m->nn; ++i) {
    int idx[3], jdx[3];
    node_index(N, dim, i, idx);
    double s = 0.0;
    for (int k = 0; k < N; ++k) {
      memcpy(jdx, idx, sizeof(idx));
      jdx[dir] = k;
      s += m->D[idx[dir] * N + k] * a[node_of(N, dim, jdx)];
    }
    b[i] = s;
  }
}

/* metric terms of one element from its node coordinates X[m][i] */
static void element_metrics(const orc_mesh *m, const double *X, double *Ja,
                            double *J) {
  int dim = m->d.dim, nn = m->nn;
  /* covariant derivatives dX[j][mm][i] = (D_j X_mm)_i */
  double *dX = (double *)malloc(sizeof(double) * 9 * nn);
  for (int j = 0; j < dim; ++j)
    for (int mm = 0; mm < dim; ++mm) ref_deriv(m, j, X + mm * nn, dX + (j * 3 + mm) * nn);
  for (int q = 0; q < 9 * nn; ++q) Ja[q] = 0.0;
  if (dim == 1) {
    for (int i = 0; i < nn; ++i) Ja[i] = 1.0;
  } else if (dim == 2) {
    /* cross-product form (Sec. 2.3) */
    for (int i = 0; i < nn; ++i) {
      Ja[(0 * 3 + 0) * nn + i] = dX[(1 * 3 + 1) * nn + i];  /* (Ja)^1_1 =  D_2 x^2 */
      Ja[(0 * 3 + 1) * nn + i] = -dX[(1 * 3 + 0) * nn + i]; /* (Ja)^1_2 = -D_2 x^1 */
      Ja[(1 * 3 + 0) * nn + i] = -dX[(0 * 3 + 1) * nn + i]; /* (Ja)^2_1 = -D_1 x^2 */
      Ja[(1 * 3 + 1) * nn + i] = dX[(0 * 3 + 0) * nn + i];  /* (Ja)^2_2 =  D_1 x^1 */
    }
  } else {
    /* conservative curl form:
     * (Ja)^i_n = D_{i+2}(X_l D_{i+1} X_m) - D_{i+1}(X_l D_{i+2} X_m),
     * (n, m, l) cyclic, directions counted modulo 3. */
    double *t1 = (double *)malloc(sizeof(double) * nn);
    double *t2 = (double *)malloc(sizeof(double) * nn);
    double *g1 = (double *)malloc(sizeof(double) * nn);
    double *g2 = (double *)malloc(sizeof(double) * nn);
    for (int i = 0; i < 3; ++i) {
      int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
      for (int n = 0; n < 3; ++n) {
        int mm = (n + 1) % 3, l = (n + 2) % 3;
        for (int q = 0; q < nn; ++q) {
          t1[q] = X[l * nn + q] * dX[(i1 * 3 + mm) * nn + q];
          t2[q] = X[l * nn + q] * dX[(i2 * 3 + mm) * nn + q];
        }
        ref_deriv(m, i2, t1, g1);
        ref_deriv(m, i1, t2, g2);
        for (int q = 0; q < nn; ++q) Ja[(i * 3 + n) * nn + q] = g1[q] - g2[q];
      }
    }
    free(t1); free(t2); free(g1); free(g2);
  }
  /* J = det(dx/dxi) with (dx/dxi)_{mm j} = D_j x^mm */
  for (int q = 0; q < nn; ++q) {
    double a[3][3];
    for (int mm = 0; mm < 3; ++mm)
      for (int j = 0; j < 3; ++j)
        a[mm][j] = (mm < dim && j < dim) ? dX[(j * 3 + mm) * nn + q] : (mm == j ? 1.0 : 0.0);
    J[q] = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
           a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
           a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  }
  free(dX);
}

/* Default node coordinates: uniform subdivision of the box; the reference
 * point of node xi in element e is lo + (e + (xi+1)/2) h, optionally warped
 * by x_m += warp * prod_j sin(pi s_j), s_j the coordinate scaled to [-1,1]. */
static void default_coords(orc_mesh *m) {
  const orc_desc *d = &m->d;
  int dim = d->dim, N = m->N, nn = m->nn;
  for (int64_t e = 0; e < m->ne; ++e) {
    int ie[3];
    elem_index(d, e, ie);
    for (int i = 0; i < nn; ++i) {
      int idx[3];
      node_index(N, dim, i, idx);
      double xh[3], s[3];
      for (int j = 0; j < dim; ++j) {
        double h = (d->hi[j] - d->lo[j]) / d->n[j];
        xh[j] = d->lo[j] + (ie[j] + 0.5 * (m->xi[idx[j]] + 1.0)) * h;
        s[j] = 2.0 * (xh[j] - d->lo[j]) / (d->hi[j] - d->lo[j]) - 1.0;
      }
      double bump = 1.0;
      for (int j = 0; j < dim; ++j) bump *= sin(M_PI * s[j]);
      for (int j = 0; j < dim; ++j)
        m->x[(e * dim + j) * nn + i] = xh[j] + d->warp * bump;
    }
  }
}

/* Build the mesh; coords (layout [elem][dim][node]) may be NULL. */
orc_mesh *orc_mesh_new(const orc_desc *desc, const double *coords) {
  if (desc->dim < 1 || desc->dim > 3 || desc->p < 1 || desc->p >= ORC_MAXN) return NULL;
  orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
  m->d = *desc;
  for (int j = desc->dim; j < 3; ++j) m->d.n[j] = 1;
  m->N = desc->p + 1;
  m->nn = ipow(m->N, desc->dim);
  m->ne = (int64_t)m->d.n[0] * m->d.n[1] * m->d.n[2];
  m->nv = desc->dim + 2;
  if (desc->nodes == 1) {
    if (desc->warp != 0.0 || coords) { free(m); return NULL; } /* affine only */
    orc_gauss(desc->p, m->xi, m->w, m->D, m->rL, m->rR);
  } else {
    orc_lgl(desc->p, m->xi, m->w, m->D);
  }
  m->x = (double *)malloc(sizeof(double) * m->ne * desc->dim * m->nn);
  m->Ja = (double *)malloc(sizeof(double) * m->ne * 9 * m->nn);
  m->J = (double *)malloc(sizeof(double) * m->ne * m->nn);
  if (coords)
    memcpy(m->x, coords, sizeof(double) * m->ne * desc->dim * m->nn);
  else
    default_coords(m);
#pragma omp parallel
  {
  double *X = (double *)malloc(sizeof(double) * 3 * m->nn);
#pragma omp for schedule(static)
  for (int64_t e = 0; e < m->ne; ++e) {
    /* Coordinates relative to the element's first node: the metric terms
     * only involve derivatives of the coordinates and, in the curl form,
     * D_a(c D_b X) - D_b(c D_a X) = 0 for a constant c, so the shift leaves
     * them unchanged while keeping the products X_l D X_m at the element's
     * own scale instead of the box's (their rounding would otherwise spoil
     * free-stream preservation on small elements far from the origin). */
    for (int j = 0; j < 3; ++j) {
      double c = j < desc->dim ? m->x[(e * desc->dim + j) * m->nn] : 0.0;
      for (int i = 0; i < m->nn; ++i)
        X[j * m->nn + i] = j < desc->dim ? m->x[(e * desc->dim + j) * m->nn + i] - c : 0.0;
    }
    element_metrics(m, X, m->Ja + e * 9 * m->nn, m->J + e * m->nn);
  }
  free(X);
  }
  return m;
}

void orc_mesh_free(orc_mesh *m) {
  if (!m) return;
  free(m->x); free(m->Ja); free(m->J); free(m);
}

void orc_mesh_sizes(const orc_mesh *m, int64_t *ne, int32_t *nn, int32_t *nv) {
  *ne = m->ne; *nn = m->nn; *nv = m->nv;
}

void orc_mesh_geometry(const orc_mesh *m, double *x, double *Ja, double *J) {
  if (x) memcpy(x, m->x, sizeof(double) * m->ne * m->d.dim * m->nn);
  if (Ja) memcpy(Ja, m->Ja, sizeof(double) * m->ne * 9 * m->nn);
  if (J) memcpy(J, m->J, sizeof(double) * m->ne * m->nn);
}

void orc_mesh_operators(const orc_mesh *m, double *xi, double *w, double *D) {
  memcpy(xi, m->xi, sizeof(double) * m->N);
  memcpy(w, m->w, sizeof(double) * m->N);
  memcpy(D, m->D, sizeof(double) * m->N * m->N);
}

/* ------------------------------------------------------------------------ */
/* Semi-discretisation du/dt = RHS(u)                                       */
/* ------------------------------------------------------------------------ */

static void gather(const orc_mesh *m, const double *u, int64_t e, int i, double *ui) {
  for (int v = 0; v < m->nv; ++v) ui[v] = u[(e * m->nv + v) * m->nn + i];
}

static void ja_row(const orc_mesh *m, int64_t e, int n, int i, double *a) {
  for (int mm = 0; mm < 3; ++mm) a[mm] = m->Ja[((e * 3 + n) * 3 + mm) * m->nn + i];
}

/* RHS_i = -(1/J_i) [ sum_n sum_k 2 D_{i_n k} f_vol(u_i, u_k, (Ja^n_i + Ja^n_k)/2)
 *                    + sum_n (boundary terms of M^-1 R^T B (f* - N f)) ]         */
/* RHS of one element (all its nodes) */
static void rhs_element(const orc_mesh *m, const double *u, double *du, int64_t e) {
  const int dim = m->d.dim, N = m->N, nn = m->nn, nv = m->nv, p = m->d.p;
  const double g = m->d.gamma;
  for (int i = 0; i < nn; ++i) {
    int idx[3];
    node_index(N, dim, i, idx);
    double ui[5], acc[5] = {0, 0, 0, 0, 0};
    gather(m, u, e, i, ui);
    for (int n = 0; n < dim; ++n) {
      double ai[3];
      ja_row(m, e, n, i, ai);
      /* volume: flux differencing along the line through i in direction n */
      for (int k = 0; k < N; ++k) {
        int jdx[3];
        memcpy(jdx, idx, sizeof(idx));
        jdx[n] = k;
        int j = node_of(N, dim, jdx);
        double uj[5], aj[3], nrm[3], f[5];
        gather(m, u, e, j, uj);
        ja_row(m, e, n, j, aj);
        for (int mm = 0; mm < 3; ++mm) nrm[mm] = 0.5 * (ai[mm] + aj[mm]);
        orc_two_point(m->d.vol_flux, dim, g, ui, uj, nrm, f);
        for (int v = 0; v < nv; ++v) acc[v] += 2.0 * m->D[idx[n] * N + k] * f[v];
      }
      /* surface: i on the + face (i_n = p) or - face (i_n = 0) */
      for (int side = 0; side < 2; ++side) {
        int at = side ? p : 0;
        if (idx[n] != at) continue;
        int64_t eo = neighbour(&m->d, e, n, side ? +1 : -1);
        int odx[3];
        memcpy(odx, idx, sizeof(idx));
        odx[n] = side ? 0 : p;
        int io = node_of(N, dim, odx);
        double uo[5], ao[3], nf[3], fstar[5], fphys[5];
        gather(m, u, eo, io, uo);
        ja_row(m, eo, n, io, ao);
        for (int mm = 0; mm < 3; ++mm) nf[mm] = 0.5 * (ai[mm] + ao[mm]);
        orc_phys_flux(dim, g, ui, ai, fphys);
        if (side) {
          /* outward reference normal +1: f* = f(u_L = u_i, u_R = u_o, n_f) */
          orc_two_point(m->d.surf_flux, dim, g, ui, uo, nf, fstar);
          for (int v = 0; v < nv; ++v) acc[v] += (fstar[v] - fphys[v]) / m->w[p];
        } else {
          /* outward reference normal -1: f* = f(u_L = u_o, u_R = u_i, n_f) */
          orc_two_point(m->d.surf_flux, dim, g, uo, ui, nf, fstar);
          for (int v = 0; v < nv; ++v) acc[v] += (-fstar[v] + fphys[v]) / m->w[0];
        }
      }
    }
    double Ji = m->J[e * nn + i];
    for (int v = 0; v < nv; ++v) du[(e * nv + v) * nn + i] = -acc[v] / Ji;
  }
}

/* Entropy-projected state at the face point of a line (Sec. 6): w along the
 * line of element e through the multi-index idx in direction n, interpolated
 * to the end `side` (0: -1, 1: +1), mapped back to conservative variables. */
static void projected_face_state(const orc_mesh *m, const double *u, int64_t e, const int idx[3], int n,
                                 int side, double *ut) {
  const int dim = m->d.dim, N = m->N, nv = m->nv;
  double wf[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < N; ++k) {
    int jdx[3];
    memcpy(jdx, idx, 3 * sizeof(int));
    jdx[n] = k;
    double uk[5], wk[5];
    gather(m, u, e, node_of(N, dim, jdx), uk);
    orc_entropy_vars(dim, m->d.gamma, uk, wk);
    const double r = side ? m->rR[k] : m->rL[k];
    for (int v = 0; v < nv; ++v) wf[v] += r * wk[v];
  }
  orc_cons_from_entropy(dim, m->d.gamma, wf, ut);
}

/* Legendre-Gauss collocation, hybridised form (Sec. 6):
 *   du/dt = -(1/J) [ M^-1 [I; R]^T f_hyb + M^-1 R^T B f_num ],
 *   f_hyb_a = sum_n sum_b 2 (Q_h,n)_ab f(u~_a, u~_b),
 *   Q_h = 1/2 [[M D - (M D)^T, R^T B], [-B R, 0]],  u~ = [u; u(R w(u))],
 * per line of an affine element (the tensor-product factors of M, B and the
 * face weights cancel line by line), B = diag(-1, +1) for the face points at
 * -1 and +1.  With abs_mode the magnitudes of all terms are summed instead
 * (rounding scale of the result). */
static void rhs_element_gauss(const orc_mesh *m, const double *u, double *out, int64_t e, int abs_mode) {
  const int dim = m->d.dim, N = m->N, nn = m->nn, nv = m->nv;
  const double g = m->d.gamma;
  const int NH = N + 2;
  double acc[5 * 4096];
  memset(acc, 0, sizeof(double) * nv * nn);
  double Q[(ORC_MAXN + 2) * (ORC_MAXN + 2)];
  for (int a = 0; a < NH * NH; ++a) Q[a] = 0.0;
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k)
      Q[i * NH + k] = 0.5 * (m->w[i] * m->D[i * N + k] - m->w[k] * m->D[k * N + i]);
  for (int k = 0; k < N; ++k) {
    Q[k * NH + N] = 0.5 * (-m->rL[k]);      /* (R^T B)_{k,L} / 2 */
    Q[k * NH + N + 1] = 0.5 * (m->rR[k]);   /* (R^T B)_{k,R} / 2 */
    Q[N * NH + k] = 0.5 * (m->rL[k]);       /* (-B R)_{L,k} / 2 */
    Q[(N + 1) * NH + k] = 0.5 * (-m->rR[k]); /* (-B R)_{R,k} / 2 */
  }
  for (int n = 0; n < dim; ++n) {
    double a[3];
    ja_row(m, e, n, 0, a); /* affine: one contravariant vector per direction */
    /* every line in direction n: the nodes with idx[n] = 0 start one */
    for (int i0 = 0; i0 < nn; ++i0) {
      int idx[3];
      node_index(N, dim, i0, idx);
      if (idx[n] != 0) continue;
      double ut[ORC_MAXN + 2][5];
      int node[ORC_MAXN];
      for (int k = 0; k < N; ++k) {
        int jdx[3];
        memcpy(jdx, idx, sizeof(jdx));
        jdx[n] = k;
        node[k] = node_of(N, dim, jdx);
        gather(m, u, e, node[k], ut[k]);
      }
      projected_face_state(m, u, e, idx, n, 0, ut[N]);
      projected_face_state(m, u, e, idx, n, 1, ut[N + 1]);
      /* neighbours' face states at the same two points */
      double un_L[5], un_R[5];
      projected_face_state(m, u, neighbour(&m->d, e, n, -1), idx, n, 1, un_L);
      projected_face_state(m, u, neighbour(&m->d, e, n, +1), idx, n, 0, un_R);
      double fh[ORC_MAXN + 2][5];
      for (int x = 0; x < NH; ++x) {
        for (int v = 0; v < nv; ++v) fh[x][v] = 0.0;
        for (int y = 0; y < NH; ++y) {
          if (Q[x * NH + y] == 0.0) continue;
          double f[5];
          orc_two_point(m->d.vol_flux, dim, g, ut[x], ut[y], a, f);
          for (int v = 0; v < nv; ++v) {
            const double t = 2.0 * Q[x * NH + y] * f[v];
            fh[x][v] += abs_mode ? fabs(t) : t;
          }
        }
      }
      double fL[5], fR[5];
      orc_two_point(m->d.surf_flux, dim, g, un_L, ut[N], a, fL);     /* face at -1: (neighbour, own) */
      orc_two_point(m->d.surf_flux, dim, g, ut[N + 1], un_R, a, fR); /* face at +1: (own, neighbour) */
      for (int k = 0; k < N; ++k)
        for (int v = 0; v < nv; ++v) {
          double t[5] = {fh[k][v], m->rL[k] * fh[N][v], m->rR[k] * fh[N + 1][v], -m->rL[k] * fL[v],
                         m->rR[k] * fR[v]};
          double sum = 0.0;
          for (int q = 0; q < 5; ++q) sum += abs_mode ? fabs(t[q]) : t[q];
          acc[v * nn + node[k]] += sum / m->w[k];
        }
    }
  }
  for (int i = 0; i < nn; ++i) {
    const double Ji = m->J[e * nn + i];
    for (int v = 0; v < nv; ++v)
      out[(e * nv + v) * nn + i] = abs_mode ? acc[v * nn + i] / fabs(Ji) : -acc[v * nn + i] / Ji;
  }
}

void orc_rhs(const orc_mesh *m, const double *u, double *du) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m->ne; ++e) {
    if (m->d.nodes == 1) rhs_element_gauss(m, u, du, e, 0);
    else rhs_element(m, u, du, e);
  }
}

/* RHS of the listed elements only (du has the full layout; other elements
 * are left untouched) -- for sampled checks of large meshes */
void orc_rhs_elements(const orc_mesh *m, const double *u, double *du, const int64_t *elems, int64_t count) {
#pragma omp parallel for schedule(dynamic)
  for (int64_t q = 0; q < count; ++q) {
    if (m->d.nodes == 1) rhs_element_gauss(m, u, du, elems[q], 0);
    else rhs_element(m, u, du, elems[q]);
  }
}

/* Rounding scale of RHS_i: the same sums as orc_rhs with every term replaced
 * by its magnitude, sc_i = (1/J_i) [ sum_n sum_k |2 D_{i_n k} f_vol| +
 * sum_n (|f*| + |f^n(u_i)|)/w_end ].  A floating-point evaluation of RHS_i in
 * any order has an error of at most a few eps * sc_i; it is the natural
 * denominator of a relative parity bound where RHS_i itself cancels. */
static void scale_element(const orc_mesh *m, const double *u, double *sc, int64_t e) {
  const int dim = m->d.dim, N = m->N, nn = m->nn, nv = m->nv, p = m->d.p;
  const double g = m->d.gamma;
  for (int i = 0; i < nn; ++i) {
    int idx[3];
    node_index(N, dim, i, idx);
    double ui[5], acc[5] = {0, 0, 0, 0, 0};
    gather(m, u, e, i, ui);
    for (int n = 0; n < dim; ++n) {
      double ai[3];
      ja_row(m, e, n, i, ai);
      for (int k = 0; k < N; ++k) {
        int jdx[3];
        memcpy(jdx, idx, sizeof(idx));
        jdx[n] = k;
        int j = node_of(N, dim, jdx);
        double uj[5], aj[3], nrm[3], f[5];
        gather(m, u, e, j, uj);
        ja_row(m, e, n, j, aj);
        for (int mm = 0; mm < 3; ++mm) nrm[mm] = 0.5 * (ai[mm] + aj[mm]);
        orc_two_point(m->d.vol_flux, dim, g, ui, uj, nrm, f);
        for (int v = 0; v < nv; ++v) acc[v] += fabs(2.0 * m->D[idx[n] * N + k] * f[v]);
      }
      for (int side = 0; side < 2; ++side) {
        int at = side ? p : 0;
        if (idx[n] != at) continue;
        int64_t eo = neighbour(&m->d, e, n, side ? +1 : -1);
        int odx[3];
        memcpy(odx, idx, sizeof(idx));
        odx[n] = side ? 0 : p;
        int io = node_of(N, dim, odx);
        double uo[5], ao[3], nf[3], fstar[5], fphys[5];
        gather(m, u, eo, io, uo);
        ja_row(m, eo, n, io, ao);
        for (int mm = 0; mm < 3; ++mm) nf[mm] = 0.5 * (ai[mm] + ao[mm]);
        orc_phys_flux(dim, g, ui, ai, fphys);
        if (side) orc_two_point(m->d.surf_flux, dim, g, ui, uo, nf, fstar);
        else orc_two_point(m->d.surf_flux, dim, g, uo, ui, nf, fstar);
        for (int v = 0; v < nv; ++v) acc[v] += (fabs(fstar[v]) + fabs(fphys[v])) / m->w[at];
      }
    }
    double Ji = m->J[e * nn + i];
    for (int v = 0; v < nv; ++v) sc[(e * nv + v) * nn + i] = acc[v] / fabs(Ji);
  }
}

void orc_rhs_scale(const orc_mesh *m, const double *u, double *sc) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m->ne; ++e) {
    if (m->d.nodes == 1) rhs_element_gauss(m, u, sc, e, 1);
    else scale_element(m, u, sc, e);
  }
}

void orc_rhs_scale_elements(const orc_mesh *m, const double *u, double *sc, const int64_t *elems, int64_t count) {
#pragma omp parallel for schedule(dynamic)
  for (int64_t q = 0; q < count; ++q) {
    if (m->d.nodes == 1) rhs_element_gauss(m, u, sc, elems[q], 1);
    else scale_element(m, u, sc, elems[q]);
  }
}

/* ------------------------------------------------------------------------ */
/* Reductions (Sec. 2: conservation and entropy of the semi-discretisation)  */
/* ------------------------------------------------------------------------ */

static double weight(const orc_mesh *m, int i) {
  int idx[3];
  node_index(m->N, m->d.dim, i, idx);
  double W = 1.0;
  for (int j = 0; j < m->d.dim; ++j) W *= m->w[idx[j]];
  return W;
}

/* totals_v = sum_e sum_i J_i W_i u_{i,v} */
void orc_totals(const orc_mesh *m, const double *u, double *tot) {
  for (int v = 0; v < m->nv; ++v) {
    long double s = 0.0L;
    for (int64_t e = 0; e < m->ne; ++e)
      for (int i = 0; i < m->nn; ++i)
        s += (long double)m->J[e * m->nn + i] * weight(m, i) * u[(e * m->nv + v) * m->nn + i];
    tot[v] = (double)s;
  }
}

/* dS/dt = sum J_i W_i w(u_i) . du_i  for a given du (e.g. RHS(u)) */
double orc_entropy_rate(const orc_mesh *m, const double *u, const double *du) {
  long double s = 0.0L;
  for (int64_t e = 0; e < m->ne; ++e)
    for (int i = 0; i < m->nn; ++i) {
      double ui[5], w[5];
      gather(m, u, e, i, ui);
      orc_entropy_vars(m->d.dim, m->d.gamma, ui, w);
      double JW = m->J[e * m->nn + i] * weight(m, i);
      for (int v = 0; v < m->nv; ++v)
        s += (long double)JW * w[v] * du[(e * m->nv + v) * m->nn + i];
    }
  return (double)s;
}

/* R17: dt = cfl * 2 / ((p+1) max_i sum_n (|v.Ja^n_i| + c_i |Ja^n_i|) / J_i) */
double orc_max_dt(const orc_mesh *m, const double *u, double cfl) {
  double lmax = 0.0;
  for (int64_t e = 0; e < m->ne; ++e)
    for (int i = 0; i < m->nn; ++i) {
      double ui[5], rho, v[3], p;
      gather(m, u, e, i, ui);
      primitives(m->d.dim, m->d.gamma, ui, &rho, v, &p);
      double c = sqrt(m->d.gamma * p / rho);
      double lam = 0.0;
      for (int n = 0; n < m->d.dim; ++n) {
        double a[3], vn = 0.0, an = 0.0;
        ja_row(m, e, n, i, a);
        for (int mm = 0; mm < m->d.dim; ++mm) {
          vn += v[mm] * a[mm];
          an += a[mm] * a[mm];
        }
        lam += fabs(vn) + c * sqrt(an);
      }
      lam /= m->J[e * m->nn + i];
      if (lam > lmax) lmax = lam;
    }
  return cfl * 2.0 / (m->N * lmax);
}

/* ------------------------------------------------------------------------ */
/* Classical RK4 (textbook form with four stage derivatives)                 */
/* ------------------------------------------------------------------------ */

/* Advance u in place by nsteps steps of size dt (dt > 0), or of the CFL step
 * size (dt <= 0, recomputed at the start of every step).  t is advanced. */
void orc_rk4(const orc_mesh *m, double *u, double dt, int nsteps, double cfl,
             double *t) {
  size_t len = (size_t)m->ne * m->nv * m->nn;
  double *k1 = (double *)malloc(sizeof(double) * len);
  double *k2 = (double *)malloc(sizeof(double) * len);
  double *k3 = (double *)malloc(sizeof(double) * len);
  double *k4 = (double *)malloc(sizeof(double) * len);
  double *y = (double *)malloc(sizeof(double) * len);
  for (int s = 0; s < nsteps; ++s) {
    double h = dt > 0.0 ? dt : orc_max_dt(m, u, cfl);
    orc_rhs(m, u, k1);
    for (size_t q = 0; q < len; ++q) y[q] = u[q] + 0.5 * h * k1[q];
    orc_rhs(m, y, k2);
    for (size_t q = 0; q < len; ++q) y[q] = u[q] + 0.5 * h * k2[q];
    orc_rhs(m, y, k3);
    for (size_t q = 0; q < len; ++q) y[q] = u[q] + h * k3[q];
    orc_rhs(m, y, k4);
    for (size_t q = 0; q < len; ++q)
      u[q] = u[q] + h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    if (t) *t += h;
  }
  free(k1); free(k2); free(k3); free(k4); free(y);
}

/* ------------------------------------------------------------------------ */
/* Five-stage, fourth-order 2N-storage RK of Carpenter and Kennedy (1994),   */
/* the scheme of the paper's FLUXO runs (Sec. 4.1), in Williamson's form:    */
/*   du <- A_i du + h RHS(u);  u <- u + B_i du,   i = 1..5, A_1 = 0          */
/* ------------------------------------------------------------------------ */

static const double CK_A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
static const double CK_B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};

void orc_ck45_coefficients(double *A, double *B) {
  for (int i = 0; i < 5; ++i) {
    A[i] = CK_A[i];
    B[i] = CK_B[i];
  }
}

/* As orc_rk4, with the 2N scheme (dt <= 0: CFL step size at the start of
 * every step). */
void orc_ck45(const orc_mesh *m, double *u, double dt, int nsteps, double cfl,
              double *t) {
  size_t len = (size_t)m->ne * m->nv * m->nn;
  double *k = (double *)malloc(sizeof(double) * len);
  double *du = (double *)calloc(len, sizeof(double));
  for (int s = 0; s < nsteps; ++s) {
    double h = dt > 0.0 ? dt : orc_max_dt(m, u, cfl);
    for (int i = 0; i < 5; ++i) {
      orc_rhs(m, u, k);
      for (size_t q = 0; q < len; ++q) {
        du[q] = CK_A[i] * du[q] + h * k[q];
        u[q] = u[q] + CK_B[i] * du[q];
      }
    }
    if (t) *t += h;
  }
  free(k); free(du);
}
