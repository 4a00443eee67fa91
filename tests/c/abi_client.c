/* A plain C99 client of the esdg C ABI (include/esdg.h), built and run by
 * tests/test_abi_c.py.  Without arguments it makes only host-side calls
 * (operators, footprint, descriptor validation, NULL handles); with --gpu it
 * also runs problems through host buffers and checks properties the method
 * fixes: free-stream preservation on a warped mesh (Sec. 2.3), discrete
 * conservation of the totals over RK steps (Sec. 2), zero entropy rate of the
 * entropy-conservative volume and surface fluxes, negative with LLF
 * (Sec. 3.2), and bit-identical results of a problem stepped alone and in a
 * batch.  Exit status 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "esdg.h"

static int failures = 0;

#define CHECK(cond, ...)                          \
  do {                                            \
    if (!(cond)) {                                \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);               \
      fprintf(stderr, "\n");                      \
      ++failures;                                 \
    }                                             \
  } while (0)

#define OK(call)                                                                      \
  do {                                                                                \
    esdg_status st_ = (call);                                                         \
    if (st_ != ESDG_OK) {                                                             \
      fprintf(stderr, "FAIL %s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #call, (int)st_, \
              esdg_last_error(NULL));                                                 \
      exit(1);                                                                        \
    }                                                                                 \
  } while (0)

static esdg_mesh_desc box(int p, int n, double warp, int vol, int surf) {
  esdg_mesh_desc d;
  int j;
  memset(&d, 0, sizeof d);
  d.dim = 3;
  d.p = p;
  for (j = 0; j < 3; ++j) {
    d.n[j] = n;
    d.lo[j] = -1.0;
    d.hi[j] = 1.0;
  }
  d.warp = warp;
  d.gamma = 1.4;
  d.volume_flux = vol;
  d.surface_flux = surf;
  d.precision = ESDG_FP64;
  d.nodes = ESDG_NODES_LGL;
  return d;
}

static void host_checks(void) {
  double x[8], w[8], D[64], Dt[64], s = 0.0;
  int i;
  int64_t bytes = 0;
  esdg_mesh_desc d = box(3, 4, 0.1, ESDG_FLUX_RANOCHA, ESDG_FLUX_LLF);
  esdg_problem *prob = (esdg_problem *)0;
  printf("%s\n", esdg_version());
  OK(esdg_operators(3, x, w, D, Dt));
  for (i = 0; i < 4; ++i) s += w[i];
  CHECK(fabs(s - 2.0) < 1e-14, "LGL weights sum to %.17g", s);
  CHECK(x[0] == -1.0 && x[3] == 1.0, "LGL end nodes %g %g", x[0], x[3]);
  CHECK(esdg_operators(ESDG_PMAX + 1, x, w, D, Dt) == ESDG_EINVAL, "degree above ESDG_PMAX accepted");
  OK(esdg_footprint(&d, &bytes));
  CHECK(bytes > 5 * 64 * 64 * 5 * 8, "footprint %lld below the five state arrays", (long long)bytes);
  d.dim = 4;
  CHECK(esdg_init_mesh(&d, &prob) == ESDG_EINVAL && prob == (esdg_problem *)0, "dim 4 accepted");
  CHECK(strlen(esdg_last_error(NULL)) > 0, "no error message for dim 4");
  CHECK(esdg_rhs((esdg_problem *)0, (double *)0, ESDG_HOST) == ESDG_EINVAL, "NULL handle accepted");
  {
    const int64_t q[3] = {10, 20, 30};
    int32_t k = -1;
    OK(esdg_server_plan(q, 3, 0, 35, 0, 0, &k));
    CHECK(k == 2, "admission of 10, 20, 30 bytes in a budget of 35: %d", (int)k);
  }
  esdg_destroy((esdg_problem *)0);
}

/* smooth periodic state from the node coordinates */
static void smooth_state(const double *x, int64_t E, int nn, double *u) {
  int64_t e;
  int i;
  const double pi = 3.14159265358979323846;
  for (e = 0; e < E; ++e)
    for (i = 0; i < nn; ++i) {
      const double *xe = x + e * 3 * nn;
      const double a = xe[i], b = xe[nn + i], c = xe[2 * nn + i];
      const double rho = 1.0 + 0.2 * sin(pi * a) * cos(pi * b);
      const double v0 = 0.1 * sin(pi * c), v1 = -0.05 * cos(pi * a), v2 = 0.08 * sin(pi * (a + b));
      const double p = 1.0 + 0.1 * cos(pi * (b + c));
      double *ue = u + e * 5 * nn;
      ue[i] = rho;
      ue[nn + i] = rho * v0;
      ue[2 * nn + i] = rho * v1;
      ue[3 * nn + i] = rho * v2;
      ue[4 * nn + i] = p / 0.4 + 0.5 * rho * (v0 * v0 + v1 * v1 + v2 * v2);
    }
}

static void gpu_checks(void) {
  esdg_mesh_desc d = box(3, 4, 0.1, ESDG_FLUX_RANOCHA, ESDG_FLUX_LLF);
  esdg_problem *g = (esdg_problem *)0, *h = (esdg_problem *)0, *ec = (esdg_problem *)0;
  esdg_batch *b = (esdg_batch *)0;
  esdg_problem *members[2];
  int64_t E, k, n;
  int32_t nn, nv, v;
  double *x, *u, *du, *u2, tot0[5], tot1[5], rate_ec, rate_llf, umax = 0.0, dmax = 0.0;

  OK(esdg_init_mesh(&d, &g));
  OK(esdg_sizes(g, &E, &nn, &nv));
  n = E * nv * nn;
  x = (double *)malloc(sizeof(double) * (size_t)(E * 3 * nn));
  u = (double *)malloc(sizeof(double) * (size_t)n);
  u2 = (double *)malloc(sizeof(double) * (size_t)n);
  du = (double *)malloc(sizeof(double) * (size_t)n);
  CHECK(esdg_get_state(g, u, ESDG_HOST) == ESDG_ESTATE, "state read before esdg_set_state");
  OK(esdg_get_coords(g, x));

  /* 1/J: positive, and sum_i W_i J_i over the warped mesh is the box volume 8
   * to round-off: the warp adds one scalar phi to every coordinate, so the
   * collocation Jacobian is (h/2)^3 (1 + sum_k D_k phi), and by the SBP
   * property the weighted sum of D_k phi over an element is a difference of
   * face values, which cancels over the periodic mesh */
  {
    double ox[4], ow[4], oD[16], oDt[16], vol = 0.0;
    double *inv_j = (double *)malloc(sizeof(double) * (size_t)(E * nn));
    int i;
    CHECK(esdg_get_inv_jacobian(g, (double *)0) == ESDG_EINVAL, "NULL 1/J buffer accepted");
    OK(esdg_get_inv_jacobian(g, inv_j));
    OK(esdg_operators(3, ox, ow, oD, oDt));
    for (k = 0; k < E; ++k)
      for (i = 0; i < nn; ++i) {
        CHECK(inv_j[k * nn + i] > 0.0, "1/J <= 0 at element %lld node %d", (long long)k, i);
        vol += ow[i % 4] * ow[(i / 4) % 4] * ow[i / 16] / inv_j[k * nn + i];
      }
    CHECK(fabs(vol - 8.0) < 1e-11, "sum W J = %.15f, box volume 8", vol);
    free(inv_j);
  }

  /* free stream on the warped mesh */
  for (k = 0; k < E; ++k)
    for (v = 0; v < nv; ++v) {
      const double c[5] = {1.2, 0.12, -0.24, 0.36, 0.9 / 0.4 + 0.5 * (0.12 * 0.12 + 0.24 * 0.24 + 0.36 * 0.36) / 1.2};
      int i;
      for (i = 0; i < nn; ++i) u[(k * nv + v) * nn + i] = c[v];
    }
  OK(esdg_set_state(g, u, ESDG_HOST));
  OK(esdg_rhs(g, du, ESDG_HOST));
  for (k = 0; k < n; ++k) dmax = fmax(dmax, fabs(du[k]));
  CHECK(dmax < 1e-11, "free stream: max |RHS| = %.3e", dmax);

  /* conservation over CFL steps */
  smooth_state(x, E, nn, u);
  OK(esdg_set_state(g, u, ESDG_HOST));
  OK(esdg_totals(g, tot0));
  OK(esdg_step(g, 0.0, 10, 0.5, (double *)0));
  OK(esdg_sync(g));
  OK(esdg_totals(g, tot1));
  for (v = 0; v < nv; ++v)
    CHECK(fabs(tot1[v] - tot0[v]) <= 1e-12 * (1.0 + fabs(tot0[v])), "total %d: %.17g -> %.17g", v, tot0[v], tot1[v]);

  /* entropy rate: EC volume + EC surface vs LLF surface, on a state with
   * jumps at the element faces (nodal noise; a continuous nodal state has no
   * jumps, and both surface fluxes then reduce to f(u).n) */
  d = box(3, 4, 0.1, ESDG_FLUX_RANOCHA, ESDG_FLUX_RANOCHA);
  OK(esdg_init_mesh(&d, &ec));
  smooth_state(x, E, nn, u);
  {
    unsigned long long r = 12345u;
    for (k = 0; k < n; ++k) {
      r = r * 6364136223846793005ull + 1442695040888963407ull;
      u[k] *= 1.0 + 0.01 * ((double)(r >> 11) / 9007199254740992.0 - 0.5);
    }
  }
  OK(esdg_set_state(ec, u, ESDG_HOST));
  OK(esdg_entropy_rate(ec, &rate_ec));
  OK(esdg_set_state(g, u, ESDG_HOST));
  OK(esdg_entropy_rate(g, &rate_llf));
  CHECK(rate_llf < 0.0, "LLF entropy rate %.3e not negative", rate_llf);
  CHECK(fabs(rate_ec) < 1e-8 * fabs(rate_llf), "EC entropy rate %.3e (LLF %.3e)", rate_ec, rate_llf);

  /* alone and in a batch: bit-identical */
  d = box(3, 4, 0.1, ESDG_FLUX_RANOCHA, ESDG_FLUX_LLF);
  OK(esdg_init_mesh(&d, &h));
  OK(esdg_set_state(g, u, ESDG_HOST));
  OK(esdg_set_state(h, u, ESDG_HOST));
  OK(esdg_step(g, 0.0, 4, 0.5, (double *)0));
  members[0] = h;
  members[1] = ec;
  OK(esdg_batch_create(members, 2, (const double *)0, (void *)0, 0, &b));
  OK(esdg_batch_step(b, 0.0, 4, 0.5));
  OK(esdg_batch_sync(b, (int32_t *)0));
  OK(esdg_get_state(g, u, ESDG_HOST));
  OK(esdg_get_state(h, u2, ESDG_HOST));
  CHECK(memcmp(u, u2, sizeof(double) * (size_t)n) == 0, "batched member differs from the problem stepped alone");
  for (k = 0; k < n; ++k) umax = fmax(umax, fabs(u[k]));
  CHECK(umax > 0.5 && umax < 10.0, "state magnitude %.3e after the steps", umax);

  esdg_batch_destroy(b);
  esdg_destroy(g);
  esdg_destroy(h);
  esdg_destroy(ec);
  free(x);
  free(u);
  free(u2);
  free(du);
}

int main(int argc, char **argv) {
  host_checks();
  if (argc > 1 && strcmp(argv[1], "--gpu") == 0) gpu_checks();
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("abi client ok%s\n", argc > 1 ? " (gpu)" : "");
  return 0;
}
