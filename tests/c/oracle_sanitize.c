/* Host sanitizer run of the oracle (built with -fsanitize=address,undefined
 * by tests/test_sanitizers.py): the oracle source is compiled into this
 * driver, which exercises every entry point on small 2D and 3D meshes (LGL
 * affine and warped, Gauss collocation, all fluxes) and checks that the
 * results are finite and that a constant state is steady. */
#include "../../oracle/esdg_oracle.c"

#include <stdio.h>

static int run(int dim, int p, int nx, double warp, int vol, int surf, int nodes) {
  orc_desc d;
  orc_mesh *m;
  int64_t ne, k, len;
  int32_t nn, nv;
  double *u, *du, *sc, tot[5], rate, dt, t = 0.0, dmax = 0.0;
  int j, v, i, bad = 0;
  memset(&d, 0, sizeof d);
  d.dim = dim;
  d.p = p;
  for (j = 0; j < 3; ++j) {
    d.n[j] = nx + j;
    d.lo[j] = -1.0;
    d.hi[j] = 1.0;
  }
  d.warp = warp;
  d.gamma = 1.4;
  d.vol_flux = vol;
  d.surf_flux = surf;
  d.nodes = nodes;
  m = orc_mesh_new(&d, NULL);
  if (!m) return 1;
  orc_mesh_sizes(m, &ne, &nn, &nv);
  len = ne * nv * nn;
  u = (double *)malloc(sizeof(double) * len);
  du = (double *)malloc(sizeof(double) * len);
  sc = (double *)malloc(sizeof(double) * len);
  /* constant state: steady */
  for (k = 0; k < ne; ++k)
    for (v = 0; v < nv; ++v)
      for (i = 0; i < nn; ++i) u[(k * nv + v) * nn + i] = v == 0 ? 1.1 : (v == nv - 1 ? 3.0 : 0.1 * v);
  orc_rhs(m, u, du);
  for (k = 0; k < len; ++k) dmax = fmax(dmax, fabs(du[k]));
  if (!(dmax < 1e-9)) bad = 1;
  /* perturbed state: every reduction and two RK4 steps */
  for (k = 0; k < len; ++k) u[k] *= 1.0 + 0.01 * sin(0.37 * (double)k);
  orc_rhs(m, u, du);
  orc_rhs_scale(m, u, sc);
  orc_totals(m, u, tot);
  rate = orc_entropy_rate(m, u, du);
  dt = orc_max_dt(m, u, 0.5);
  orc_rk4(m, u, 0.0, 2, 0.5, &t);
  for (k = 0; k < len; ++k)
    if (!isfinite(u[k]) || !isfinite(du[k]) || !isfinite(sc[k])) bad = 1;
  if (!isfinite(rate) || !(dt > 0.0) || !(t > 0.0)) bad = 1;
  printf("dim %d p %d warp %.1f flux %d/%d nodes %d: free-stream %.1e, rate %.2e, dt %.2e %s\n", dim, p, warp, vol,
         surf, nodes, dmax, rate, dt, bad ? "FAIL" : "ok");
  free(u);
  free(du);
  free(sc);
  orc_mesh_free(m);
  return bad;
}

int main(void) {
  int bad = 0;
  double x[8], w[8], D[64], rL[8], rR[8];
  bad |= orc_lgl(5, x, w, D) != 0;
  orc_gauss(4, x, w, D, rL, rR);
  bad |= !(fabs(orc_logmean(1.0, 1.0 + 1e-9) - 1.0) < 1e-8);
  bad |= !(orc_inv_logmean(2.0, 3.0) > 0.0);
  bad |= run(2, 3, 3, 0.0, 0, 2, 0);
  bad |= run(2, 5, 2, 0.1, 1, 0, 0);
  bad |= run(3, 2, 2, 0.1, 0, 0, 0);
  bad |= run(3, 4, 1, 0.1, 3, 3, 0);
  bad |= run(3, 3, 2, 0.0, 0, 2, 1);
  bad |= run(2, 6, 2, 0.0, 1, 1, 1);
  printf("%s\n", bad ? "oracle sanitize FAIL" : "oracle sanitize ok");
  return bad;
}
