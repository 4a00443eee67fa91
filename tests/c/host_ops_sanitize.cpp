// Host sanitizer run of the library's host code (operators and geometry,
// built with -fsanitize=address,undefined by tests/test_sanitizers.py):
// LGL and Gauss operators for every degree, and box meshes in 2D and 3D,
// affine, warped and from caller coordinates, including the periodic
// single-element case.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "host_ops.hpp"

using namespace esdg;

static int mesh(int dim, int p, int n0, double warp, bool with_coords) {
  Operators ops;
  std::string err;
  if (!make_operators(p, &ops, &err)) return 1;
  MeshSpec s;
  s.dim = dim;
  s.p = p;
  for (int j = 0; j < 3; ++j) s.n[j] = j < dim ? n0 + j : 1;
  s.warp = warp;
  Geometry g;
  if (!make_geometry(s, ops, &g, &err)) {
    std::printf("geometry: %s\n", err.c_str());
    return 1;
  }
  if (with_coords) {
    std::vector<double> x = g.coords;  // the warped nodes again, as caller coordinates
    MeshSpec c = s;
    c.warp = 0.0;
    c.coords = x.data();
    Geometry g2;
    if (!make_geometry(c, ops, &g2, &err)) return 1;
    for (size_t i = 0; i < g.metric.size(); ++i)
      if (std::fabs(g.metric[i] - g2.metric[i]) > 1e-12 * (1.0 + std::fabs(g.metric[i]))) return 1;
  }
  for (double v : g.metric)
    if (!std::isfinite(v)) return 1;
  return 0;
}

int main() {
  int bad = 0;
  std::string err;
  for (int p = 1; p <= kMaxN - 1; ++p) {
    Operators a, b;
    bad |= !make_operators(p, &a, &err);
    bad |= !make_gauss_operators(p, &b, &err);
    double s = 0.0;
    for (int i = 0; i <= p; ++i) s += a.w[i] + b.w[i];
    bad |= !(std::fabs(s - 4.0) < 1e-13);
  }
  Operators bad_ops;
  bad |= make_operators(kMaxN, &bad_ops, &err);  // out of range: must fail
  bad |= mesh(2, 3, 3, 0.0, false);
  bad |= mesh(2, 4, 2, 0.1, true);
  bad |= mesh(3, 3, 2, 0.1, true);
  bad |= mesh(3, 7, 1, 0.1, false);
  bad |= mesh(3, 2, 1, 0.0, false);
  std::printf("%s\n", bad ? "host_ops sanitize FAIL" : "host_ops sanitize ok");
  return bad;
}
