// Host-side LGL operators and mesh geometry (built once per problem).
#include "host_ops.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

namespace esdg {

namespace {

// Legendre P_p(x) by the three-term recurrence.
long double legendre_p(int p, long double x) {
  long double a = 1.0L, b = x;
  if (p == 0) return a;
  for (int k = 1; k < p; ++k) {
    long double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
    a = b;
    b = c;
  }
  return b;
}

// d/dx P_p and d2/dx2 P_p from the Legendre ODE:
// (1-x^2) P'' = 2x P' - p(p+1) P and P' = p (x P_p - P_{p-1}) / (x^2 - 1).
void legendre_derivs(int p, long double x, long double* d1, long double* d2) {
  long double pp = legendre_p(p, x), pm = legendre_p(p - 1, x);
  long double q = x * x - 1.0L;
  *d1 = p * (x * pp - pm) / q;
  *d2 = (2.0L * x * (*d1) - p * (p + 1.0L) * pp) / (1.0L - x * x);
}

// Number of eigenvalues below s of the symmetric tridiagonal matrix with zero
// diagonal and off-diagonal e[0..m-2] (Sturm sequence count).
int sturm_count(const long double* e, int m, long double s) {
  int cnt = 0;
  long double q = -s;
  if (q < 0) ++cnt;
  for (int i = 1; i < m; ++i) {
    long double prev = (q == 0.0L) ? 1e-300L : q;
    q = -s - e[i - 1] * e[i - 1] / prev;
    if (q < 0) ++cnt;
  }
  return cnt;
}

}  // namespace

bool make_operators(int p, Operators* ops, std::string* err) {
  if (p < 1 || p + 1 > kMaxN) {
    *err = "polynomial degree must be in [1, 7]";
    return false;
  }
  const int N = p + 1;
  long double x[kMaxN];
  x[0] = -1.0L;
  x[p] = 1.0L;
  // Interior LGL nodes = roots of P'_p, i.e. of the Gegenbauer polynomial
  // C^(3/2)_{p-1}: eigenvalues of its Jacobi matrix (zero diagonal,
  // off-diagonal sqrt(k(k+2)/((2k+1)(2k+3)))), located by bisection on the
  // Sturm count and polished by Newton on P'_p.
  const int m = p - 1;
  long double e[kMaxN];
  for (int k = 1; k < m; ++k) e[k - 1] = sqrtl((long double)k * (k + 2) / ((2.0L * k + 1) * (2.0L * k + 3)));
  for (int r = 0; r < m; ++r) {
    long double a = -1.0L, b = 1.0L;
    for (int it = 0; it < 200 && b - a > 1e-19L; ++it) {
      long double c = 0.5L * (a + b);
      if (sturm_count(e, m, c) > r) b = c; else a = c;
    }
    long double t = 0.5L * (a + b);
    for (int it = 0; it < 3; ++it) {
      long double d1, d2;
      legendre_derivs(p, t, &d1, &d2);
      if (d2 != 0.0L) t -= d1 / d2;
    }
    x[r + 1] = t;
  }
  // exact mirror symmetry of the node set
  for (int i = 0; i < N / 2; ++i) {
    long double h = 0.5L * (x[p - i] - x[i]);
    x[i] = -h;
    x[p - i] = h;
  }
  if (N % 2) x[p / 2] = 0.0L;

  // quadrature weights 2 / (p(p+1) P_p(x_i)^2) and barycentric weights
  long double bw[kMaxN];
  for (int i = 0; i < N; ++i) {
    long double P = legendre_p(p, x[i]);
    ops->x[i] = (double)x[i];
    ops->w[i] = (double)(2.0L / ((long double)p * (p + 1) * P * P));
    long double prod = 1.0L;
    for (int j = 0; j < N; ++j)
      if (j != i) prod *= (x[i] - x[j]);
    bw[i] = 1.0L / prod;
  }
  // Lagrange differentiation matrix in barycentric form; the diagonal is the
  // negative row sum so that D annihilates constants.
  for (int i = 0; i < N; ++i) {
    long double diag = 0.0L;
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      long double v = (bw[j] / bw[i]) / (x[i] - x[j]);
      ops->D[i * N + j] = (double)v;
      diag -= v;
    }
    ops->D[i * N + i] = (double)diag;
  }
  // D~ = 2D - M^-1 B with B = diag(-1, 0, ..., 0, 1); its diagonal vanishes
  // (skew-symmetry of M D~, Sec. 2.2) and is set to exactly zero.
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) ops->Dt[i * N + j] = (i == j) ? 0.0 : 2.0 * ops->D[i * N + j];
  ops->p = p;
  ops->N = N;
  return true;
}

bool make_gauss_operators(int p, Operators* ops, std::string* err) {
  if (p < 1 || p + 1 > kMaxN) {
    *err = "polynomial degree must be in [1, 7]";
    return false;
  }
  const int N = p + 1;
  // Gauss nodes = roots of P_N: eigenvalues of the Jacobi matrix of the
  // Legendre recurrence (zero diagonal, off-diagonal k/sqrt(4k^2-1)), by
  // bisection on the Sturm count, polished by Newton on P_N.
  long double e[kMaxN];
  for (int k = 1; k < N; ++k) e[k - 1] = (long double)k / sqrtl(4.0L * k * k - 1.0L);
  long double x[kMaxN];
  for (int r = 0; r < N; ++r) {
    long double a = -1.0L, b = 1.0L;
    for (int it = 0; it < 200 && b - a > 1e-19L; ++it) {
      long double c = 0.5L * (a + b);
      if (sturm_count(e, N, c) > r) b = c; else a = c;
    }
    long double t = 0.5L * (a + b);
    for (int it = 0; it < 3; ++it) {
      long double d1, d2;
      legendre_derivs(N, t, &d1, &d2);
      const long double P = legendre_p(N, t);
      if (d1 != 0.0L) t -= P / d1;
    }
    x[r] = t;
  }
  for (int i = 0; i < N / 2; ++i) {
    long double h = 0.5L * (x[N - 1 - i] - x[i]);
    x[i] = -h;
    x[N - 1 - i] = h;
  }
  if (N % 2) x[N / 2] = 0.0L;
  long double bw[kMaxN], wl[kMaxN];
  for (int i = 0; i < N; ++i) {
    long double d1, d2;
    legendre_derivs(N, x[i], &d1, &d2);
    wl[i] = 2.0L / ((1.0L - x[i] * x[i]) * d1 * d1);
    ops->x[i] = (double)x[i];
    ops->w[i] = (double)wl[i];
    long double prod = 1.0L;
    for (int j = 0; j < N; ++j)
      if (j != i) prod *= (x[i] - x[j]);
    bw[i] = 1.0L / prod;
  }
  long double Dl[kMaxN * kMaxN];
  for (int i = 0; i < N; ++i) {
    long double diag = 0.0L;
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      const long double v = (bw[j] / bw[i]) / (x[i] - x[j]);
      Dl[i * N + j] = v;
      diag -= v;
    }
    Dl[i * N + i] = diag;
  }
  // Lagrange basis at the ends, barycentric form l_k(s) = (bw_k/(s-x_k)) / sum_j bw_j/(s-x_j)
  for (int side = 0; side < 2; ++side) {
    const long double s = side ? 1.0L : -1.0L;
    long double den = 0.0L;
    for (int j = 0; j < N; ++j) den += bw[j] / (s - x[j]);
    for (int k = 0; k < N; ++k) (side ? ops->rR : ops->rL)[k] = (double)((bw[k] / (s - x[k])) / den);
  }
  // T = M^-1 (M D - (M D)^T) with an exact zero diagonal; M^-1 R^T B
  for (int i = 0; i < N; ++i) {
    for (int k = 0; k < N; ++k) {
      ops->D[i * N + k] = (double)Dl[i * N + k];
      ops->Dt[i * N + k] = i == k ? 0.0 : (double)((wl[i] * Dl[i * N + k] - wl[k] * Dl[k * N + i]) / wl[i]);
    }
    ops->cL[i] = (double)(-(long double)ops->rL[i] / wl[i]);
    ops->cR[i] = (double)((long double)ops->rR[i] / wl[i]);
  }
  ops->p = p;
  ops->N = N;
  ops->gauss = true;
  return true;
}

namespace {

inline int ipow(int b, int k) {
  int r = 1;
  while (k-- > 0) r *= b;
  return r;
}

// fn(begin, end) over [0, n) split across the host's threads
template <typename Fn>
void parallel_for(int64_t n, Fn fn) {
  const int64_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int64_t nt = std::min<int64_t>(hw, std::max<int64_t>(1, n / 64));
  if (nt <= 1) {
    fn(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve((size_t)nt);
  int64_t t = 0;
  try {
    for (; t < nt; ++t) th.emplace_back(fn, n * t / nt, n * (t + 1) / nt);
  } catch (...) {
    // a thread could not be started: the remaining ranges run here
    for (int64_t r = t; r < nt; ++r) fn(n * r / nt, n * (r + 1) / nt);
  }
  for (auto& x : th) x.join();
}

// b = D_dir a over one element's nodal field (x-fastest tensor layout)
void apply_d(const Operators& ops, int dim, int dir, const double* a, double* b) {
  const int N = ops.N, nn = ipow(N, dim);
  const int stride = ipow(N, dir);
  for (int q = 0; q < nn; ++q) {
    const int id = (q / stride) % N;
    const int base = q - id * stride;
    double s = 0.0;
    for (int k = 0; k < N; ++k) s += ops.D[id * N + k] * a[base + k * stride];
    b[q] = s;
  }
}

}  // namespace

bool make_geometry(const MeshSpec& s, const Operators& ops, Geometry* g, std::string* err) {
  const int dim = s.dim, N = ops.N;
  if (dim != 2 && dim != 3) {
    *err = "dim must be 2 or 3";
    return false;
  }
  int n[3] = {s.n[0], s.n[1], dim == 3 ? s.n[2] : 1};
  for (int j = 0; j < dim; ++j) {
    if (n[j] < 1) {
      *err = "element counts must be >= 1";
      return false;
    }
    if (!(s.hi[j] > s.lo[j])) {
      *err = "box must satisfy hi > lo";
      return false;
    }
  }
  const int nn = ipow(N, dim), nf = ipow(N, dim - 1);
  const int64_t E = (int64_t)n[0] * n[1] * n[2];
  g->E = E;
  g->nn = nn;
  g->nf = nf;
  g->affine = (s.warp == 0.0 && s.coords == nullptr);
  double h[3];
  g->J_affine = 1.0;
  for (int j = 0; j < dim; ++j) {
    h[j] = (s.hi[j] - s.lo[j]) / n[j];
    g->inv_half_h[j] = 2.0 / h[j];
    g->J_affine *= 0.5 * h[j];
  }

  // node coordinates
  g->coords.assign((size_t)E * dim * nn, 0.0);
  if (s.coords) {
    std::memcpy(g->coords.data(), s.coords, sizeof(double) * g->coords.size());
  } else {
    parallel_for(E, [&](int64_t eb, int64_t ee_) {
    for (int64_t e = eb; e < ee_; ++e) {
      const int64_t ie[3] = {e % n[0], (e / n[0]) % n[1], e / ((int64_t)n[0] * n[1])};
      for (int q = 0; q < nn; ++q) {
        double xh[3], bump = 1.0;
        for (int j = 0; j < dim; ++j) {
          const int id = (q / ipow(N, j)) % N;
          xh[j] = s.lo[j] + h[j] * ((double)ie[j] + 0.5 * (ops.x[id] + 1.0));
          const double sj = 2.0 * (xh[j] - s.lo[j]) / (s.hi[j] - s.lo[j]) - 1.0;
          bump *= std::sin(M_PI * sj);
        }
        for (int j = 0; j < dim; ++j) g->coords[((size_t)e * dim + j) * nn + q] = xh[j] + s.warp * bump;
      }
    }
    });
  }
  if (g->affine) return true;

  // metric terms per node: 2D cross-product form, 3D conservative curl form
  const int nm = dim * dim + 1;
  g->metric.assign((size_t)E * nm * nn, 0.0);
  std::atomic<bool> positive{true};
  parallel_for(E, [&](int64_t eb, int64_t ee_) {
  std::vector<double> X(3 * nn), dX(9 * nn), t(nn), t2(nn), r1(nn), r2(nn);
  for (int64_t e = eb; e < ee_; ++e) {
    for (int m = 0; m < dim; ++m) {
      const double* xs = &g->coords[((size_t)e * dim + m) * nn];
      double mean = 0.0;
      for (int q = 0; q < nn; ++q) mean += xs[q];
      mean /= nn;  // the metric terms are invariant under a constant shift
      for (int q = 0; q < nn; ++q) X[m * nn + q] = xs[q] - mean;
    }
    for (int j = 0; j < dim; ++j)
      for (int m = 0; m < dim; ++m) apply_d(ops, dim, j, &X[m * nn], &dX[(j * 3 + m) * nn]);
    double* Me = &g->metric[(size_t)e * nm * nn];
    auto Ja = [&](int a, int m) { return Me + (a * dim + m) * nn; };
    if (dim == 2) {
      for (int q = 0; q < nn; ++q) {
        Ja(0, 0)[q] = dX[(1 * 3 + 1) * nn + q];
        Ja(0, 1)[q] = -dX[(1 * 3 + 0) * nn + q];
        Ja(1, 0)[q] = -dX[(0 * 3 + 1) * nn + q];
        Ja(1, 1)[q] = dX[(0 * 3 + 0) * nn + q];
      }
    } else {
      for (int a = 0; a < 3; ++a) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
        for (int c = 0; c < 3; ++c) {
          const int cm = (c + 1) % 3, cl = (c + 2) % 3;
          for (int q = 0; q < nn; ++q) {
            t[q] = X[cl * nn + q] * dX[(a1 * 3 + cm) * nn + q];
            t2[q] = X[cl * nn + q] * dX[(a2 * 3 + cm) * nn + q];
          }
          apply_d(ops, dim, a2, t.data(), r1.data());
          apply_d(ops, dim, a1, t2.data(), r2.data());
          double* out = Ja(a, c);
          for (int q = 0; q < nn; ++q) out[q] = r1[q] - r2[q];
        }
      }
    }
    double* invJ = Me + dim * dim * nn;
    for (int q = 0; q < nn; ++q) {
      double J;
      auto d = [&](int j, int m) { return dX[(j * 3 + m) * nn + q]; };  // d x_m / d xi_j
      if (dim == 2) {
        J = d(0, 0) * d(1, 1) - d(1, 0) * d(0, 1);
      } else {
        J = d(0, 0) * (d(1, 1) * d(2, 2) - d(2, 1) * d(1, 2)) -
            d(1, 0) * (d(0, 1) * d(2, 2) - d(2, 1) * d(0, 2)) +
            d(2, 0) * (d(0, 1) * d(1, 2) - d(1, 1) * d(0, 2));
      }
      if (!(J > 0.0)) positive.store(false, std::memory_order_relaxed);
      invJ[q] = 1.0 / J;
    }
  }
  });
  if (!positive.load()) {
    *err = "mesh has a non-positive Jacobian";
    return false;
  }

  // one normal per face node: average of both sides' (Ja)^a
  g->nface.assign((size_t)dim * E * dim * nf, 0.0);
  for (int a = 0; a < dim; ++a) {
    const int sa = ipow(N, a);
    parallel_for(E, [&](int64_t eb, int64_t ee_) {
    for (int64_t e = eb; e < ee_; ++e) {
      int64_t ie[3] = {e % n[0], (e / n[0]) % n[1], e / ((int64_t)n[0] * n[1])};
      ie[a] = (ie[a] + 1) % n[a];
      const int64_t eR = ie[0] + (int64_t)n[0] * (ie[1] + (int64_t)n[1] * ie[2]);
      for (int f = 0; f < nf; ++f) {
        // face node f enumerates the other directions, lowest first
        const int lo_part = f % sa, hi_part = f / sa;
        const int qL = lo_part + (N - 1) * sa + hi_part * sa * N;
        const int qR = lo_part + hi_part * sa * N;
        for (int m = 0; m < dim; ++m) {
          const double vL = g->metric[((size_t)e * nm + a * dim + m) * nn + qL];
          const double vR = g->metric[((size_t)eR * nm + a * dim + m) * nn + qR];
          g->nface[(((size_t)a * E + e) * dim + m) * nf + f] = 0.5 * (vL + vR);
        }
      }
    }
    });
  }
  return true;
}

}  // namespace esdg
