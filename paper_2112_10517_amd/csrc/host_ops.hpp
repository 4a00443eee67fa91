// Host-side operators and geometry of the library (FP64, built once per
// problem at esdg_init_mesh; not part of the timed right-hand side).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace esdg {

constexpr int kMaxN = 8;  // nodes per line: degree <= 7

// 1D Legendre-Gauss-Lobatto operators of degree p (Sec. 2, LGL-DGSEM example)
// and the flux-differencing operator D~ = 2D - M^-1 B of Sec. 2.1.
//
// Legendre-Gauss collocation (Sec. 6) uses the Gauss nodes and weights, D on
// them, the Lagrange basis at the element ends rL, rR (operator R) and, in the
// slot of D~, T = M^-1 (M D - (M D)^T): the volume block of the hybridised
// operator 2 Q_h scaled by M^-1 (zero diagonal), with the face coefficients
// cL = -rL / w and cR = rR / w (M^-1 R^T B).
struct Operators {
  int p = 0, N = 0;
  bool gauss = false;
  double x[kMaxN] = {}, w[kMaxN] = {};
  double D[kMaxN * kMaxN] = {};   // row-major D[i*N+j]
  double Dt[kMaxN * kMaxN] = {};  // LGL: D~; Gauss: T; exact zero diagonal
  double rL[kMaxN] = {}, rR[kMaxN] = {};  // Gauss: Lagrange basis at -1, +1
  double cL[kMaxN] = {}, cR[kMaxN] = {};  // Gauss: -rL/w, rR/w
};

bool make_operators(int p, Operators* ops, std::string* err);
bool make_gauss_operators(int p, Operators* ops, std::string* err);

// Mesh description as the library sees it (a copy of the ABI descriptor).
struct MeshSpec {
  int dim = 3, p = 3;
  int n[3] = {1, 1, 1};
  double lo[3] = {-1, -1, -1}, hi[3] = {1, 1, 1};
  double warp = 0.0;
  const double* coords = nullptr;  // caller's, only read during construction
};

// Geometry of a periodic structured box mesh.
//   coords : [E][dim][nn] node coordinates
//   metric : [E][dim*dim + 1][nn]  (Ja)^n_m at index n*dim+m, then 1/J
//   nface  : [dim][E][dim][nf] one contravariant normal per face node of the
//            face on the + side (direction n) of element e: the average of
//            (Ja)^n seen from both elements sharing it
//   affine : true for the undeformed uniform box (no per-node metrics are
//            needed: Ja^n/J = (2/h_n) e_n)
struct Geometry {
  int64_t E = 0;
  int nn = 0, nf = 0;
  bool affine = true;
  double inv_half_h[3] = {1, 1, 1};  // 2/h_n of the uniform box
  double J_affine = 1.0;
  std::vector<double> coords, metric, nface;
};

bool make_geometry(const MeshSpec& spec, const Operators& ops, Geometry* g, std::string* err);

}  // namespace esdg
