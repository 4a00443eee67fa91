// Writes the library's host-built metric array of a warped 3D box (the
// [E][Ja^1_1 .. Ja^3_3, 1/J][node] array the stage kernels read) to a file,
// so that a CPU test can compare it with the oracle's independent curl-form
// metrics.  Usage: geometry_dump p n0 n1 n2 warp out.bin
#include <cstdio>
#include <cstdlib>
#include <string>

#include "host_ops.hpp"

int main(int argc, char** argv) {
  if (argc != 7) {
    std::fprintf(stderr, "usage: %s p n0 n1 n2 warp out.bin\n", argv[0]);
    return 2;
  }
  esdg::Operators ops;
  std::string err;
  const int p = std::atoi(argv[1]);
  if (!esdg::make_operators(p, &ops, &err)) {
    std::fprintf(stderr, "operators: %s\n", err.c_str());
    return 1;
  }
  esdg::MeshSpec s;
  s.dim = 3;
  s.p = p;
  for (int j = 0; j < 3; ++j) s.n[j] = std::atoi(argv[2 + j]);
  s.warp = std::atof(argv[5]);
  esdg::Geometry g;
  if (!esdg::make_geometry(s, ops, &g, &err)) {
    std::fprintf(stderr, "geometry: %s\n", err.c_str());
    return 1;
  }
  FILE* f = std::fopen(argv[6], "wb");
  if (!f) return 1;
  const size_t n = g.metric.size();
  const bool ok = std::fwrite(g.metric.data(), sizeof(double), n, f) == n;
  return (std::fclose(f) == 0 && ok) ? 0 : 1;
}
