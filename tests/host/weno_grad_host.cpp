// The adjoint's closed-form reconstruction gradients -- WENO5 and the MC
// edge values -- against dual-number evaluations (one seeded stencil slot at
// a time), all compiled for the host from the library's source, for a
// comparison under AddressSanitizer and UndefinedBehaviorSanitizer.
//
//   weno_grad_host <in> <out>
// in:  int32 ncases, float64 eps, then per case float64 x[5]
// out: per case float64 closed-form WENO5 gradient[5], dual gradient[5],
//      closed-form gradients of mc_left(x0, x1, x2) and mc_right(x1, x2, x3)
//      [3 + 3], then their dual gradients [3 + 3]
#include <stdio.h>
#include <stdlib.h>
#include <vector>

#include "hip/hip_runtime.h"
#include "../../include/grmhd.h"
#include "../../paper_2408_01361_amd/csrc/physics.hpp"

using namespace grmhd;

static void need(bool ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "weno_grad_host: %s\n", what);
    exit(2);
  }
}

int main(int argc, char** argv) {
  need(argc == 3, "usage: weno_grad_host <in> <out>");
  FILE* f = fopen(argv[1], "rb");
  need(f != nullptr, "cannot open input");
  int n;
  double eps;
  need(fread(&n, sizeof(int), 1, f) == 1 && fread(&eps, sizeof(double), 1, f) == 1, "short header");
  need(n >= 0 && n < (1 << 24), "bad case count");
  std::vector<double> in((size_t)n * 5), out((size_t)n * 22);
  need(fread(in.data(), sizeof(double), in.size(), f) == in.size(), "short input");
  fclose(f);
  for (int q = 0; q < n; q++) {
    const double* x = &in[(size_t)q * 5];
    double* g = &out[(size_t)q * 22];
    weno5_grad(x[0], x[1], x[2], x[3], x[4], eps, g[0], g[1], g[2], g[3], g[4]);
    for (int s = 0; s < 5; s++) {
      Dual d[5];
      for (int z = 0; z < 5; z++) d[z] = Dual(x[z], z == s ? 1.0 : 0.0);
      g[5 + s] = weno5(d[0], d[1], d[2], d[3], d[4], Dual(eps)).d;
    }
    mc_left_grad(x[0], x[1], x[2], g[10], g[11], g[12]);
    mc_right_grad(x[1], x[2], x[3], g[13], g[14], g[15]);
    for (int s = 0; s < 3; s++) {
      Dual a[4];
      for (int z = 0; z < 4; z++) a[z] = Dual(x[z], z == s ? 1.0 : 0.0);
      g[16 + s] = mc_left(a[0], a[1], a[2]).d;
      Dual b[4];
      for (int z = 0; z < 4; z++) b[z] = Dual(x[z], z == s + 1 ? 1.0 : 0.0);
      g[19 + s] = mc_right(b[1], b[2], b[3]).d;
    }
  }
  FILE* o = fopen(argv[2], "wb");
  need(o != nullptr, "cannot open output");
  need(fwrite(out.data(), sizeof(double), out.size(), o) == out.size(), "short write");
  fclose(o);
  return 0;
}
