// The adjoint's closed-form WENO5 gradient against the dual-number WENO5
// (one seeded stencil slot at a time), both compiled for the host from the
// library's source, for a comparison under AddressSanitizer and
// UndefinedBehaviorSanitizer.
//
//   weno_grad_host <in> <out>
// in:  int32 ncases, float64 eps, then per case float64 x[5]
// out: per case float64 closed-form gradient[5], then dual gradient[5]
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
  std::vector<double> in((size_t)n * 5), out((size_t)n * 10);
  need(fread(in.data(), sizeof(double), in.size(), f) == in.size(), "short input");
  fclose(f);
  for (int q = 0; q < n; q++) {
    const double* x = &in[(size_t)q * 5];
    double* g = &out[(size_t)q * 10];
    weno5_grad(x[0], x[1], x[2], x[3], x[4], eps, g[0], g[1], g[2], g[3], g[4]);
    for (int s = 0; s < 5; s++) {
      Dual d[5];
      for (int z = 0; z < 5; z++) d[z] = Dual(x[z], z == s ? 1.0 : 0.0);
      out[(size_t)q * 10 + 5 + s] = weno5(d[0], d[1], d[2], d[3], d[4], Dual(eps)).d;
    }
  }
  FILE* o = fopen(argv[2], "wb");
  need(o != nullptr, "cannot open output");
  need(fwrite(out.data(), sizeof(double), out.size(), o) == out.size(), "short write");
  fclose(o);
  return 0;
}
