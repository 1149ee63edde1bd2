// The library's primitive-variable recoveries (1D_W, Kastaun, the implicit
// solver's Newton-Raphson with its LDS-layout Jacobian) and its zone-centre
// metric, compiled for the host from the same source files as the GPU
// kernels, for runs under AddressSanitizer and UndefinedBehaviorSanitizer,
// and under MemorySanitizer.
//
//   inversion_host <in> <out>
// in:  int32 ncases, int32 inverter (0 1D_W, 1 Kastaun, 2 implicit),
//      int32 kerr, int32 maxit, float64 gam, tol, vmax2, a, hslope,
//      then per case float64 x1, x2, U[8], guess[8]
// out: per case float64 P[8], then int32 failure flags
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

#include "hip/hip_runtime.h"
#include "../../include/grmhd.h"
#include "../../paper_2408_01361_amd/csrc/geometry.hpp"
#include "../../paper_2408_01361_amd/csrc/physics.hpp"

using namespace grmhd;

namespace {

constexpr int BLOCK = 256;  // the Jacobian's LDS stride, as on the GPU

// The fields of the kernels' grid description that the recoveries read.
struct Dev {
  double gam, tol;
  int maxit;
  int inverter;
  double vmax2;
  int floors;
};

#include "../../paper_2408_01361_amd/csrc/inversion.hpp"

}  // namespace

static void need(bool ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "inversion_host: %s\n", what);
    exit(2);
  }
}

int main(int argc, char** argv) {
  need(argc == 3, "usage: inversion_host <in> <out>");
  FILE* f = fopen(argv[1], "rb");
  need(f != nullptr, "cannot open input");
  int hdr[4];
  double par[5];
  need(fread(hdr, sizeof(int), 4, f) == 4 && fread(par, sizeof(double), 5, f) == 5, "short header");
  const int n = hdr[0];
  need(n >= 0 && n < (1 << 24), "bad case count");
  Dev g{par[0], par[1], hdr[3], hdr[1], par[2], 0};
  const SpaceTime st{hdr[2], par[3], par[4]};
  std::vector<double> in((size_t)n * 18), out((size_t)n * 8);
  std::vector<int> flags(n);
  need(fread(in.data(), sizeof(double), in.size(), f) == in.size(), "short input");
  fclose(f);
  for (int q = 0; q < n; q++) {
    const double* c = &in[(size_t)q * 18];
    PointMetric<double> m;
    metric_point(st, c[0], c[1], m.gcov, m.gcon, m.gdet, m.alpha);
    double P[NVAR];
    if (g.inverter == GRMHD_INV_IMPLICIT) {
      // one thread's slots of a workgroup's Jacobian array (stride BLOCK),
      // freshly allocated and left uninitialised for every zone, so that a
      // read of a slot the solver has not written is seen (MemorySanitizer;
      // AddressSanitizer fills new blocks with garbage)
      double* jac = (double*)malloc(sizeof(double) * 25 * BLOCK);
      need(jac != nullptr, "out of memory");
      flags[q] = invert_implicit(g, m, c + 2, c + 10, P, jac + (q % BLOCK));
      free(jac);
    } else
      flags[q] = invert(g, m, c + 2, c + 10, P);
    memcpy(&out[(size_t)q * 8], P, sizeof(P));
  }
  FILE* o = fopen(argv[2], "wb");
  need(o != nullptr, "cannot open output");
  need(fwrite(out.data(), sizeof(double), out.size(), o) == out.size() &&
           fwrite(flags.data(), sizeof(int), flags.size(), o) == flags.size(),
       "short write");
  fclose(o);
  return 0;
}
