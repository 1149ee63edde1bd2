// The library's geometric source of the momentum equations -- the
// metric-derivative rows of the geometry tables and their contraction with
// T^{kl} -- compiled for the host from the same source files as the GPU
// kernels, for a comparison with the oracle's connection form under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
//   source_host <in> <out>
// in:  int32 npoints, int32 kerr, float64 gam, a, hslope,
//      then per point float64 x1, x2, P[8]
// out: per point float64 S1, S2 (the x1 and x2 momentum sources)
#include <stdio.h>
#include <stdlib.h>
#include <vector>

#include "hip/hip_runtime.h"
#include "../../include/grmhd.h"
#include "../../paper_2408_01361_amd/csrc/geometry.hpp"
#include "../../paper_2408_01361_amd/csrc/physics.hpp"

using namespace grmhd;

static void need(bool ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "source_host: %s\n", what);
    exit(2);
  }
}

int main(int argc, char** argv) {
  need(argc == 3, "usage: source_host <in> <out>");
  FILE* f = fopen(argv[1], "rb");
  need(f != nullptr, "cannot open input");
  int hdr[2];
  double par[3];
  need(fread(hdr, sizeof(int), 2, f) == 2 && fread(par, sizeof(double), 3, f) == 3, "short header");
  const int n = hdr[0];
  need(n >= 0 && n < (1 << 24), "bad point count");
  const SpaceTime st{hdr[1], par[1], par[2]};
  std::vector<double> in((size_t)n * 10), out((size_t)n * 2);
  need(fread(in.data(), sizeof(double), in.size(), f) == in.size(), "short input");
  fclose(f);
  for (int q = 0; q < n; q++) {
    const double* c = &in[(size_t)q * 10];
    PointMetric<double> m;
    metric_point(st, c[0], c[1], m.gcov, m.gcon, m.gdet, m.alpha);
    double D[NDG];
    source_metric_point(st, c[0], c[1], D);
    for (int r = 0; r < NDG; r++)
      if (x2_offdiag(r % 10)) D[r] = 0.0;  // never read by the source, as in the kernels
    Fluid<double> fl;
    fluid_state(c + 2, m, fl);
    double S[2];
    metric_source(c + 2, fl, m, par[0], D, S);
    out[(size_t)q * 2] = S[0];
    out[(size_t)q * 2 + 1] = S[1];
  }
  FILE* o = fopen(argv[2], "wb");
  need(o != nullptr, "cannot open output");
  need(fwrite(out.data(), sizeof(double), out.size(), o) == out.size(), "short write");
  fclose(o);
  return 0;
}
