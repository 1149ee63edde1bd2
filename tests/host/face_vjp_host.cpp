// The adjoint's reverse-mode face state (state_vjp) against dual-number
// evaluations of the same state, one seeded prim (or the adiabatic index) at
// a time, both compiled for the host from the library's source, under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
//   face_vjp_host <in> <out>
// in:  int32 npoints, int32 kerr, int32 dir, float64 a, hslope, then per
//      point float64 x1, x2, gam, q[8], Fb[8], Ub[8], cpb, cmb
// out: per point float64 reverse qb[8], gamb, then dual qb[8], gamb, then the
//      scale sum of |terms| of each of the nine dual products
#include <stdio.h>
#include <stdlib.h>
#include <math.h>
#include <vector>

#include "hip/hip_runtime.h"
#include "../../include/grmhd.h"
#include "../../paper_2408_01361_amd/csrc/geometry.hpp"
#include "../../paper_2408_01361_amd/csrc/physics.hpp"

using namespace grmhd;

#include "../../paper_2408_01361_amd/csrc/face_vjp.hpp"

static void need(bool ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "face_vjp_host: %s\n", what);
    exit(2);
  }
}

template <int D>
static void one(const double* c, const PointMetric<double>& m, double* out) {
  const double gam = c[2];
  const double* q = c + 3;
  const double* Fb = c + 11;
  const double* Ub = c + 19;
  const double cpb = c[27], cmb = c[28];
  state_vjp<D>(q, m, gam, Fb, Ub, cpb, cmb, out, out[8]);
  for (int s = 0; s <= NVAR; s++) {
    Dual p[NVAR];
    for (int v = 0; v < NVAR; v++) p[v] = Dual(q[v], v == s ? 1.0 : 0.0);
    const Dual gd(gam, s == NVAR ? 1.0 : 0.0);
    Fluid<Dual> f;
    fluid_state(p, m, f);
    Dual F[NVAR], U[NVAR], cp, cm;
    prim_to_flux(p, f, m, gd, D, F);
    prim_to_flux(p, f, m, gd, 0, U);
    char_speeds(p, f, m, gd, D, cp, cm);
    double acc = cpb * cp.d + cmb * cm.d, sc = fabs(cpb * cp.d) + fabs(cmb * cm.d);
    for (int v = 0; v < NVAR; v++) {
      acc += Fb[v] * F[v].d + Ub[v] * U[v].d;
      sc += fabs(Fb[v] * F[v].d) + fabs(Ub[v] * U[v].d);
    }
    out[9 + s] = acc;
    out[18 + s] = sc;
  }
}

int main(int argc, char** argv) {
  need(argc == 3, "usage: face_vjp_host <in> <out>");
  FILE* f = fopen(argv[1], "rb");
  need(f != nullptr, "cannot open input");
  int hdr[3];
  double par[2];
  need(fread(hdr, sizeof(int), 3, f) == 3 && fread(par, sizeof(double), 2, f) == 2, "short header");
  const int n = hdr[0], dir = hdr[2];
  need(n >= 0 && n < (1 << 24) && dir >= 1 && dir <= 3, "bad header");
  const SpaceTime st{hdr[1], par[0], par[1]};
  std::vector<double> in((size_t)n * 29), out((size_t)n * 27);
  need(fread(in.data(), sizeof(double), in.size(), f) == in.size(), "short input");
  fclose(f);
  for (int k = 0; k < n; k++) {
    const double* c = &in[(size_t)k * 29];
    PointMetric<double> m;
    metric_point(st, c[0], c[1], m.gcov, m.gcon, m.gdet, m.alpha);
    double* o = &out[(size_t)k * 27];
    if (dir == 1) one<1>(c, m, o);
    else if (dir == 2) one<2>(c, m, o);
    else one<3>(c, m, o);
  }
  FILE* o = fopen(argv[2], "wb");
  need(o != nullptr, "cannot open output");
  need(fwrite(out.data(), sizeof(double), out.size(), o) == out.size(), "short write");
  fclose(o);
  return 0;
}
