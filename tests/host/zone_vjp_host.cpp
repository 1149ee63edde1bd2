// The adjoint's reverse-mode zone terms (zone_vjp: geometric source through
// the connection, and conserved variables) against dual-number evaluations
// of the same terms, one seeded prim (or the adiabatic index) at a time,
// both compiled for the host from the library's source, under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
//   zone_vjp_host <in> <out>
// in:  int32 npoints, int32 kerr, int32 with_u, float64 a, hslope, then per
//      point float64 x1, x2, gam, q[8], Sb[4], Ub[8]
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
    fprintf(stderr, "zone_vjp_host: %s\n", what);
    exit(2);
  }
}

int main(int argc, char** argv) {
  need(argc == 3, "usage: zone_vjp_host <in> <out>");
  FILE* f = fopen(argv[1], "rb");
  need(f != nullptr, "cannot open input");
  int hdr[3];
  double par[2];
  need(fread(hdr, sizeof(int), 3, f) == 3 && fread(par, sizeof(double), 2, f) == 2, "short header");
  const int n = hdr[0];
  const bool with_u = hdr[2] != 0;
  need(n >= 0 && n < (1 << 24), "bad header");
  const SpaceTime st{hdr[1], par[0], par[1]};
  std::vector<double> in((size_t)n * 23), out((size_t)n * 27);
  need(fread(in.data(), sizeof(double), in.size(), f) == in.size(), "short input");
  fclose(f);
  for (int k = 0; k < n; k++) {
    const double* c = &in[(size_t)k * 23];
    PointMetric<double> m;
    metric_point(st, c[0], c[1], m.gcov, m.gcon, m.gdet, m.alpha);
    double cn[40];
    connection_point(st, c[0], c[1], cn);
    const double gam = c[2];
    const double* q = c + 3;
    const double* Sb = c + 11;
    const double* Ub = c + 15;
    double* o = &out[(size_t)k * 27];
    zone_vjp(q, m, gam, cn, Sb, with_u ? Ub : nullptr, o, o[8]);
    for (int s = 0; s <= NVAR; s++) {
      Dual p[NVAR];
      for (int v = 0; v < NVAR; v++) p[v] = Dual(q[v], v == s ? 1.0 : 0.0);
      const Dual gd(gam, s == NVAR ? 1.0 : 0.0);
      Fluid<Dual> fl;
      fluid_state(p, m, fl);
      double acc = 0.0, sc = 0.0;
      for (int nu = 0; nu < 4; nu++) {
        Dual sacc(0.0);
        for (int kk = 0; kk < 4; kk++) {
          Dual T[4];
          tmunu_row(p, fl, gd, kk, T);
          for (int l = 0; l < 4; l++) sacc = sacc + T[l] * cn[l * 10 + sidx(nu, kk)];
        }
        const double d = (m.gdet * sacc).d * Sb[nu];
        acc += d;
        sc += fabs(d);
      }
      if (with_u) {
        Dual U[NVAR];
        prim_to_flux(p, fl, m, gd, 0, U);
        for (int v = 0; v < NVAR; v++) {
          acc += U[v].d * Ub[v];
          sc += fabs(U[v].d * Ub[v]);
        }
      }
      o[9 + s] = acc;
      o[18 + s] = sc;
    }
  }
  FILE* o = fopen(argv[2], "wb");
  need(o != nullptr, "cannot open output");
  need(fwrite(out.data(), sizeof(double), out.size(), o) == out.size(), "short write");
  fclose(o);
  return 0;
}
