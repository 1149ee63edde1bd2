// Geometry of the stationary spacetimes on the device: the metric, its
// inverse and sqrt(-g) at any (x1, x2), and the connection
// Gamma^l_{mn} = g^{lk} Gamma_{kmn}, Gamma_{kmn} = (d_m g_kn + d_n g_km - d_k g_mn)/2.
//
// Metric derivatives come from forward-mode dual numbers carried through the
// closed-form Kerr-Schild metric and the modified-KS coordinate map, so no
// derivative is written by hand and none is approximated by differences.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "physics.hpp"

namespace grmhd {

// Value and derivatives with respect to x1 and x2.
struct Dual2 {
  double v, d1, d2;
};
__device__ __forceinline__ Dual2 dconst(double c) { return {c, 0.0, 0.0}; }
__device__ __forceinline__ Dual2 operator+(Dual2 a, Dual2 b) { return {a.v + b.v, a.d1 + b.d1, a.d2 + b.d2}; }
__device__ __forceinline__ Dual2 operator-(Dual2 a, Dual2 b) { return {a.v - b.v, a.d1 - b.d1, a.d2 - b.d2}; }
__device__ __forceinline__ Dual2 operator-(Dual2 a) { return {-a.v, -a.d1, -a.d2}; }
__device__ __forceinline__ Dual2 operator*(Dual2 a, Dual2 b) {
  return {a.v * b.v, a.d1 * b.v + a.v * b.d1, a.d2 * b.v + a.v * b.d2};
}
__device__ __forceinline__ Dual2 operator*(double c, Dual2 a) { return {c * a.v, c * a.d1, c * a.d2}; }
__device__ __forceinline__ Dual2 operator/(Dual2 a, Dual2 b) {
  double q = a.v / b.v;
  return {q, (a.d1 - q * b.d1) / b.v, (a.d2 - q * b.d2) / b.v};
}
__device__ __forceinline__ Dual2 dsin(Dual2 a) {
  double s = sin(a.v), c = cos(a.v);
  return {s, c * a.d1, c * a.d2};
}
__device__ __forceinline__ Dual2 dcos(Dual2 a) {
  double s = sin(a.v), c = cos(a.v);
  return {c, -s * a.d1, -s * a.d2};
}
__device__ __forceinline__ Dual2 dexp(Dual2 a) {
  double e = exp(a.v);
  return {e, e * a.d1, e * a.d2};
}

struct SpaceTime {
  int kerr;      // 0: Minkowski Cartesian, 1: Kerr in modified KS
  double a, h;   // spin, theta squeeze
};

// Covariant metric (10 symmetric entries) with first derivatives, at (x1, x2).
__device__ __forceinline__ void metric_cov_dual(const SpaceTime& st, double x1, double x2, Dual2 g[10]) {
  for (int q = 0; q < 10; q++) g[q] = dconst(0.0);
  if (!st.kerr) {
    g[sidx(0, 0)] = dconst(-1.0);
    g[sidx(1, 1)] = g[sidx(2, 2)] = g[sidx(3, 3)] = dconst(1.0);
    return;
  }
  const double a = st.a;
  Dual2 X1 = {x1, 1.0, 0.0}, X2 = {x2, 0.0, 1.0};
  const double tp = 2.0 * M_PI;
  Dual2 r = dexp(X1);
  Dual2 th = M_PI * X2 + (0.5 * (1.0 - st.h)) * dsin(tp * X2);
  Dual2 dth = M_PI * (dconst(1.0) + (1.0 - st.h) * dcos(tp * X2));
  Dual2 s = dsin(th), c = dcos(th);
  Dual2 s2 = s * s;
  Dual2 sig = r * r + (a * a) * (c * c);
  Dual2 z = 2.0 * r / sig;
  Dual2 one = dconst(1.0);
  // Kerr-Schild (t, r, theta, phi), then the diagonal coordinate Jacobian
  // L = (1, dr/dx1 = r, dtheta/dx2, 1): g_mn -> L_m L_n g_mn.
  Dual2 gks[10];
  for (int q = 0; q < 10; q++) gks[q] = dconst(0.0);
  gks[sidx(0, 0)] = z - one;
  gks[sidx(0, 1)] = z;
  gks[sidx(0, 3)] = -a * (z * s2);
  gks[sidx(1, 1)] = one + z;
  gks[sidx(1, 3)] = -a * (s2 * (one + z));
  gks[sidx(2, 2)] = sig;
  gks[sidx(3, 3)] = s2 * (sig + (a * a) * (s2 * (one + z)));
  Dual2 L[4] = {one, r, dth, one};
  for (int m = 0; m < 4; m++)
    for (int n = m; n < 4; n++) g[sidx(m, n)] = gks[sidx(m, n)] * (L[m] * L[n]);
}

// Metric, inverse, sqrt(-g) and lapse at (x1, x2) as doubles.  The inverse is
// the closed-form Kerr-Schild inverse divided by L_m L_n; sqrt(-g) takes
// |sin theta| so that positions continued past a pole stay finite.
__device__ __forceinline__ void metric_point(const SpaceTime& st, double x1, double x2, double gcov[10],
                                    double gcon[10], double& gdet, double& alpha) {
  for (int q = 0; q < 10; q++) gcov[q] = gcon[q] = 0.0;
  if (!st.kerr) {
    gcov[sidx(0, 0)] = gcon[sidx(0, 0)] = -1.0;
    for (int i = 1; i < 4; i++) gcov[sidx(i, i)] = gcon[sidx(i, i)] = 1.0;
    gdet = 1.0;
    alpha = 1.0;
    return;
  }
  Dual2 gd[10];
  metric_cov_dual(st, x1, x2, gd);
  for (int q = 0; q < 10; q++) gcov[q] = gd[q].v;
  const double a = st.a;
  double r = exp(x1);
  double th = M_PI * x2 + 0.5 * (1.0 - st.h) * sin(2.0 * M_PI * x2);
  double dth = M_PI * (1.0 + (1.0 - st.h) * cos(2.0 * M_PI * x2));
  double s = sin(th), c = cos(th);
  double sig = r * r + a * a * c * c;
  double z = 2.0 * r / sig;
  double del = r * r - 2.0 * r + a * a;
  double L[4] = {1.0, r, dth, 1.0};
  double ks[10];
  for (int q = 0; q < 10; q++) ks[q] = 0.0;
  ks[sidx(0, 0)] = -(1.0 + z);
  ks[sidx(0, 1)] = z;
  ks[sidx(1, 1)] = del / sig;
  ks[sidx(1, 3)] = a / sig;
  ks[sidx(2, 2)] = 1.0 / sig;
  ks[sidx(3, 3)] = 1.0 / (sig * s * s);
  for (int m = 0; m < 4; m++)
    for (int n = m; n < 4; n++) gcon[sidx(m, n)] = ks[sidx(m, n)] / (L[m] * L[n]);
  gdet = sig * fabs(s) * r * dth;
  alpha = 1.0 / sqrt(-gcon[0]);
}

// Connection at (x1, x2), stored as Gamma^l_{mn} for m <= n: index l*10 + sidx(m, n).
__device__ __forceinline__ void connection_point(const SpaceTime& st, double x1, double x2, double conn[40]) {
  for (int q = 0; q < 40; q++) conn[q] = 0.0;
  if (!st.kerr) return;
  Dual2 gd[10];
  metric_cov_dual(st, x1, x2, gd);
  double gcov[10], gcon[10], gdet, alpha;
  metric_point(st, x1, x2, gcov, gcon, gdet, alpha);
  // dg(k, m, n) = d g_mn / d x^k, nonzero for k = 1, 2 only
  auto dg = [&](int k, int m, int n) -> double {
    const Dual2& e = gd[sidx(m, n)];
    return k == 1 ? e.d1 : (k == 2 ? e.d2 : 0.0);
  };
  for (int m = 0; m < 4; m++)
    for (int n = m; n < 4; n++) {
      double low[4];
      for (int k = 0; k < 4; k++) low[k] = 0.5 * (dg(m, k, n) + dg(n, k, m) - dg(k, m, n));
      for (int l = 0; l < 4; l++) {
        double s = 0.0;
        for (int k = 0; k < 4; k++) s += gcon[sidx(l, k)] * low[k];
        conn[l * 10 + sidx(m, n)] = s;
      }
    }
}

// Metric-derivative rows of the geometric source at (x1, x2) (layout NDG):
// D[(nu - 1) * 10 + s] = d_nu g_s / 2 on the diagonal, d_nu g_s off it.
__device__ __forceinline__ void source_metric_point(const SpaceTime& st, double x1, double x2, double D[NDG]) {
  Dual2 gd[10];
  metric_cov_dual(st, x1, x2, gd);
  for (int a = 0; a < 4; a++)
    for (int b = a; b < 4; b++) {
      const int q = sidx(a, b);
      const double f = a == b ? 0.5 : 1.0;
      D[q] = f * gd[q].d1;
      D[10 + q] = f * gd[q].d2;
    }
}

}  // namespace grmhd
