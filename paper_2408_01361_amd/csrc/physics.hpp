// Per-point HARM physics for gfx950, templated on the arithmetic type R
// (double for the FP64 path, float for the reduced-precision flux path).
//
//   * fluid four-vectors from the normal-observer velocity u~ (McKinney &
//     Gammie form the Algorithm section cites);
//   * rows of the ideal stress-energy tensor (EGRMHD section, ideal part);
//   * conserved variables / fluxes with the rest-mass energy removed;
//   * fast-magnetosonic characteristic speeds;
//   * linear-MC and WENO5 (Jiang-Shu weights) reconstruction.
#pragma once

#include <hip/hip_runtime.h>

namespace grmhd {

enum { RHO = 0, UU = 1, U1 = 2, U2 = 3, U3 = 4, B1 = 5, B2 = 6, B3 = 7, NVAR = 8 };

// Symmetric 4x4 stored as 10 values: tt t1 t2 t3 11 12 13 22 23 33.
__host__ __device__ constexpr int sidx(int m, int n) {
  return (m < n ? m : n) == 0   ? (m < n ? n : m)
         : (m < n ? m : n) == 1 ? 3 + (m < n ? n : m)
         : (m < n ? m : n) == 2 ? 5 + (m < n ? n : m)
                                : 9;
}

// Geometry at one point, in the arithmetic type of the caller.
template <typename R>
struct PointMetric {
  R gcov[10];
  R gcon[10];
  R gdet;
  R alpha;
};

// Layout of a per-location geometry table: field-major over the padded
// (x1, x2) plane, so consecutive x1 columns are consecutive addresses.
enum { G_COV = 0, G_CON = 10, G_DET = 20, G_ALPHA = 21, G_NF = 22 };
enum { NCONN = 40 };  // Gamma^l_{mn}, m <= n

template <typename R>
__device__ __forceinline__ void load_metric(const double* __restrict__ tab, long plane, long q,
                                   PointMetric<R>& m) {
#pragma unroll
  for (int f = 0; f < 10; f++) {
    m.gcov[f] = (R)tab[(G_COV + f) * plane + q];
    m.gcon[f] = (R)tab[(G_CON + f) * plane + q];
  }
  m.gdet = (R)tab[G_DET * plane + q];
  m.alpha = (R)tab[G_ALPHA * plane + q];
}

template <typename R>
struct Fluid {
  R ucon[4], ucov[4], bcon[4], bcov[4], bsq;
};

template <typename R>
__device__ __forceinline__ void lower4(const R v[4], const PointMetric<R>& m, R out[4]) {
#pragma unroll
  for (int a = 0; a < 4; a++)
    out[a] = m.gcov[sidx(a, 0)] * v[0] + m.gcov[sidx(a, 1)] * v[1] + m.gcov[sidx(a, 2)] * v[2] +
             m.gcov[sidx(a, 3)] * v[3];
}

// gamma = sqrt(1 + g_ij u~i u~j); u^t = gamma/alpha; u^i = u~i - gamma alpha g^{ti};
// b^t = B^i u_i; b^i = (B^i + b^t u^i)/u^t.
template <typename R>
__device__ __forceinline__ void fluid_state(const R p[NVAR], const PointMetric<R>& m, Fluid<R>& f) {
  const R v1 = p[U1], v2 = p[U2], v3 = p[U3];
  R qsq = m.gcov[sidx(1, 1)] * v1 * v1 + m.gcov[sidx(2, 2)] * v2 * v2 + m.gcov[sidx(3, 3)] * v3 * v3 +
          (R)2 * (m.gcov[sidx(1, 2)] * v1 * v2 + m.gcov[sidx(1, 3)] * v1 * v3 +
                  m.gcov[sidx(2, 3)] * v2 * v3);
  R gamma = sqrt((R)1 + qsq);
  R ga = gamma * m.alpha;
  f.ucon[0] = gamma / m.alpha;
  f.ucon[1] = v1 - ga * m.gcon[sidx(0, 1)];
  f.ucon[2] = v2 - ga * m.gcon[sidx(0, 2)];
  f.ucon[3] = v3 - ga * m.gcon[sidx(0, 3)];
  lower4(f.ucon, m, f.ucov);
  R bt = p[B1] * f.ucov[1] + p[B2] * f.ucov[2] + p[B3] * f.ucov[3];
  R iut = (R)1 / f.ucon[0];
  f.bcon[0] = bt;
  f.bcon[1] = (p[B1] + bt * f.ucon[1]) * iut;
  f.bcon[2] = (p[B2] + bt * f.ucon[2]) * iut;
  f.bcon[3] = (p[B3] + bt * f.ucon[3]) * iut;
  lower4(f.bcon, m, f.bcov);
  f.bsq = f.bcon[0] * f.bcov[0] + f.bcon[1] * f.bcov[1] + f.bcon[2] * f.bcov[2] +
          f.bcon[3] * f.bcov[3];
}

// Row mu of the mixed stress-energy tensor T^mu_nu, nu = 0..3.
template <typename R>
__device__ __forceinline__ void tmunu_row(const R p[NVAR], const Fluid<R>& f, R gam, int mu, R T[4]) {
  R pg = (gam - (R)1) * p[UU];
  R w = p[RHO] + p[UU] + pg + f.bsq;
  R ptot = pg + (R)0.5 * f.bsq;
  R wu = w * f.ucon[mu];
  R bm = f.bcon[mu];
#pragma unroll
  for (int nu = 0; nu < 4; nu++) T[nu] = wu * f.ucov[nu] - bm * f.bcov[nu];
  T[mu] += ptot;
}

// Flux along x^d (d = 1..3) or conserved variables (d = 0):
// sqrt(-g) (rho u^d, T^d_t + rho u^d, T^d_i, b^k u^d - b^d u^k); for d = 0 the
// field slots are sqrt(-g) B^k exactly.
template <typename R>
__device__ __forceinline__ void prim_to_flux(const R p[NVAR], const Fluid<R>& f, const PointMetric<R>& m,
                                    R gam, int d, R F[NVAR]) {
  R T[4];
  tmunu_row(p, f, gam, d, T);
  R mflux = p[RHO] * f.ucon[d];
  F[RHO] = m.gdet * mflux;
  F[UU] = m.gdet * (T[0] + mflux);
  F[U1] = m.gdet * T[1];
  F[U2] = m.gdet * T[2];
  F[U3] = m.gdet * T[3];
  if (d == 0) {
    F[B1] = m.gdet * p[B1];
    F[B2] = m.gdet * p[B2];
    F[B3] = m.gdet * p[B3];
  } else {
    F[B1] = m.gdet * (f.bcon[1] * f.ucon[d] - f.bcon[d] * f.ucon[1]);
    F[B2] = m.gdet * (f.bcon[2] * f.ucon[d] - f.bcon[d] * f.ucon[2]);
    F[B3] = m.gdet * (f.bcon[3] * f.ucon[d] - f.bcon[d] * f.ucon[3]);
  }
}

// Roots v = dx^d/dt of (k.u)^2 (1 - c^2) = c^2 k.k for k_mu = (-v, e_d), with
// the fast-speed bound c^2 = cs^2 + vA^2 - cs^2 vA^2.
template <typename R>
__device__ __forceinline__ void char_speeds(const R p[NVAR], const Fluid<R>& f, const PointMetric<R>& m,
                                   R gam, int d, R& cmax, R& cmin) {
  R pg = (gam - (R)1) * p[UU];
  R w = p[RHO] + gam * p[UU];
  R cs2 = gam * pg / w;
  R va2 = f.bsq / (f.bsq + w);
  R c2 = cs2 + va2 - cs2 * va2;
  R Au = f.ucon[d], Bu = f.ucon[0];
  R Asq = m.gcon[sidx(d, d)], Bsq = m.gcon[0], AB = m.gcon[sidx(0, d)];
  R A = Bu * Bu - c2 * (Bsq + Bu * Bu);
  R B = (R)-2 * (Au * Bu - c2 * (AB + Au * Bu));
  R C = Au * Au - c2 * (Asq + Au * Au);
  R disc = B * B - (R)4 * A * C;
  disc = disc > (R)0 ? disc : (R)0;
  R sq = sqrt(disc);
  R i2a = (R)0.5 / A;
  R v1 = (-B + sq) * i2a;
  R v2 = (-B - sq) * i2a;
  cmax = v1 > v2 ? v1 : v2;
  cmin = v1 > v2 ? v2 : v1;
}

// van Leer's monotonised-central slope.
template <typename R>
__device__ __forceinline__ R mc_slope(R l, R c, R r) {
  R dl = c - l, dr = r - c, dc = r - l;
  R m = fmin(fabs((R)2 * dl), fabs((R)2 * dr));
  m = fmin(m, fabs((R)0.5 * dc));
  m = dc > (R)0 ? m : -m;
  return dl * dr > (R)0 ? m : (R)0;
}

// WENO5 value at the right edge of zone c from point values a..e.  The three
// nonlinear weights d_k/(eps + beta_k)^2 are formed over a common
// denominator, so one division normalises them.
template <typename R>
__device__ __forceinline__ R weno5(R a, R b, R c, R d, R e, R eps) {
  const R r6 = (R)(1.0 / 6.0), k1312 = (R)(13.0 / 12.0);
  R p0 = ((R)2 * a - (R)7 * b + (R)11 * c) * r6;
  R p1 = (-b + (R)5 * c + (R)2 * d) * r6;
  R p2 = ((R)2 * c + (R)5 * d - e) * r6;
  R t0 = a - (R)2 * b + c, u0 = a - (R)4 * b + (R)3 * c;
  R t1 = b - (R)2 * c + d, u1 = b - d;
  R t2 = c - (R)2 * d + e, u2 = (R)3 * c - (R)4 * d + e;
  R s0 = eps + (k1312 * t0 * t0 + (R)0.25 * u0 * u0);
  R s1 = eps + (k1312 * t1 * t1 + (R)0.25 * u1 * u1);
  R s2 = eps + (k1312 * t2 * t2 + (R)0.25 * u2 * u2);
  s0 *= s0;
  s1 *= s1;
  s2 *= s2;
  R w0 = (R)0.1 * (s1 * s2), w1 = (R)0.6 * (s0 * s2), w2 = (R)0.3 * (s0 * s1);
  return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
}

// FP32 form: the weights are written through ratios of (eps + beta_k), so
// that no product of squared indicators underflows the single-precision range;
// a ratio that overflows drives its weight to the correct limit of zero.
__device__ __forceinline__ float weno5(float a, float b, float c, float d, float e, float eps) {
  const float r6 = 1.0f / 6.0f, k1312 = 13.0f / 12.0f;
  float p0 = (2.0f * a - 7.0f * b + 11.0f * c) * r6;
  float p1 = (-b + 5.0f * c + 2.0f * d) * r6;
  float p2 = (2.0f * c + 5.0f * d - e) * r6;
  float t0 = a - 2.0f * b + c, u0 = a - 4.0f * b + 3.0f * c;
  float t1 = b - 2.0f * c + d, u1 = b - d;
  float t2 = c - 2.0f * d + e, u2 = 3.0f * c - 4.0f * d + e;
  float s0 = eps + (k1312 * t0 * t0 + 0.25f * u0 * u0);
  float s1 = eps + (k1312 * t1 * t1 + 0.25f * u1 * u1);
  float s2 = eps + (k1312 * t2 * t2 + 0.25f * u2 * u2);
  float r01 = s0 / s1, r02 = s0 / s2, r12 = s1 / s2;
  float w0 = 0.1f / (0.1f + 0.6f * (r01 * r01) + 0.3f * (r02 * r02));
  float w1 = 0.6f / (0.1f / (r01 * r01) + 0.6f + 0.3f * (r12 * r12));
  float w2 = 0.3f / (0.1f / (r02 * r02) + 0.6f / (r12 * r12) + 0.3f);
  return w0 * p0 + w1 * p1 + w2 * p2;
}

}  // namespace grmhd
