// Per-point HARM physics for gfx950 in two arithmetics: double for the FP64
// path, float for the reduced-precision flux path.  Overloads on the
// argument type select between them.
//
//   * fluid four-vectors from the normal-observer velocity u~ (McKinney &
//     Gammie form the Algorithm section cites);
//   * rows of the ideal stress-energy tensor (EGRMHD section, ideal part);
//   * conserved variables / fluxes with the rest-mass energy removed;
//   * fast-magnetosonic characteristic speeds;
//   * linear-MC and WENO5 (Jiang-Shu weights) reconstruction.
#pragma once

#include <hip/hip_runtime.h>

#include "dual.hpp"

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
// Metric-derivative table of the geometric source: for nu = 1, 2 (row nu - 1)
// and each symmetric index s = (k, l), d_nu g_kl / 2 if k = l and d_nu g_kl if
// k < l (the pair (l, k) folded in), so that sum_s T^s D[s] = T^{kl} d_nu g_kl / 2.
enum { NDG = 20 };

// Both spacetimes of the library (flat space, and Kerr in modified
// Kerr-Schild coordinates) have g_{2 mu} = g^{2 mu} = 0 for mu != 2: x2 is
// orthogonal to the other coordinates, and the tables hold exact zeros
// there.  Those six entries are set to the constant zero rather than loaded,
// which gives the same values (and the same rounding of every expression
// that reads them) while keeping them out of registers.
__host__ __device__ constexpr bool x2_offdiag(int f) {
  return f == sidx(0, 2) || f == sidx(1, 2) || f == sidx(2, 3);
}

template <typename R>
__device__ __forceinline__ void load_metric(const double* __restrict__ tab, long plane, long q,
                                   PointMetric<R>& m) {
#pragma unroll
  for (int f = 0; f < 10; f++) {
    m.gcov[f] = x2_offdiag(f) ? (R)0 : (R)tab[(G_COV + f) * plane + q];
    m.gcon[f] = x2_offdiag(f) ? (R)0 : (R)tab[(G_CON + f) * plane + q];
  }
  m.gdet = (R)tab[G_DET * plane + q];
  m.alpha = (R)tab[G_ALPHA * plane + q];
}

template <typename R>
struct Fluid {
  R ucon[4], ucov[4], bcon[4], bcov[4], bsq;
};

// FP64: every operation is rounded on its own, in the order written, so the
// face fluxes reproduce a plain evaluation of the same formulas; in flat
// space (exact metric constants) they agree with it bit for bit.
namespace f64 {
using R = double;
#pragma clang fp contract(off)
__device__ __forceinline__ R fdiv(R a, R b) { return a / b; }
#include "physics_body.inc"
}  // namespace f64

// FP32: contraction into fused multiply-adds allowed, fast divisions.
namespace f32 {
using R = float;
#pragma clang fp contract(fast)
__device__ __forceinline__ R fdiv(R a, R b) { return a * __builtin_amdgcn_rcpf(b); }
#include "physics_body.inc"
}  // namespace f32

// Dual numbers: local Jacobians for the adjoint.
namespace fdual {
using R = Dual;
__device__ __forceinline__ R fdiv(R a, R b) { return a / b; }
__device__ __forceinline__ R fdiv(R a, double b) { return a / b; }
#include "physics_body.inc"
}  // namespace fdual

using f64::lower4;
using f32::lower4;
using fdual::lower4;
using f64::fluid_state;
using f32::fluid_state;
using fdual::fluid_state;
using f64::tmunu_row;
using f32::tmunu_row;
using fdual::tmunu_row;
using f64::metric_source;
using fdual::metric_source;
using f64::prim_to_flux;
using f32::prim_to_flux;
using fdual::prim_to_flux;
using f64::char_speeds;
using f32::char_speeds;
using fdual::char_speeds;
using f64::mc_slope;
using f32::mc_slope;
using fdual::mc_slope;
using f64::mc_left;
using f32::mc_left;
using fdual::mc_left;
using f64::mc_right;
using f32::mc_right;
using fdual::mc_right;
using f64::vl_left;
using f32::vl_left;
using f64::vl_right;
using f32::vl_right;
using f64::mp5;
using f32::mp5;
using f64::ppm_edges;
using f32::ppm_edges;
using f64::ppmx_edges;
using f32::ppmx_edges;
using f64::llf;
using f32::llf;
using fdual::llf;

// WENO5 (Jiang-Shu weights d_k / (eps + beta_k)^2, d = (1, 6, 3)/10) from
// point values a..e of zones c-2..c+2: the value at the right edge of zone c.
// The smoothness indicator of each three-zone stencil is formed by an
// expression that is symmetric under reversing the stencil -- (x + z) - 2y,
// fma(-4, y, fma(3, centre, outer)), y - z squared -- so a zone's left-edge
// value, weno5(e, d, c, b, a), reuses its right edge's indicators and
// weight products bit for bit (weno5_pair).  Arranged for few operations:
// every indicator is scaled by 12 (12 beta_k = 13 t_k^2 + 3 u_k^2, with
// 12 eps), which leaves the weights unchanged; the factors 1/10 of d and 1/6
// of the candidate polynomials cancel or move into the single quotient that
// normalises the weights over a common denominator.
//
// FP64: only the fused multiply-adds written out (contraction off), so an
// evaluation rounds the same way in whatever code it is inlined; the
// normalising quotient comes from the hardware reciprocal refined by Newton
// steps (within about an ulp of the correctly rounded quotient; the weights'
// denominator is a sum of positive normal numbers for weno_eps >= 1e-36).
#pragma clang fp contract(off)
namespace wd {
typedef double R;
__device__ __forceinline__ R qdiv(R n, R d) {
  R r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, (R)1), r, r);
  r = fma(fma(-d, r, (R)1), r, r);
  const R q = n * r;
  return fma(fma(-d, q, n), r, q);
}
// 12 (eps + beta) of the stencils (a, b, c), (b, c, d), (c, d, e)
__device__ __forceinline__ void indicators12(R a, R b, R c, R d, R e, R eps, R& s0, R& s1, R& s2) {
  const R eps12 = (R)12 * eps;
  R t0 = fma((R)-2, b, a + c), u0 = fma((R)-4, b, fma((R)3, c, a));
  R t1 = fma((R)-2, c, b + d), u1 = b - d;
  R t2 = fma((R)-2, d, c + e), u2 = fma((R)-4, d, fma((R)3, c, e));
  s0 = fma((R)13 * t0, t0, fma((R)3 * u0, u0, eps12));
  s1 = fma((R)13 * t1, t1, fma((R)3 * u1, u1, eps12));
  s2 = fma((R)13 * t2, t2, fma((R)3 * u2, u2, eps12));
}
// (eps + beta)^2 of the three stencils, scaled by 144
__device__ __forceinline__ void indicators(R a, R b, R c, R d, R e, R eps, R& s0, R& s1, R& s2) {
  indicators12(a, b, c, d, e, eps, s0, s1, s2);
  s0 *= s0;
  s1 *= s1;
  s2 *= s2;
}
// weighted value with weight products w0 = s1 s2, w1 = 6 s0 s2, w2 = 3 s0 s1
__device__ __forceinline__ R combine(R a, R b, R c, R d, R e, R s12, R s02, R s01) {
  R p0 = fma((R)11, c, fma((R)-7, b, (R)2 * a));
  R p1 = fma((R)2, d, fma((R)5, c, -b));
  R p2 = fma((R)5, d, fma((R)2, c, -e));
  R w0 = s12, w1 = (R)6 * s02, w2 = (R)3 * s01;
  return qdiv(fma(w0, p0, fma(w1, p1, w2 * p2)), (R)6 * ((w0 + w1) + w2));
}
}  // namespace wd

__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e, double eps) {
  double s0, s1, s2;
  wd::indicators(a, b, c, d, e, eps, s0, s1, s2);
  return wd::combine(a, b, c, d, e, s1 * s2, s0 * s2, s0 * s1);
}

// Both edges of zone c: left = weno5(e, d, c, b, a), right = weno5(a, b, c,
// d, e), from one set of indicators (reversing the stencil swaps s0 and s2).
__device__ __forceinline__ void weno5_pair(double a, double b, double c, double d, double e, double eps,
                                           double& left, double& right) {
  double s0, s1, s2;
  wd::indicators(a, b, c, d, e, eps, s0, s1, s2);
  const double s12 = s1 * s2, s02 = s0 * s2, s01 = s0 * s1;
  right = wd::combine(a, b, c, d, e, s12, s02, s01);
  left = wd::combine(e, d, c, b, a, s01, s02, s12);
}

// WENO-Z (Borges et al. 2008, power 2 as in Castro, Costa & Don 2011): the
// WENO5 candidates and indicators with weights d_k (1 + (tau5 / (eps +
// beta_k))^2), tau5 = |beta_0 - beta_2|.  Over the common denominator of the
// squared indicators s_k = (12 (eps + beta_k))^2 (tau5 scaled by 12 alike,
// T = (12 tau5)^2) the weight products are d_k (s_k + T) prod_{j != k} s_j,
// formed like WENO5's; with weno_eps >= 1e-36 they stay normal while
// 12 (eps + beta) < 1e100, i.e. for differences of primitives below ~1e49.
__device__ __forceinline__ double wenoz(double a, double b, double c, double d, double e, double eps) {
  double s0, s1, s2;
  wd::indicators12(a, b, c, d, e, eps, s0, s1, s2);
  const double tau = fabs(s0 - s2), T = tau * tau;
  s0 *= s0;
  s1 *= s1;
  s2 *= s2;
  return wd::combine(a, b, c, d, e, (s0 + T) * (s1 * s2), (s1 + T) * (s0 * s2), (s2 + T) * (s0 * s1));
}

// FP32 forms: contraction into fused multiply-adds allowed.
#pragma clang fp contract(fast)

// FP32 form.  The indicators are scaled by 12 as in the FP64 form and then
// normalised by the smallest one, r_k = s_k / min s in [1, 1e6] (clamped:
// a stencil 1e6 times rougher than the smoothest keeps a relative weight
// below 1e-12 either way, under FP32 resolution); the weights d_k / r_k^2 are
// formed over the common denominator as in the FP64 form, so the products
// stay below 1e25 (no overflow, no 0/0), and the two divisions are hardware
// reciprocals (v_rcp_f32).
namespace wf {
typedef float R;
__device__ __forceinline__ R weno5(R a, R b, R c, R d, R e, R eps) {
  const R eps12 = 12.0f * eps;
  R t0 = (a + c) - 2.0f * b, u0 = fmaf(-4.0f, b, fmaf(3.0f, c, a));
  R t1 = (b + d) - 2.0f * c, u1 = b - d;
  R t2 = (c + e) - 2.0f * d, u2 = fmaf(-4.0f, d, fmaf(3.0f, c, e));
  R s0 = fmaf(13.0f * t0, t0, fmaf(3.0f * u0, u0, eps12));
  R s1 = fmaf(13.0f * t1, t1, fmaf(3.0f * u1, u1, eps12));
  R s2 = fmaf(13.0f * t2, t2, fmaf(3.0f * u2, u2, eps12));
  const R im = __builtin_amdgcn_rcpf(fminf(fminf(s0, s1), s2));
  R r0 = fminf(s0 * im, 1e6f), r1 = fminf(s1 * im, 1e6f), r2 = fminf(s2 * im, 1e6f);
  r0 *= r0;
  r1 *= r1;
  r2 *= r2;
  R p0 = fmaf(11.0f, c, fmaf(-7.0f, b, 2.0f * a));
  R p1 = fmaf(2.0f, d, fmaf(5.0f, c, -b));
  R p2 = fmaf(5.0f, d, fmaf(2.0f, c, -e));
  R w0 = r1 * r2, w1 = 6.0f * (r0 * r2), w2 = 3.0f * (r0 * r1);
  return fmaf(w0, p0, fmaf(w1, p1, w2 * p2)) * __builtin_amdgcn_rcpf(6.0f * ((w0 + w1) + w2));
}
}  // namespace wf

__device__ __forceinline__ float weno5(float a, float b, float c, float d, float e, float eps) {
  return wf::weno5(a, b, c, d, e, eps);
}

// FP32 form of weno5_pair (the normalised indicators are symmetric too).
namespace wf {
__device__ __forceinline__ R wcomb(R a, R b, R c, R d, R e, R w0, R w1, R w2) {
  R p0 = fmaf(11.0f, c, fmaf(-7.0f, b, 2.0f * a));
  R p1 = fmaf(2.0f, d, fmaf(5.0f, c, -b));
  R p2 = fmaf(5.0f, d, fmaf(2.0f, c, -e));
  return fmaf(w0, p0, fmaf(w1, p1, w2 * p2)) * __builtin_amdgcn_rcpf(6.0f * ((w0 + w1) + w2));
}
__device__ __forceinline__ void weno5_pair(R a, R b, R c, R d, R e, R eps, R& left, R& right) {
  const R eps12 = 12.0f * eps;
  R t0 = (a + c) - 2.0f * b, u0 = fmaf(-4.0f, b, fmaf(3.0f, c, a));
  R t1 = (b + d) - 2.0f * c, u1 = b - d;
  R t2 = (c + e) - 2.0f * d, u2 = fmaf(-4.0f, d, fmaf(3.0f, c, e));
  R s0 = fmaf(13.0f * t0, t0, fmaf(3.0f * u0, u0, eps12));
  R s1 = fmaf(13.0f * t1, t1, fmaf(3.0f * u1, u1, eps12));
  R s2 = fmaf(13.0f * t2, t2, fmaf(3.0f * u2, u2, eps12));
  const R im = __builtin_amdgcn_rcpf(fminf(fminf(s0, s1), s2));
  R r0 = fminf(s0 * im, 1e6f), r1 = fminf(s1 * im, 1e6f), r2 = fminf(s2 * im, 1e6f);
  r0 *= r0;
  r1 *= r1;
  r2 *= r2;
  const R r12 = r1 * r2, r02 = r0 * r2, r01 = r0 * r1;
  right = wcomb(a, b, c, d, e, r12, 6.0f * r02, 3.0f * r01);
  left = wcomb(e, d, c, b, a, r01, 6.0f * r02, 3.0f * r12);
}
}  // namespace wf

__device__ __forceinline__ void weno5_pair(float a, float b, float c, float d, float e, float eps,
                                           float& left, float& right) {
  wf::weno5_pair(a, b, c, d, e, eps, left, right);
}

// FP32 WENO-Z.  With b_k = 12 (eps + beta_k), rho_k = b_k / min b >= 1 and
// theta = 12 tau5 / min b (clamped at 1e18; beyond it the weights agree
// with the clamped ones to FP32 resolution), the weights divided by the
// common factor 1 + theta^2 are d_k (e + q / rho_k^2), e = 1 / (1 + theta^2),
// q = theta^2 e: each in (0, d_k], the smoothest stencil's equal to d_k, so
// nothing overflows and the sum never vanishes.  Hardware reciprocals.
namespace wf {
__device__ __forceinline__ R wenoz(R a, R b, R c, R d, R e, R eps) {
  const R eps12 = 12.0f * eps;
  R t0 = (a + c) - 2.0f * b, u0 = fmaf(-4.0f, b, fmaf(3.0f, c, a));
  R t1 = (b + d) - 2.0f * c, u1 = b - d;
  R t2 = (c + e) - 2.0f * d, u2 = fmaf(-4.0f, d, fmaf(3.0f, c, e));
  R s0 = fmaf(13.0f * t0, t0, fmaf(3.0f * u0, u0, eps12));
  R s1 = fmaf(13.0f * t1, t1, fmaf(3.0f * u1, u1, eps12));
  R s2 = fmaf(13.0f * t2, t2, fmaf(3.0f * u2, u2, eps12));
  const R im = __builtin_amdgcn_rcpf(fminf(fminf(s0, s1), s2));
  const R th = fminf(fabsf(s0 - s2) * im, 1e18f);
  const R th2 = th * th;
  const R ee = __builtin_amdgcn_rcpf(1.0f + th2), q = th2 * ee;
  R r0 = s0 * im, r1 = s1 * im, r2 = s2 * im;
  R w0 = fmaf(q, __builtin_amdgcn_rcpf(r0 * r0), ee);
  R w1 = 6.0f * fmaf(q, __builtin_amdgcn_rcpf(r1 * r1), ee);
  R w2 = 3.0f * fmaf(q, __builtin_amdgcn_rcpf(r2 * r2), ee);
  R p0 = fmaf(11.0f, c, fmaf(-7.0f, b, 2.0f * a));
  R p1 = fmaf(2.0f, d, fmaf(5.0f, c, -b));
  R p2 = fmaf(5.0f, d, fmaf(2.0f, c, -e));
  return fmaf(w0, p0, fmaf(w1, p1, w2 * p2)) * __builtin_amdgcn_rcpf(6.0f * ((w0 + w1) + w2));
}
}  // namespace wf

__device__ __forceinline__ float wenoz(float a, float b, float c, float d, float e, float eps) {
  return wf::wenoz(a, b, c, d, e, eps);
}

// Dual-number WENO5: the same weights, in the plain single-division form;
// only its derivative part is used (local Jacobians of the adjoint).
__device__ __forceinline__ Dual weno5(Dual a, Dual b, Dual c, Dual d, Dual e, Dual eps) {
  const Dual k1312 = 13.0 / 12.0;
  Dual p0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  Dual p1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  Dual p2 = (2.0 * c + 5.0 * d - e) / 6.0;
  Dual t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
  Dual t1 = b - 2.0 * c + d, u1 = b - d;
  Dual t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
  Dual s0 = eps + (k1312 * t0 * t0 + 0.25 * u0 * u0);
  Dual s1 = eps + (k1312 * t1 * t1 + 0.25 * u1 * u1);
  Dual s2 = eps + (k1312 * t2 * t2 + 0.25 * u2 * u2);
  s0 *= s0;
  s1 *= s1;
  s2 *= s2;
  Dual w0 = 0.1 * (s1 * s2), w1 = 0.6 * (s0 * s2), w2 = 0.3 * (s0 * s1);
  return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
}

// Partial derivatives g0..g4 of the WENO5 edge value weno5(a, .., e) with
// respect to the five stencil values, by the chain rule through the weights: with
// s_k = eps + beta_k, w_k = d_k / s_k^2, W = sum w_k, o_k = w_k / W and
// v = sum o_k p_k,
//   dv/dx = sum_k o_k dp_k/dx - 2 sum_k o_k ((p_k - v) / s_k) dbeta_k/dx,
// where beta_k = 13/12 t_k^2 + 1/4 u_k^2 (t_k, u_k linear in x).  The same
// function as the dual-number form above, differentiated in closed form.
__device__ __forceinline__ void weno5_grad(double a, double b, double c, double d, double e, double eps,
                                           double& g0, double& g1, double& g2, double& g3, double& g4) {
#pragma clang fp contract(off)
  const double t0 = (a - 2.0 * b) + c, u0 = (a - 4.0 * b) + 3.0 * c;
  const double t1 = (b - 2.0 * c) + d, u1 = b - d;
  const double t2 = (c - 2.0 * d) + e, u2 = (3.0 * c - 4.0 * d) + e;
  const double k = 13.0 / 12.0;
  const double s0 = eps + (k * t0 * t0 + 0.25 * u0 * u0);
  const double s1 = eps + (k * t1 * t1 + 0.25 * u1 * u1);
  const double s2 = eps + (k * t2 * t2 + 0.25 * u2 * u2);
  const double w0 = 0.1 / (s0 * s0), w1 = 0.6 / (s1 * s1), w2 = 0.3 / (s2 * s2);
  const double iW = 1.0 / ((w0 + w1) + w2);
  const double o0 = w0 * iW, o1 = w1 * iW, o2 = w2 * iW;
  const double p0 = ((2.0 * a - 7.0 * b) + 11.0 * c) / 6.0;
  const double p1 = ((-b + 5.0 * c) + 2.0 * d) / 6.0;
  const double p2 = ((2.0 * c + 5.0 * d) - e) / 6.0;
  const double v = (o0 * p0 + o1 * p1) + o2 * p2;
  // -2 o_k (p_k - v) / s_k: the weight of dbeta_k/dx
  const double r0 = -2.0 * o0 * (p0 - v) / s0;
  const double r1 = -2.0 * o1 * (p1 - v) / s1;
  const double r2 = -2.0 * o2 * (p2 - v) / s2;
  const double h = 13.0 / 6.0;
  g0 = o0 * (2.0 / 6.0) + r0 * (h * t0 + 0.5 * u0);
  g1 = (o0 * (-7.0 / 6.0) + o1 * (-1.0 / 6.0)) + (r0 * (-2.0 * h * t0 - 2.0 * u0) + r1 * (h * t1 + 0.5 * u1));
  g2 = ((o0 * (11.0 / 6.0) + o1 * (5.0 / 6.0)) + o2 * (2.0 / 6.0)) +
         ((r0 * (h * t0 + 1.5 * u0) + r1 * (-2.0 * h * t1)) + r2 * (h * t2 + 1.5 * u2));
  g3 = (o1 * (2.0 / 6.0) + o2 * (5.0 / 6.0)) + (r1 * (h * t1 - 0.5 * u1) + r2 * (-2.0 * h * t2 - 2.0 * u2));
  g4 = o2 * (-1.0 / 6.0) + r2 * (h * t2 + 0.5 * u2);
}

// Partial derivatives of the MC edge values with respect to their three
// stencil values.  The MC slope minmod(2 dl, 2 dr, dc/2) (dl = c - l,
// dr = r - c, dc = r - l) is, away from its switching points, the selected
// candidate times a sign: the gradient is that candidate's, chosen by the
// same comparisons as the evaluation (fmin keeps the first operand on ties,
// |x| counts x = 0 as positive, a non-positive dl dr gives the zero slope).
__device__ __forceinline__ void mc_slope_grad(double l, double c, double r, double& gl, double& gc,
                                              double& gr) {
  const double dl = c - l, dr = r - c, dc = r - l;
  const double al = fabs(2.0 * dl), ar = fabs(2.0 * dr), ac = fabs(0.5 * dc);
  const bool pick_r = ar < al;
  const double m = pick_r ? ar : al;
  const bool pick_c = ac < m;
  const double sg = (dc > 0.0 ? 1.0 : -1.0) * (dl * dr > 0.0 ? 1.0 : 0.0);
  // d|k x|/dx = k sign(x), sign(0) = +1
  const double kl = sg * (dl < 0.0 ? -2.0 : 2.0), kr = sg * (dr < 0.0 ? -2.0 : 2.0);
  const double kc = sg * (dc < 0.0 ? -0.5 : 0.5);
  gl = pick_c ? -kc : (pick_r ? 0.0 : -kl);
  gc = pick_c ? 0.0 : (pick_r ? -kr : kl);
  gr = pick_c ? kc : (pick_r ? kr : 0.0);
}
// mc_left(l, c, r) = c + slope/2 and mc_right(l, c, r) = c - slope/2.
__device__ __forceinline__ void mc_left_grad(double l, double c, double r, double& g0, double& g1, double& g2) {
  double sl, sc, sr;
  mc_slope_grad(l, c, r, sl, sc, sr);
  g0 = 0.5 * sl;
  g1 = 1.0 + 0.5 * sc;
  g2 = 0.5 * sr;
}
__device__ __forceinline__ void mc_right_grad(double l, double c, double r, double& g0, double& g1, double& g2) {
  double sl, sc, sr;
  mc_slope_grad(l, c, r, sl, sc, sr);
  g0 = -0.5 * sl;
  g1 = 1.0 - 0.5 * sc;
  g2 = -0.5 * sr;
}

// ---------------------------------------------------------- face physics --
//
// The state on one side of a face as the flux kernels need it: conserved
// variables U, the flux F^d along the face normal (both without the factor
// sqrt(-g), which is common to the two sides and applied once to their
// Lax-Friedrichs combination) and the two fast signal speeds, from the
// reconstructed prims and the face metric.  The same
// formulas as fluid_state / prim_to_flux / char_speeds, arranged for the
// face, where these evaluations dominate the step's arithmetic:
//   * the face metric holds only the entries that are not identically zero
//     in the library's two spacetimes: flat space and Kerr in modified
//     Kerr-Schild coordinates both have g_{2 mu} = g^{2 mu} = 0 for mu != 2
//     (x2 is orthogonal to the other coordinates), so those table entries,
//     exactly zero, are never read and their products never formed;
//   * one reciprocal each of u^t, of w (b^2 + w) (sound and Alfven speeds
//     together) and of 2A (the two roots) per side, and of the lapse per
//     face, in place of the eight quotients per side of the written form;
//   * fused multiply-adds, written out (contraction off), so that a face
//     rounds the same way in every kernel that evaluates it.
// In FP64 the reciprocals are the hardware estimate refined by two Newton
// steps; the results differ from the written form by rounding only.
#pragma clang fp contract(off)

__device__ __forceinline__ double face_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}
__device__ __forceinline__ float face_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename R>
struct FaceMetric {
  R gtt, gt1, gt3, g11, g13, g22, g33;   // covariant
  R ctt, ct1, ct3, c11, c13, c22, c33;   // contravariant
  R gdet, alpha, ialpha;
};

template <typename R>
__device__ __forceinline__ void load_face_metric(const double* __restrict__ tab, long plane, long q,
                                                 FaceMetric<R>& m) {
  auto at = [&](int f) { return (R)tab[f * plane + q]; };
  m.gtt = at(G_COV + sidx(0, 0));
  m.gt1 = at(G_COV + sidx(0, 1));
  m.gt3 = at(G_COV + sidx(0, 3));
  m.g11 = at(G_COV + sidx(1, 1));
  m.g13 = at(G_COV + sidx(1, 3));
  m.g22 = at(G_COV + sidx(2, 2));
  m.g33 = at(G_COV + sidx(3, 3));
  m.ctt = at(G_CON + sidx(0, 0));
  m.ct1 = at(G_CON + sidx(0, 1));
  m.ct3 = at(G_CON + sidx(0, 3));
  m.c11 = at(G_CON + sidx(1, 1));
  m.c13 = at(G_CON + sidx(1, 3));
  m.c22 = at(G_CON + sidx(2, 2));
  m.c33 = at(G_CON + sidx(3, 3));
  m.gdet = at(G_DET);
  m.alpha = at(G_ALPHA);
  m.ialpha = face_rcp(m.alpha);
}

// U / sqrt(-g), F^D / sqrt(-g) (D = 1..3) and the signal speeds cp >= cm of
// the prims p.
template <int D, typename R>
__device__ __forceinline__ void face_side(const R p[NVAR], const FaceMetric<R>& m, R gam, R F[NVAR],
                                          R U[NVAR], R& cp, R& cm) {
  const R rho = p[RHO], uu = p[UU], v1 = p[U1], v2 = p[U2], v3 = p[U3];
  const R Bc1 = p[B1], Bc2 = p[B2], Bc3 = p[B3];
  // four-velocity: gamma^2 = 1 + g_ij u~i u~j, u^t = gamma / alpha,
  // u^i = u~i - gamma alpha g^{ti}, lowered with the face metric
  const R qsq = fma(m.g11 * v1, v1, fma(m.g22 * v2, v2, fma(m.g33 * v3, v3, (R)2 * (m.g13 * v1) * v3)));
  const R gamma = sqrt((R)1 + qsq);
  const R ga = gamma * m.alpha;
  const R ut = gamma * m.ialpha;
  const R iut = m.alpha * face_rcp(gamma);
  const R u1 = fma(-ga, m.ct1, v1), u2 = v2, u3 = fma(-ga, m.ct3, v3);
  const R l0 = fma(m.gtt, ut, fma(m.gt1, u1, m.gt3 * u3));
  const R l1 = fma(m.gt1, ut, fma(m.g11, u1, m.g13 * u3));
  const R l2 = m.g22 * u2;
  const R l3 = fma(m.gt3, ut, fma(m.g13, u1, m.g33 * u3));
  // magnetic four-vector: b^t = B^i u_i, b^i = (B^i + b^t u^i) / u^t
  const R bt = fma(Bc1, l1, fma(Bc2, l2, Bc3 * l3));
  const R b1 = fma(bt, u1, Bc1) * iut, b2 = fma(bt, u2, Bc2) * iut, b3 = fma(bt, u3, Bc3) * iut;
  const R k0 = fma(m.gtt, bt, fma(m.gt1, b1, m.gt3 * b3));
  const R k1 = fma(m.gt1, bt, fma(m.g11, b1, m.g13 * b3));
  const R k2 = m.g22 * b2;
  const R k3 = fma(m.gt3, bt, fma(m.g13, b1, m.g33 * b3));
  const R bsq = fma(bt, k0, fma(b1, k1, fma(b2, k2, b3 * k3)));
  // rows t (conserved variables) and D (flux) of
  // T^mu_nu = (rho + u + p + b^2) u^mu u_nu + (p + b^2/2) delta^mu_nu - b^mu b_nu
  const R pg = (gam - (R)1) * uu;
  const R w = ((rho + uu) + pg) + bsq;
  const R ptot = fma((R)0.5, bsq, pg);
  const R ud = D == 1 ? u1 : (D == 2 ? u2 : u3);
  const R bd = D == 1 ? b1 : (D == 2 ? b2 : b3);
  {
    const R wu = w * ut;
    const R ru = rho * ut;
    U[RHO] = ru;
    U[UU] = fma(wu, l0, fma(-bt, k0, ptot)) + ru;
    U[U1] = fma(wu, l1, -bt * k1);
    U[U2] = fma(wu, l2, -bt * k2);
    U[U3] = fma(wu, l3, -bt * k3);
    U[B1] = Bc1;
    U[B2] = Bc2;
    U[B3] = Bc3;
  }
  {
    const R wu = w * ud;
    const R ru = rho * ud;
    F[RHO] = ru;
    F[UU] = fma(wu, l0, -bd * k0) + ru;
    F[U1] = fma(wu, l1, fma(-bd, k1, D == 1 ? ptot : (R)0));
    F[U2] = fma(wu, l2, fma(-bd, k2, D == 2 ? ptot : (R)0));
    F[U3] = fma(wu, l3, fma(-bd, k3, D == 3 ? ptot : (R)0));
    F[B1] = fma(b1, ud, -bd * u1);
    F[B2] = fma(b2, ud, -bd * u2);
    F[B3] = fma(b3, ud, -bd * u3);
  }
  // fast speeds: roots v of (u^D - v u^t)^2 (1 - c^2) = c^2 (v^2 g^tt - 2 v g^tD + g^DD),
  // c^2 = cs^2 + vA^2 - cs^2 vA^2, cs^2 = gam p / w, vA^2 = b^2 / (b^2 + w), w = rho + gam u
  const R we = fma(gam, uu, rho);
  const R sw = bsq + we;
  const R rr = face_rcp(we * sw);
  const R cs2 = ((gam * pg) * sw) * rr;
  const R va2 = (bsq * we) * rr;
  const R c2 = fma(-cs2, va2, cs2 + va2);
  const R cdd = D == 1 ? m.c11 : (D == 2 ? m.c22 : m.c33);
  const R ctd = D == 1 ? m.ct1 : (D == 2 ? (R)0 : m.ct3);
  const R ut2 = ut * ut, udt = ud * ut, ud2 = ud * ud;
  const R A = fma(-c2, m.ctt + ut2, ut2);
  const R B = (R)-2 * fma(-c2, ctd + udt, udt);
  const R C = fma(-c2, cdd + ud2, ud2);
  R disc = fma(B, B, (R)-4 * A * C);
  disc = disc > (R)0 ? disc : (R)0;
  const R sq = sqrt(disc);
  const R i2a = (R)0.5 * face_rcp(A);
  const R va = (sq - B) * i2a, vb = (-B - sq) * i2a;
  cp = va > vb ? va : vb;
  cm = va > vb ? vb : va;
}

}  // namespace grmhd
