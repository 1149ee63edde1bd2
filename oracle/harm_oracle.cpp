// TEST INFRASTRUCTURE ONLY.  Plain, slow, scalar FP64 CPU reference of one
// HARM ideal-GRMHD step; only the test-suite, the smoke check and the CPU
// baseline leg of the benchmark load it.  It shares no code with the HIP
// library.
//
// What it computes (the Algorithm section names the scheme; the stress-energy
// tensor is the ideal part of the EGRMHD section):
//   * geometry: Minkowski, or Kerr in modified Kerr-Schild coordinates, with
//     the metric and connection cached per (x1, x2) as the GRCoordinates
//     description says (Core section);
//   * primitive -> conserved / flux with the normal-observer velocity;
//   * linear MC or WENO5 reconstruction of each primitive (Algorithm section),
//     or, among the further schemes the Solvers section lists, WENO-Z, MP5,
//     PPM, linear with van Leer's limiter and donor cell;
//   * local Lax-Friedrichs fluxes with the fast-magnetosonic speed bound;
//   * Flux-CT: B fluxes replaced by corner-averaged EMFs;
//   * flux divergence + geometric source, two-stage SSP Runge-Kutta;
//   * 1D_W Newton-Raphson inversion of conserved -> primitive (Algorithm and
//     Performance sections name the 1D_w inverter);
//   * ghost-zone boundary conditions, CFL time step and the corner div B.
// Readings where the paper is silent are stated next to the code they shape.
//
// State layout: double[8][n3+6][n2+6][n1+6], x1 fastest, variables
// (rho, u, u~1, u~2, u~3, B1, B2, B3).
//
// Build: g++ -O2 -fopenmp -fPIC -shared (no -ffast-math; x86-64 code without
// FMA, so every operation is individually rounded).

#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_COUNTING
#include "flopcount.hpp"
typedef CountedReal real;
FlopTally g_flops;
#else
typedef double real;
using std::sqrt;
using std::fabs;
using std::sin;
using std::cos;
using std::exp;
using std::isfinite;
#endif

namespace {

const int NV = 8, NG = 3;
enum { RHO = 0, UU = 1, U1 = 2, U2 = 3, U3 = 4, B1 = 5, B2 = 6, B3 = 7 };
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_POLAR = 2, BC_FROZEN = 3 };
enum { MINKOWSKI = 0, KERR_MKS = 1 };
enum { RECON_MC = 0, RECON_WENO5 = 1, RECON_DONOR = 2, RECON_WENOZ = 3, RECON_VL = 4, RECON_MP5 = 5,
       RECON_PPM = 6, RECON_PPMX = 7 };

}  // namespace

extern "C" {
typedef struct {
  int n1, n2, n3;
  double x1min, x1max, x2min, x2max, x3min, x3max;
  int bc[6];
  int metric;
  double a, hslope;
  double gam;          // adiabatic index
  int recon;
  double weno_eps;
  double newton_tol;
  int newton_maxit;
  double cfl;
  int nthreads;
  int inverter;        // 0: 1D_W (Noble et al.), 1: Kastaun et al. bracketed recovery,
                       // 2: the implicit solver's Newton (secant Jacobian, pivoted QR)
  double kastaun_wmax; // Lorentz-factor cap of the Kastaun recovery
  int floors;          // 1: density/energy floors and ceilings after every inversion
  double rho_min_geom, u_min_geom;        // geometric floors rho r^-3/2, u r^-5/2
  double bsq_over_rho_max, bsq_over_u_max; // magnetisation floors
  double u_over_rho_max, gamma_max;       // temperature and Lorentz-factor ceilings
  int fofc;            // 1: first-order flux correction of zones a stage would break
  int ct;              // 0: Flux-CT; face-centred CT with 1: averaged, 2: upwinded edge EMFs
  int integrator;      // 0: SSPRK2; 1: predictor-corrector (half-step predictor, then the
                       // full step from U^n with the predicted state's rates); 2: RK1 (forward Euler);
                       // 3: SSPRK(5,4) (Spiteri & Ruuth 2002)
  double tau_r, chi_emhd, nu_emhd;  // Extended GRMHD closure constants (orc_run_emhd)
} orc_cfg;
}

namespace {

// ---------------------------------------------------------------- geometry --

struct Geom {
  real gcov[4][4], gcon[4][4], gdet, alpha;
};

// Kerr-Schild metric (M = 1) and its first derivatives with respect to r and
// theta, written out from the closed form.
//   Sigma = r^2 + a^2 cos^2 th,  z = 2 r / Sigma,
//   g_tt = z - 1, g_tr = z, g_tph = -a z s^2, g_rr = 1 + z,
//   g_rph = -a s^2 (1 + z), g_thth = Sigma, g_phph = s^2 (Sigma + a^2 s^2 (1+z)).
void ks_metric(real a, real r, real th, real g[4][4], real dgr[4][4], real dgth[4][4]) {
  real s = sin(th), c = cos(th);
  real s2 = s * s, c2 = c * c;
  real sig = r * r + a * a * c2;
  real z = 2.0 * r / sig;
  real sig_r = 2.0 * r, sig_th = -2.0 * a * a * c * s;
  real z_r = 2.0 / sig - 2.0 * r * sig_r / (sig * sig);
  real z_th = -2.0 * r * sig_th / (sig * sig);
  real s2_th = 2.0 * s * c;
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) g[m][n] = dgr[m][n] = dgth[m][n] = 0.0;
  g[0][0] = z - 1.0;            dgr[0][0] = z_r;  dgth[0][0] = z_th;
  g[0][1] = z;                  dgr[0][1] = z_r;  dgth[0][1] = z_th;
  g[0][3] = -a * z * s2;        dgr[0][3] = -a * z_r * s2;
  dgth[0][3] = -a * (z_th * s2 + z * s2_th);
  g[1][1] = 1.0 + z;            dgr[1][1] = z_r;  dgth[1][1] = z_th;
  g[1][3] = -a * s2 * (1.0 + z); dgr[1][3] = -a * s2 * z_r;
  dgth[1][3] = -a * (s2_th * (1.0 + z) + s2 * z_th);
  g[2][2] = sig;                dgr[2][2] = sig_r; dgth[2][2] = sig_th;
  real inner = sig + a * a * s2 * (1.0 + z);
  g[3][3] = s2 * inner;
  dgr[3][3] = s2 * (sig_r + a * a * s2 * z_r);
  dgth[3][3] = s2_th * inner + s2 * (sig_th + a * a * (s2_th * (1.0 + z) + s2 * z_th));
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < m; n++) { g[m][n] = g[n][m]; dgr[m][n] = dgr[n][m]; dgth[m][n] = dgth[n][m]; }
}

// Metric at a point.  Modified KS: r = exp(x1), th = pi x2 + (1-h)/2 sin(2 pi x2),
// ph = x3, so g_MKS[m][n] = L_m L_n g_KS[m][n] with L = (1, r, dth/dx2, 1).
// The inverse is the closed-form KS inverse scaled by 1/(L_m L_n); sqrt(-g)
// uses |sin th| so that zones continued past a pole stay finite.
void geom_point(const orc_cfg& c, real x1, real x2, Geom& G) {
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) G.gcov[m][n] = G.gcon[m][n] = 0.0;
  if (c.metric == MINKOWSKI) {
    G.gcov[0][0] = G.gcon[0][0] = -1.0;
    for (int i = 1; i < 4; i++) G.gcov[i][i] = G.gcon[i][i] = 1.0;
    G.gdet = 1.0;
    G.alpha = 1.0;
    return;
  }
  const real a = c.a, h = c.hslope;
  real r = exp(x1);
  real th = M_PI * x2 + 0.5 * (1.0 - h) * sin(2.0 * M_PI * x2);
  real dth = M_PI * (1.0 + (1.0 - h) * cos(2.0 * M_PI * x2));
  real L[4] = {1.0, r, dth, 1.0};
  real g[4][4], dgr[4][4], dgth[4][4];
  ks_metric(a, r, th, g, dgr, dgth);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) G.gcov[m][n] = g[m][n] * L[m] * L[n];
  real s = sin(th), cth = cos(th);
  real s2 = s * s;
  real sig = r * r + a * a * cth * cth;
  real z = 2.0 * r / sig;
  real del = r * r - 2.0 * r + a * a;
  real gi[4][4];
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) gi[m][n] = 0.0;
  gi[0][0] = -(1.0 + z);
  gi[0][1] = gi[1][0] = z;
  gi[1][1] = del / sig;
  gi[1][3] = gi[3][1] = a / sig;
  gi[2][2] = 1.0 / sig;
  gi[3][3] = 1.0 / (sig * s2);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) G.gcon[m][n] = gi[m][n] / (L[m] * L[n]);
  G.gdet = sig * fabs(s) * r * dth;
  G.alpha = 1.0 / sqrt(-G.gcon[0][0]);
}

// Connection Gamma^l_{mn} = 1/2 g^{lk} (d_m g_kn + d_n g_km - d_k g_mn) at a
// point, from analytic metric derivatives (only d/dx1 and d/dx2 are nonzero).
void conn_point(const orc_cfg& c, real x1, real x2, real conn[4][4][4]) {
  for (int l = 0; l < 4; l++)
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) conn[l][m][n] = 0.0;
  if (c.metric == MINKOWSKI) return;
  const real a = c.a, h = c.hslope;
  real r = exp(x1);
  real th = M_PI * x2 + 0.5 * (1.0 - h) * sin(2.0 * M_PI * x2);
  real dth = M_PI * (1.0 + (1.0 - h) * cos(2.0 * M_PI * x2));
  real d2th = -2.0 * M_PI * M_PI * (1.0 - h) * sin(2.0 * M_PI * x2);
  real L[4] = {1.0, r, dth, 1.0};
  real g[4][4], dgr[4][4], dgth[4][4];
  ks_metric(a, r, th, g, dgr, dgth);
  // dg[k][m][n] = d g_MKS[m][n] / d x^k
  real dg[4][4][4];
  for (int k = 0; k < 4; k++)
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) dg[k][m][n] = 0.0;
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) {
      real LL = L[m] * L[n];
      // x1: dL_1/dx1 = r = L_1, d g_KS/dx1 = r d g_KS/dr
      real f1 = (m == 1 ? 1.0 : 0.0) + (n == 1 ? 1.0 : 0.0);
      dg[1][m][n] = LL * (f1 * g[m][n] + r * dgr[m][n]);
      // x2: dL_2/dx2 = d2th, d g_KS/dx2 = dth d g_KS/dth
      real f2 = (m == 2 ? 1.0 : 0.0) + (n == 2 ? 1.0 : 0.0);
      dg[2][m][n] = LL * (f2 * (d2th / dth) * g[m][n] + dth * dgth[m][n]);
    }
  Geom G;
  geom_point(c, x1, x2, G);
  for (int l = 0; l < 4; l++)
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) {
        real sum = 0.0;
        for (int k = 0; k < 4; k++)
          sum += G.gcon[l][k] * (dg[m][k][n] + dg[n][k][m] - dg[k][m][n]);
        conn[l][m][n] = 0.5 * sum;
      }
}

// --------------------------------------------------- primitive -> fluxes --

struct FluidState {
  real ucon[4], ucov[4], bcon[4], bcov[4], bsq;
};

void lower(const real v[4], const Geom& G, real out[4]) {
  for (int m = 0; m < 4; m++) {
    real s = 0.0;
    for (int n = 0; n < 4; n++) s += G.gcov[m][n] * v[n];
    out[m] = s;
  }
}

// Four-velocity from the normal-observer velocity u~ (McKinney & Gammie form):
// gamma = sqrt(1 + g_ij u~i u~j), u^t = gamma/alpha, u^i = u~i - gamma alpha g^{ti};
// field four-vector b^t = B^i u_i, b^i = (B^i + b^t u^i)/u^t.
void fluid_state(const real P[NV], const Geom& G, FluidState& S) {
  real qsq = 0.0;
  for (int i = 1; i < 4; i++)
    for (int j = 1; j < 4; j++) qsq += G.gcov[i][j] * P[U1 + i - 1] * P[U1 + j - 1];
  real gamma = sqrt(1.0 + qsq);
  S.ucon[0] = gamma / G.alpha;
  for (int i = 1; i < 4; i++) S.ucon[i] = P[U1 + i - 1] - gamma * G.alpha * G.gcon[0][i];
  lower(S.ucon, G, S.ucov);
  S.bcon[0] = 0.0;
  for (int i = 1; i < 4; i++) S.bcon[0] += P[B1 + i - 1] * S.ucov[i];
  for (int i = 1; i < 4; i++) S.bcon[i] = (P[B1 + i - 1] + S.bcon[0] * S.ucon[i]) / S.ucon[0];
  lower(S.bcon, G, S.bcov);
  S.bsq = 0.0;
  for (int m = 0; m < 4; m++) S.bsq += S.bcon[m] * S.bcov[m];
}

// Mixed stress-energy T^mu_nu = (rho+u+p+b^2) u^mu u_nu + (p + b^2/2) delta - b^mu b_nu.
real tmunu(const real P[NV], const FluidState& S, real gam, int mu, int nu) {
  real p = (gam - 1.0) * P[UU];
  real w = P[RHO] + P[UU] + p + S.bsq;
  real ptot = p + 0.5 * S.bsq;
  return w * S.ucon[mu] * S.ucov[nu] + (mu == nu ? ptot : 0.0) - S.bcon[mu] * S.bcov[nu];
}

// Conserved variables (d = 0) or fluxes along x^d (d = 1..3):
// sqrt(-g) (rho u^d, T^d_t + rho u^d, T^d_1, T^d_2, T^d_3, b^k u^d - b^d u^k).
// The energy slot carries T^d_t + rho u^d (rest-mass energy removed).
void prim_to_flux(const real P[NV], const FluidState& S, const Geom& G, real gam, int d, real F[NV]) {
  F[RHO] = G.gdet * P[RHO] * S.ucon[d];
  F[UU] = G.gdet * (tmunu(P, S, gam, d, 0) + P[RHO] * S.ucon[d]);
  for (int i = 1; i < 4; i++) F[U1 + i - 1] = G.gdet * tmunu(P, S, gam, d, i);
  for (int k = 1; k < 4; k++) {
    if (d == 0)
      F[B1 + k - 1] = G.gdet * P[B1 + k - 1];
    else
      F[B1 + k - 1] = G.gdet * (S.bcon[k] * S.ucon[d] - S.bcon[d] * S.ucon[k]);
  }
}

// Characteristic speeds dx^d/dt of the fast magnetosonic bound: roots of
// (k.u)^2 (1 - c^2) = c^2 k.k for the covector k = (-v, e_d), with
// c^2 = cs^2 + vA^2 - cs^2 vA^2, cs^2 = gam p / w, vA^2 = b^2/(b^2 + w), w = rho + gam u.
void vchar(const real P[NV], const FluidState& S, const Geom& G, real gam, int d,
           real& cmax, real& cmin) {
  real p = (gam - 1.0) * P[UU];
  real w = P[RHO] + gam * P[UU];
  real cs2 = gam * p / w;
  real va2 = S.bsq / (S.bsq + w);
  real c2 = cs2 + va2 - cs2 * va2;
  real Au = S.ucon[d], Bu = S.ucon[0];
  real Asq = G.gcon[d][d], Bsq = G.gcon[0][0], AB = G.gcon[0][d];
  real A = Bu * Bu - c2 * (Bsq + Bu * Bu);
  real B = -2.0 * (Au * Bu - c2 * (AB + Au * Bu));
  real C = Au * Au - c2 * (Asq + Au * Au);
  real disc = B * B - 4.0 * A * C;
  if (disc < 0.0) disc = 0.0;
  real sq = sqrt(disc);
  real v1 = (-B + sq) / (2.0 * A);
  real v2 = (-B - sq) / (2.0 * A);
  cmax = v1 > v2 ? v1 : v2;
  cmin = v1 > v2 ? v2 : v1;
}

// ---------------------------------------------------------- reconstruction --

// Monotonised-central limited slope of zone c with neighbours l, r.
real mc_slope(real l, real c, real r) {
  real dl = c - l, dr = r - c, dc = r - l;
  if (dl * dr <= 0.0) return 0.0;
  real m = fabs(2.0 * dl);
  if (fabs(2.0 * dr) < m) m = fabs(2.0 * dr);
  if (fabs(0.5 * dc) < m) m = fabs(0.5 * dc);
  return dc > 0.0 ? m : -m;
}

// WENO5 value at the right edge of zone c from point values (a,b,c,d,e):
// Jiang-Shu smoothness indicators, linear weights (1/10, 6/10, 3/10), power 2.
real weno5(real a, real b, real c, real d, real e, real eps) {
  real p0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  real p1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  real p2 = (2.0 * c + 5.0 * d - e) / 6.0;
  real t;
  t = a - 2.0 * b + c; real s0 = 13.0 / 12.0 * t * t;
  t = a - 4.0 * b + 3.0 * c; s0 += 0.25 * t * t;
  t = b - 2.0 * c + d; real s1 = 13.0 / 12.0 * t * t;
  t = b - d; s1 += 0.25 * t * t;
  t = c - 2.0 * d + e; real s2 = 13.0 / 12.0 * t * t;
  t = 3.0 * c - 4.0 * d + e; s2 += 0.25 * t * t;
  real a0 = 0.1 / ((eps + s0) * (eps + s0));
  real a1 = 0.6 / ((eps + s1) * (eps + s1));
  real a2 = 0.3 / ((eps + s2) * (eps + s2));
  return (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
}

// WENO-Z value at the right edge of zone c (Borges et al. 2008, with the
// power of Castro, Costa & Don 2011, here 2): the WENO5 candidates and
// indicators, weights d_k (1 + (tau5 / (eps + beta_k))^2) normalised, where
// tau5 = |beta_0 - beta_2|.
real wenoz(real a, real b, real c, real d, real e, real eps) {
  real p0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  real p1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  real p2 = (2.0 * c + 5.0 * d - e) / 6.0;
  real t;
  t = a - 2.0 * b + c; real s0 = 13.0 / 12.0 * t * t;
  t = a - 4.0 * b + 3.0 * c; s0 += 0.25 * t * t;
  t = b - 2.0 * c + d; real s1 = 13.0 / 12.0 * t * t;
  t = b - d; s1 += 0.25 * t * t;
  t = c - 2.0 * d + e; real s2 = 13.0 / 12.0 * t * t;
  t = 3.0 * c - 4.0 * d + e; s2 += 0.25 * t * t;
  real tau = fabs(s0 - s2);
  real z0 = tau / (eps + s0), z1 = tau / (eps + s1), z2 = tau / (eps + s2);
  real a0 = 0.1 * (1.0 + z0 * z0);
  real a1 = 0.6 * (1.0 + z1 * z1);
  real a2 = 0.3 * (1.0 + z2 * z2);
  return (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
}

// Van Leer's limited slope of zone c: the harmonic mean of the two one-sided
// differences, zero where they differ in sign (an extremum) or one vanishes.
real vl_slope(real l, real c, real r) {
  real dl = c - l, dr = r - c;
  if (dl * dr <= 0.0) return 0.0;
  return 2.0 * dl * dr / (dl + dr);
}

static real rmin(real a, real b) { return b < a ? b : a; }
static real rmax(real a, real b) { return b > a ? b : a; }
static real min3(real a, real b, real c) { return rmin(a, rmin(b, c)); }
static real max3(real a, real b, real c) { return rmax(a, rmax(b, c)); }
static real minmod2(real a, real b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}
static real minmod4(real w, real x, real y, real z) {
  if (!((w > 0.0 && x > 0.0 && y > 0.0 && z > 0.0) || (w < 0.0 && x < 0.0 && y < 0.0 && z < 0.0)))
    return 0.0;
  real m = rmin(rmin(fabs(w), fabs(x)), rmin(fabs(y), fabs(z)));
  return w > 0.0 ? m : -m;
}

// MP5 value at the right edge of zone c from (a, b, c, d, e) (Suresh & Huynh
// 1997): the linear fifth-order edge value, kept when it lies between c and
// the monotonicity-preserving bound c + minmod(d - c, 4 (c - b)); otherwise
// moved to the nearest point of [v_min, v_max], the interval built from the
// upper and lower limits with the curvature measures d^M4 (alpha = 4).
real mp5(real a, real b, real c, real d, real e) {
  const real alpha = 4.0;
  real vl = (2.0 * a - 13.0 * b + 47.0 * c + 27.0 * d - 3.0 * e) / 60.0;
  real vmp = c + minmod2(d - c, alpha * (c - b));
  if ((vl - c) * (vl - vmp) <= 0.0) return vl;
  real djm1 = a + c - 2.0 * b, dj = b + d - 2.0 * c, djp1 = c + e - 2.0 * d;
  real dm4p = minmod4(4.0 * dj - djp1, 4.0 * djp1 - dj, dj, djp1);
  real dm4m = minmod4(4.0 * dj - djm1, 4.0 * djm1 - dj, dj, djm1);
  real vul = c + alpha * (c - b);
  real vav = 0.5 * (c + d);
  real vmd = vav - 0.5 * dm4p;
  real vlc = c + 0.5 * (c - b) + 4.0 / 3.0 * dm4m;
  real vmin = rmax(min3(c, d, vmd), min3(c, vul, vlc));
  real vmax = rmin(max3(c, d, vmd), max3(c, vul, vlc));
  return vl + minmod2(vmin - vl, vmax - vl);
}

// PPM (Colella & Woodward 1984) edge values of zone c from (a, b, c, d, e):
// interface values a_{c+-1/2} = x + (y - x)/2 - (da_y - da_x)/6 with the
// limited slopes da (the monotonised-central slope, their limiter), then the
// parabola through (aL, c, aR) made monotone in the zone: flattened to c at
// an extremum, otherwise the edge on the side of an interior extremum moved
// to 3c - 2 (other edge).
void ppm_edges(real a, real b, real c, real d, real e, real& aL, real& aR) {
  real sb = mc_slope(a, b, c), sc = mc_slope(b, c, d), sd = mc_slope(c, d, e);
  aL = b + 0.5 * (c - b) - (sc - sb) / 6.0;
  aR = c + 0.5 * (d - c) - (sd - sc) / 6.0;
  if ((aR - c) * (c - aL) <= 0.0) {
    aL = c;
    aR = c;
    return;
  }
  real da = aR - aL, a6 = 6.0 * (c - 0.5 * (aL + aR));
  if (da * a6 > da * da)
    aL = 3.0 * c - 2.0 * aR;
  else if (-(da * da) > da * a6)
    aR = 3.0 * c - 2.0 * aL;
}

// PPMX: PPM with the extremum-preserving limiter of Colella & Sekora
// (2008), C = 1.25.  Interface value of the face between y and z from
// (x, y, z, w): the fourth-order 7/12 (y + z) - 1/12 (x + w); where it does
// not lie between y and z it becomes (y + z)/2 - D/6 with the second
// difference D = 3 (y - 2a + z) limited against C (x - 2y + z) and
// C (y - 2z + w): the smallest magnitude with their common sign, 0 if the
// signs differ.
real ppmx_interface(real x, real y, real z, real w) {
  const real C = 1.25;
  real a = 7.0 / 12.0 * (y + z) - 1.0 / 12.0 * (x + w);
  if ((a - y) * (z - a) < 0.0) {
    real d = 3.0 * (y - 2.0 * a + z), dl = x - 2.0 * y + z, dr = y - 2.0 * z + w;
    real lim = 0.0;
    if (d > 0.0 && dl > 0.0 && dr > 0.0) lim = rmin(d, rmin(C * dl, C * dr));
    if (d < 0.0 && dl < 0.0 && dr < 0.0) lim = -rmin(-d, rmin(-C * dl, -C * dr));
    a = 0.5 * (y + z) - lim / 6.0;
  }
  return a;
}

// PPMX edge values of zone c from (a, b, c, d, e): the two interface values,
// then, where the zone holds an extremum (of the parabola, (aR - c)(c - aL)
// <= 0, or of the data, (d - c)(c - b) <= 0), the parabola's curvature
// 6 (aL + aR - 2c) limited against C times the second differences centred
// on b, c and d (smallest magnitude with the common sign, else 0) and both
// edges' offsets from c scaled by limited / unlimited (c itself when the
// curvature is 0); elsewhere Colella & Woodward's overshoot correction: an
// edge more than twice as far from c as the other is moved to c - 2 (other
// edge - c).
void ppmx_edges(real a, real b, real c, real d, real e, real& aL, real& aR) {
  const real C = 1.25;
  aL = ppmx_interface(a, b, c, d);
  aR = ppmx_interface(b, c, d, e);
  if ((aR - c) * (c - aL) <= 0.0 || (d - c) * (c - b) <= 0.0) {
    real d2 = 6.0 * (aL + aR - 2.0 * c);
    real d2l = a - 2.0 * b + c, d2c = b - 2.0 * c + d, d2r = c - 2.0 * d + e;
    real lim = 0.0;
    if (d2 > 0.0 && d2l > 0.0 && d2c > 0.0 && d2r > 0.0)
      lim = rmin(d2, rmin(C * d2l, rmin(C * d2c, C * d2r)));
    if (d2 < 0.0 && d2l < 0.0 && d2c < 0.0 && d2r < 0.0)
      lim = -rmin(-d2, rmin(-C * d2l, rmin(-C * d2c, -C * d2r)));
    if (d2 != 0.0) {
      aL = c + (aL - c) * (lim / d2);
      aR = c + (aR - c) * (lim / d2);
    } else {
      aL = c;
      aR = c;
    }
    return;
  }
  const real dl = aL - c, dr = aR - c;
  if (fabs(dl) >= 2.0 * fabs(dr)) aL = c - 2.0 * dr;
  if (fabs(dr) >= 2.0 * fabs(dl)) aR = c - 2.0 * dl;
}

// ------------------------------------------------------------------ grid --

struct Grid {
  orc_cfg c;
  int n[3];
  int s1, s2, s3;     // padded extents
  long nz;            // padded zones per variable
  real dx[3], xmin[3];
  // geometry cached per padded (i, j): centre, x1 face, x2 face, x1-x2 corner
  std::vector<Geom> gC, gF1, gF2, gCorner;
  std::vector<real> conn;  // 64 per (i, j)
  bool pole_lo, pole_hi;   // x2 boundaries that sit on the polar axis

  explicit Grid(const orc_cfg& cfg) : c(cfg) {
    n[0] = c.n1; n[1] = c.n2; n[2] = c.n3;
    s1 = c.n1 + 2 * NG; s2 = c.n2 + 2 * NG; s3 = c.n3 + 2 * NG;
    nz = (long)s1 * s2 * s3;
    xmin[0] = c.x1min; xmin[1] = c.x2min; xmin[2] = c.x3min;
    dx[0] = (c.x1max - c.x1min) / c.n1;
    dx[1] = (c.x2max - c.x2min) / c.n2;
    dx[2] = (c.x3max - c.x3min) / c.n3;
    // In modified KS the faces x2 = 0 and x2 = 1 are the polar axis (theta = 0, pi).
    pole_lo = c.metric == KERR_MKS && std::fabs(c.x2min) < 1e-10;
    pole_hi = c.metric == KERR_MKS && std::fabs(c.x2max - 1.0) < 1e-10;
    long n2d = (long)s1 * s2;
    gC.resize(n2d); gF1.resize(n2d); gF2.resize(n2d); gCorner.resize(n2d);
    conn.resize(n2d * 64);
    for (int j = -NG; j < c.n2 + NG; j++)
      for (int i = -NG; i < c.n1 + NG; i++) {
        long q = (long)(j + NG) * s1 + (i + NG);
        real xc1 = xmin[0] + (i + 0.5) * dx[0], xc2 = xmin[1] + (j + 0.5) * dx[1];
        real xf1 = xmin[0] + i * dx[0], xf2 = xmin[1] + j * dx[1];
        geom_point(c, xc1, xc2, gC[q]);
        geom_point(c, xf1, xc2, gF1[q]);
        if (!((pole_lo && j == 0) || (pole_hi && j == c.n2)))
          geom_point(c, xc1, xf2, gF2[q]);
        if (!((pole_lo && j == 0) || (pole_hi && j == c.n2)))
          geom_point(c, xf1, xf2, gCorner[q]);
        real cn[4][4][4];
        conn_point(c, xc1, xc2, cn);
        for (int l = 0; l < 4; l++)
          for (int m = 0; m < 4; m++)
            for (int nn = 0; nn < 4; nn++) conn[q * 64 + l * 16 + m * 4 + nn] = cn[l][m][nn];
      }
  }
  long id(int i, int j, int k) const {
    return ((long)(k + NG) * s2 + (j + NG)) * s1 + (i + NG);
  }
  long id2(int i, int j) const { return (long)(j + NG) * s1 + (i + NG); }
  // x3 faces lie at the zone-centre (x1, x2), and the metric does not depend on x3.
  const Geom& face_geom(int d, int i, int j) const {
    if (d == 1) return gF1[id2(i, j)];
    if (d == 2) return gF2[id2(i, j)];
    return gC[id2(i, j)];
  }
  bool pole_face(int d, int j) const {
    return d == 2 && ((pole_lo && j == 0) || (pole_hi && j == c.n2));
  }
};

inline real& V(std::vector<real>& a, const Grid& g, int v, int i, int j, int k) {
  return a[v * g.nz + g.id(i, j, k)];
}
inline real Vc(const std::vector<real>& a, const Grid& g, int v, int i, int j, int k) {
  return a[v * g.nz + g.id(i, j, k)];
}

// ------------------------------------------------------------ boundaries --

// Ghost fill, one axis after another (x1, then x2 over the x1 ghosts too,
// then x3 over everything), so edge and corner ghosts are consistent.
//   periodic: wrap;  outflow: copy the nearest interior zone (all prims);
//   polar: mirror across the axis, flipping u~2 and B2;  frozen: untouched.
// nvar variables of array A; flip: bit v set flips variable v across a polar axis.
void fill_ghosts_vars(const Grid& g, std::vector<real>& P, int nvar, unsigned flip_mask) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  for (int v = 0; v < nvar; v++) {
    // x1
    for (int k = 0; k < n3; k++)
      for (int j = 0; j < n2; j++)
        for (int m = 1; m <= NG; m++) {
          int lo = -m, hi = n1 - 1 + m;
          if (g.c.bc[0] == BC_PERIODIC) V(P, g, v, lo, j, k) = V(P, g, v, ((lo % n1) + n1) % n1, j, k);
          else if (g.c.bc[0] == BC_OUTFLOW) V(P, g, v, lo, j, k) = V(P, g, v, 0, j, k);
          if (g.c.bc[1] == BC_PERIODIC) V(P, g, v, hi, j, k) = V(P, g, v, hi % n1, j, k);
          else if (g.c.bc[1] == BC_OUTFLOW) V(P, g, v, hi, j, k) = V(P, g, v, n1 - 1, j, k);
        }
    // x2
    real flip = ((flip_mask >> v) & 1u) ? -1.0 : 1.0;
    for (int k = 0; k < n3; k++)
      for (int i = -NG; i < n1 + NG; i++)
        for (int m = 1; m <= NG; m++) {
          int lo = -m, hi = n2 - 1 + m;
          if (g.c.bc[2] == BC_PERIODIC) V(P, g, v, i, lo, k) = V(P, g, v, i, ((lo % n2) + n2) % n2, k);
          else if (g.c.bc[2] == BC_OUTFLOW) V(P, g, v, i, lo, k) = V(P, g, v, i, 0, k);
          else if (g.c.bc[2] == BC_POLAR) V(P, g, v, i, lo, k) = flip * V(P, g, v, i, m - 1, k);
          if (g.c.bc[3] == BC_PERIODIC) V(P, g, v, i, hi, k) = V(P, g, v, i, hi % n2, k);
          else if (g.c.bc[3] == BC_OUTFLOW) V(P, g, v, i, hi, k) = V(P, g, v, i, n2 - 1, k);
          else if (g.c.bc[3] == BC_POLAR) V(P, g, v, i, hi, k) = flip * V(P, g, v, i, n2 - m, k);
        }
    // x3
    for (int j = -NG; j < n2 + NG; j++)
      for (int i = -NG; i < n1 + NG; i++)
        for (int m = 1; m <= NG; m++) {
          int lo = -m, hi = n3 - 1 + m;
          if (g.c.bc[4] == BC_PERIODIC) V(P, g, v, i, j, lo) = V(P, g, v, i, j, ((lo % n3) + n3) % n3);
          else if (g.c.bc[4] == BC_OUTFLOW) V(P, g, v, i, j, lo) = V(P, g, v, i, j, 0);
          if (g.c.bc[5] == BC_PERIODIC) V(P, g, v, i, j, hi) = V(P, g, v, i, j, hi % n3);
          else if (g.c.bc[5] == BC_OUTFLOW) V(P, g, v, i, j, hi) = V(P, g, v, i, j, n3 - 1);
        }
  }
}

void fill_ghosts(const Grid& g, std::vector<real>& P) {
  fill_ghosts_vars(g, P, NV, (1u << U2) | (1u << B2));
}

// ----------------------------------------------------------------- fluxes --

// Left and right states at the lower face (along d) of zone (i, j, k).
// Donor cell: the two zones' own values.
// Left and right states at the face between zones -1 and 0 of the six
// values q[0..5] = zones -3 .. +2 along the axis.
void recon_one(const real q[6], int recon, real eps, real& qL, real& qR) {
  if (recon == RECON_DONOR) {
    qL = q[2];
    qR = q[3];
  } else if (recon == RECON_MC) {
    qL = q[2] + 0.5 * mc_slope(q[1], q[2], q[3]);
    qR = q[3] - 0.5 * mc_slope(q[2], q[3], q[4]);
  } else if (recon == RECON_VL) {
    qL = q[2] + 0.5 * vl_slope(q[1], q[2], q[3]);
    qR = q[3] - 0.5 * vl_slope(q[2], q[3], q[4]);
  } else if (recon == RECON_WENOZ) {
    qL = wenoz(q[0], q[1], q[2], q[3], q[4], eps);
    qR = wenoz(q[5], q[4], q[3], q[2], q[1], eps);
  } else if (recon == RECON_MP5) {
    qL = mp5(q[0], q[1], q[2], q[3], q[4]);
    qR = mp5(q[5], q[4], q[3], q[2], q[1]);
  } else if (recon == RECON_PPM) {
    real l, r;
    ppm_edges(q[0], q[1], q[2], q[3], q[4], l, r);  // zone -1: its right edge
    qL = r;
    ppm_edges(q[1], q[2], q[3], q[4], q[5], l, r);  // zone 0: its left edge
    qR = l;
  } else if (recon == RECON_PPMX) {
    real l, r;
    ppmx_edges(q[0], q[1], q[2], q[3], q[4], l, r);  // zone -1: its right edge
    qL = r;
    ppmx_edges(q[1], q[2], q[3], q[4], q[5], l, r);  // zone 0: its left edge
    qR = l;
  } else {
    qL = weno5(q[0], q[1], q[2], q[3], q[4], eps);
    qR = weno5(q[5], q[4], q[3], q[2], q[1], eps);
  }
}

// Left and right states at the lower face (along d) of zone (i, j, k) of the
// nvar variables of array A.  Donor cell: the two zones' own values.
void reconstruct_vars(const Grid& g, const std::vector<real>& A, int nvar, int recon, int d, int i, int j,
                      int k, real* qL, real* qR) {
  int di = d == 1, dj = d == 2, dk = d == 3;
  for (int v = 0; v < nvar; v++) {
    real q[6];  // zones -3 .. +2 relative to (i, j, k) along d
    for (int s = -3; s <= 2; s++) q[s + 3] = Vc(A, g, v, i + s * di, j + s * dj, k + s * dk);
    recon_one(q, recon, g.c.weno_eps, qL[v], qR[v]);
  }
}

void reconstruct(const Grid& g, const std::vector<real>& P, int recon, int d, int i, int j, int k,
                 real qL[NV], real qR[NV]) {
  reconstruct_vars(g, P, NV, recon, d, i, j, k, qL, qR);
}

// Local Lax-Friedrichs flux at the lower d-face of zone (i, j, k):
// F = (F_L + F_R)/2 - c_max (U_R - U_L)/2, c_max = max(0, c+_L, c+_R, -c-_L, -c-_R).
// Faces on the polar axis carry no flux (sqrt(-g) = 0 there).
// With face fields phi (face-centred CT), the normal field of both states
// is the face value phi_d / sqrt(-g) at the face.
void face_flux(const Grid& g, const std::vector<real>& P, int recon, int d, int i, int j, int k,
               real F[NV], const std::vector<real>* phi = nullptr) {
  if (g.pole_face(d, j)) {
    for (int v = 0; v < NV; v++) F[v] = 0.0;
    return;
  }
  real qL[NV], qR[NV];
  reconstruct(g, P, recon, d, i, j, k, qL, qR);
  const Geom& G = g.face_geom(d, i, j);
  if (phi) {
    qL[B1 + d - 1] = phi[d - 1][g.id(i, j, k)] / G.gdet;
    qR[B1 + d - 1] = qL[B1 + d - 1];
  }
  FluidState SL, SR;
  fluid_state(qL, G, SL);
  fluid_state(qR, G, SR);
  real FL[NV], FR[NV], UL[NV], UR[NV];
  prim_to_flux(qL, SL, G, g.c.gam, d, FL);
  prim_to_flux(qR, SR, G, g.c.gam, d, FR);
  prim_to_flux(qL, SL, G, g.c.gam, 0, UL);
  prim_to_flux(qR, SR, G, g.c.gam, 0, UR);
  real cpl, cml, cpr, cmr;
  vchar(qL, SL, G, g.c.gam, d, cpl, cml);
  vchar(qR, SR, G, g.c.gam, d, cpr, cmr);
  real cmax = 0.0;
  if (cpl > cmax) cmax = cpl;
  if (cpr > cmax) cmax = cpr;
  if (-cml > cmax) cmax = -cml;
  if (-cmr > cmax) cmax = -cmr;
  for (int v = 0; v < NV; v++) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * cmax * (UR[v] - UL[v]);
}

// Fluxes along every direction on the faces the update and Flux-CT need:
// x1 faces i in [0, n1] over j in [-1, n2], k in [-1, n3] (and cyclically).
void compute_fluxes(const Grid& g, const std::vector<real>& P, std::vector<real> F[3],
                    const std::vector<real>* phi = nullptr) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  for (int d = 1; d <= 3; d++) {
    int lo[3] = {-1, -1, -1}, hi[3] = {n1, n2, n3};  // inclusive
    lo[d - 1] = 0;
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads)
    for (int k = lo[2]; k <= hi[2]; k++)
      for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
          real f[NV];
          face_flux(g, P, g.c.recon, d, i, j, k, f, phi);
          for (int v = 0; v < NV; v++) V(F[d - 1], g, v, i, j, k) = f[v];
        }
  }
}

// Flux-CT (Toth 2000).  The EMF on the edge at the lower corner of zone
// (i, j, k) averages the four face fluxes of the transverse field around it:
//   emf3 = [F1(B2) + F1(B2)_{j-1} - F2(B1) - F2(B1)_{i-1}] / 4
//   emf2 = [F3(B1) + F3(B1)_{i-1} - F1(B3) - F1(B3)_{k-1}] / 4
//   emf1 = [F2(B3) + F2(B3)_{k-1} - F3(B2) - F3(B2)_{j-1}] / 4
// and the field fluxes are rebuilt from edge averages; the normal ones vanish.
// Edges on the polar axis (sqrt(-g) = 0) carry zero emf1 and emf3, consistent
// with the zero flux through the pole faces.
void flux_ct(const Grid& g, std::vector<real> F[3]) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  std::vector<real> e1(g.nz, 0.0), e2(g.nz, 0.0), e3(g.nz, 0.0);
  std::vector<real>& F1 = F[0];
  std::vector<real>& F2 = F[1];
  std::vector<real>& F3 = F[2];
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads)
  for (int k = 0; k <= n3; k++)
    for (int j = 0; j <= n2; j++)
      for (int i = 0; i <= n1; i++) {
        bool pole = (g.pole_lo && j == 0) || (g.pole_hi && j == n2);
        long q = g.id(i, j, k);
        e3[q] = pole ? 0.0
                     : 0.25 * (Vc(F1, g, B2, i, j, k) + Vc(F1, g, B2, i, j - 1, k) -
                               Vc(F2, g, B1, i, j, k) - Vc(F2, g, B1, i - 1, j, k));
        e2[q] = 0.25 * (Vc(F3, g, B1, i, j, k) + Vc(F3, g, B1, i - 1, j, k) -
                        Vc(F1, g, B3, i, j, k) - Vc(F1, g, B3, i, j, k - 1));
        e1[q] = pole ? 0.0
                     : 0.25 * (Vc(F2, g, B3, i, j, k) + Vc(F2, g, B3, i, j, k - 1) -
                               Vc(F3, g, B2, i, j, k) - Vc(F3, g, B2, i, j - 1, k));
      }
  auto E = [&](std::vector<real>& e, int i, int j, int k) -> real { return e[g.id(i, j, k)]; };
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads)
  for (int k = 0; k <= n3; k++)
    for (int j = 0; j <= n2; j++)
      for (int i = 0; i <= n1; i++) {
        if (j < n2 && k < n3) {
          V(F1, g, B1, i, j, k) = 0.0;
          V(F1, g, B2, i, j, k) = 0.5 * (E(e3, i, j, k) + E(e3, i, j + 1, k));
          V(F1, g, B3, i, j, k) = -0.5 * (E(e2, i, j, k) + E(e2, i, j, k + 1));
        }
        if (i < n1 && k < n3) {
          V(F2, g, B1, i, j, k) = -0.5 * (E(e3, i, j, k) + E(e3, i + 1, j, k));
          V(F2, g, B2, i, j, k) = 0.0;
          V(F2, g, B3, i, j, k) = 0.5 * (E(e1, i, j, k) + E(e1, i, j, k + 1));
        }
        if (i < n1 && j < n2) {
          V(F3, g, B1, i, j, k) = 0.5 * (E(e2, i, j, k) + E(e2, i + 1, j, k));
          V(F3, g, B2, i, j, k) = -0.5 * (E(e1, i, j, k) + E(e1, i, j + 1, k));
          V(F3, g, B3, i, j, k) = 0.0;
        }
      }
}

// ------------------------------------------------------- face-centred CT --
// Face-centred constrained transport (Algorithm section: the scheme of Stone
// & Gardiner, edge EMFs with or without upwinding).  The magnetic state is
// the face field phi_d = sqrt(-g) B^d on the lower d-face of every zone; the
// zone-centred B^d is the mean of the zone's two d-faces over sqrt(-g) at its
// centre.  Edge EMFs, E3 = F^1(B^2) = -F^2(B^1) on x1-x2 edges and
// cyclically (E1 = F^2(B^3), E2 = F^3(B^1)):
//  * averaged: the mean of the four face values around the edge;
//  * upwinded (Gardiner & Stone 2005): that mean plus, along each of the two
//    in-plane directions, a quarter of (lower minus upper) EMF gradient
//    across the edge, each gradient the difference of a face value and a
//    zone-centre EMF (from the zone's prims) over half a zone, taken in the
//    zone the mass flux through the adjoining face comes from (the mean of
//    both where that flux is zero).  The sign makes the edge EMF equal the
//    face EMF for flow that varies along one grid direction only.  A face
//    mass flux no larger than 1e-10 of the two zones' mass-current scale,
//    sqrt(-g) rho (|u^t| + sum_d |u^d|) each, counts as zero: its sign
//    would be roundoff (flow along or symmetric about the face, e.g. gas at
//    rest in theta, or the torus's equatorial plane).
// Edges on the polar axis carry zero E1 and E3, as in Flux-CT.  Faces evolve
// by Stokes' theorem: d phi_1/dt = dE3/dx2 - dE2/dx3, d phi_2/dt =
// dE1/dx3 - dE3/dx1, d phi_3/dt = dE2/dx1 - dE1/dx2, so the face divergence
// sum_d (phi_d(+) - phi_d(-))/dx_d keeps its value to roundoff.
enum { CT_FLUX = 0, CT_FACE_AVG = 1, CT_FACE_GS = 2 };

// Ghost faces, axis by axis like the zone ghosts.  Along a face array's own
// axis (faces 0..n are evolved): periodic wraps modulo n, outflow copies the
// boundary face, polar mirrors about the axis face with the sign flipped;
// across it: the zone rules (periodic wrap, outflow copy, polar mirror
// without flip).  Frozen ghosts keep their values.
void fill_face_ghosts(const Grid& g, std::vector<real> phi[3]) {
  for (int d = 0; d < 3; d++) {
    for (int a = 0; a < 3; a++) {
      const int n = g.n[a];
      const int lo_bc = g.c.bc[2 * a], hi_bc = g.c.bc[2 * a + 1];
      const bool normal = a == d;
      const int last = normal ? n : n - 1;   // last valid index along a
      for (int k = -NG; k < g.n[2] + NG; k++)
        for (int j = -NG; j < g.n[1] + NG; j++)
          for (int i = -NG; i < g.n[0] + NG; i++) {
            int idx[3] = {i, j, k};
            // passes over earlier axes cover their ghosts; later axes only their valid range
            bool skip = false;
            for (int b = a + 1; b < 3; b++) {
              int lb = (b == d) ? g.n[b] : g.n[b] - 1;
              if (idx[b] < 0 || idx[b] > lb) skip = true;
            }
            if (skip) continue;
            int x = idx[a];
            if (x >= 0 && x <= last) continue;
            const int bc = x < 0 ? lo_bc : hi_bc;
            int src = x;
            real sgn = 1.0;
            if (bc == BC_PERIODIC) {
              src = ((x % n) + n) % n;  // faces n and 0 coincide
            } else if (bc == BC_OUTFLOW) {
              src = x < 0 ? 0 : last;
            } else if (bc == BC_POLAR) {
              if (normal) {
                src = x < 0 ? -x : 2 * n - x;
                sgn = -1.0;
              } else {
                src = x < 0 ? -1 - x : 2 * n - 1 - x;
              }
            } else {
              continue;  // frozen
            }
            int sidx[3] = {idx[0], idx[1], idx[2]};
            sidx[a] = src;
            phi[d][g.id(i, j, k)] = sgn * phi[d][g.id(sidx[0], sidx[1], sidx[2])];
          }
    }
  }
}

// Edge EMFs at the lower corners of every zone (edges 0..n along each axis)
// from face fluxes F (not Flux-CT corrected) and, for the upwinded scheme,
// zone-centre EMFs from the prims P.
void edge_emfs(const Grid& g, const std::vector<real>& P, const std::vector<real> F[3], int scheme,
               std::vector<real> E[3]) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  for (int c = 0; c < 3; c++) E[c].assign(g.nz, 0.0);
  // zone-centre EMFs over zones -1..n: ec[c] = F^a(B^b) with (a, b) cyclic before c
  std::vector<real> ec[3], cs;  // zone-centre EMFs and mass-current scale
  if (scheme == CT_FACE_GS) {
    for (int c = 0; c < 3; c++) ec[c].assign(g.nz, 0.0);
    cs.assign(g.nz, 0.0);
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads)
    for (int k = -1; k <= n3; k++)
      for (int j = -1; j <= n2; j++)
        for (int i = -1; i <= n1; i++) {
          real p[NV];
          for (int v = 0; v < NV; v++) p[v] = Vc(P, g, v, i, j, k);
          const Geom& G = g.gC[g.id2(i, j)];
          FluidState S;
          fluid_state(p, G, S);
          real f0[NV], f1[NV], f2[NV], f3[NV];
          prim_to_flux(p, S, G, g.c.gam, 0, f0);
          prim_to_flux(p, S, G, g.c.gam, 1, f1);
          prim_to_flux(p, S, G, g.c.gam, 2, f2);
          prim_to_flux(p, S, G, g.c.gam, 3, f3);
          long q = g.id(i, j, k);
          ec[2][q] = f1[B2];  // E3 = F^1(B^2)
          ec[0][q] = f2[B3];  // E1 = F^2(B^3)
          ec[1][q] = f3[B1];  // E2 = F^3(B^1)
          cs[q] = ((fabs(f0[RHO]) + fabs(f1[RHO])) + fabs(f2[RHO])) + fabs(f3[RHO]);
        }
  }
  // upwind choice by the face mass flux, zero within 1e-10 of its zones' scale
  auto up = [](real flux, real scale, real lower, real upper) -> real {
    if (fabs(flux) <= 1e-10 * scale) return 0.5 * (lower + upper);
    return flux > 0.0 ? lower : upper;
  };
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads)
  for (int k = 0; k <= n3; k++)
    for (int j = 0; j <= n2; j++)
      for (int i = 0; i <= n1; i++) {
        const bool pole = (g.pole_lo && j == 0) || (g.pole_hi && j == n2);
        const int x[3] = {i, j, k};
        for (int c = 0; c < 3; c++) {
          if (pole && c != 1) continue;  // E1 and E3 vanish on the axis
          const int a = (c + 1) % 3, b = (c + 2) % 3;  // axes of the plane, cyclic
          const int Bb = B1 + b, Ba = B1 + a;
          auto at = [&](int da, int db, int* out) {
            out[0] = x[0]; out[1] = x[1]; out[2] = x[2];
            out[a] -= da; out[b] -= db;
          };
          int p00[3], p10[3], p01[3], p11[3];  // x, x - e_a, x - e_b, x - e_a - e_b
          at(0, 0, p00); at(1, 0, p10); at(0, 1, p01); at(1, 1, p11);
          auto ID = [&](const int* q) { return g.id(q[0], q[1], q[2]); };
          // face values: on a-faces F^a(B^b), on b-faces -F^b(B^a)
          const real ea0 = F[a][Bb * g.nz + ID(p00)], ea1 = F[a][Bb * g.nz + ID(p01)];
          const real eb0 = -F[b][Ba * g.nz + ID(p00)], eb1 = -F[b][Ba * g.nz + ID(p10)];
          real e = 0.25 * (((ea0 + ea1) + eb0) + eb1);
          if (scheme == CT_FACE_GS) {
            const std::vector<real>& C = ec[c];
            // along b, at the edge's a-position: zones in column x (upper a) or x - e_a
            const real fa0 = F[a][RHO * g.nz + ID(p00)], fa1 = F[a][RHO * g.nz + ID(p01)];
            const real sa0 = cs[ID(p10)] + cs[ID(p00)], sa1 = cs[ID(p11)] + cs[ID(p01)];
            const real dbp = up(fa0, sa0, C[ID(p10)] - eb1, C[ID(p00)] - eb0);
            const real dbm = up(fa1, sa1, eb1 - C[ID(p11)], eb0 - C[ID(p01)]);
            // along a, at the edge's b-position: zones in row x (upper b) or x - e_b
            const real fb0 = F[b][RHO * g.nz + ID(p00)], fb1 = F[b][RHO * g.nz + ID(p10)];
            const real sb0 = cs[ID(p01)] + cs[ID(p00)], sb1 = cs[ID(p11)] + cs[ID(p10)];
            const real dap = up(fb0, sb0, C[ID(p01)] - ea1, C[ID(p00)] - ea0);
            const real dam = up(fb1, sb1, ea1 - C[ID(p11)], ea0 - C[ID(p10)]);
            e = e + 0.25 * (dbm - dbp) + 0.25 * (dam - dap);
          }
          E[c][g.id(i, j, k)] = e;
        }
      }
}

// Face update of one stage: phi_out = phi_base + h (Stokes' rate), over the
// evolved faces (0..n along the face's axis, interior across it).
void face_update(const Grid& g, const std::vector<real> E[3], const std::vector<real> base[3], real h,
                 std::vector<real> out[3]) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  auto e = [&](int c, int i, int j, int k) { return E[c][g.id(i, j, k)]; };
  for (int d = 0; d < 3; d++) out[d] = base[d];
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads)
  for (int k = 0; k <= n3; k++)
    for (int j = 0; j <= n2; j++)
      for (int i = 0; i <= n1; i++) {
        long q = g.id(i, j, k);
        if (j < n2 && k < n3) {
          real r = (e(2, i, j + 1, k) - e(2, i, j, k)) / g.dx[1] - (e(1, i, j, k + 1) - e(1, i, j, k)) / g.dx[2];
          out[0][q] = base[0][q] + h * r;
        }
        if (i < n1 && k < n3) {
          real r = (e(0, i, j, k + 1) - e(0, i, j, k)) / g.dx[2] - (e(2, i + 1, j, k) - e(2, i, j, k)) / g.dx[0];
          out[1][q] = base[1][q] + h * r;
        }
        if (i < n1 && j < n2) {
          real r = (e(1, i + 1, j, k) - e(1, i, j, k)) / g.dx[0] - (e(0, i, j + 1, k) - e(0, i, j, k)) / g.dx[1];
          out[2][q] = base[2][q] + h * r;
        }
      }
}

// Zone-centred conserved field of zone (i, j, k): the mean of its two faces.
inline void cell_field(const Grid& g, const std::vector<real> phi[3], int i, int j, int k, real UB[3]) {
  UB[0] = 0.5 * (phi[0][g.id(i, j, k)] + phi[0][g.id(i + 1, j, k)]);
  UB[1] = 0.5 * (phi[1][g.id(i, j, k)] + phi[1][g.id(i, j + 1, k)]);
  UB[2] = 0.5 * (phi[2][g.id(i, j, k)] + phi[2][g.id(i, j, k + 1)]);
}

// ------------------------------------------------------- source, update --

// Geometric source sqrt(-g) T^k_l Gamma^l_{nu k} for the four momentum-energy
// slots (the energy equation has rest mass removed, which has no source).
void source_point(const Geom& G, const real* cn, real gam, const real P[NV], real S[NV]) {
  FluidState st;
  fluid_state(P, G, st);
  real T[4][4];
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) T[m][n] = tmunu(P, st, gam, m, n);
  for (int v = 0; v < NV; v++) S[v] = 0.0;
  for (int nu = 0; nu < 4; nu++) {
    real s = 0.0;
    for (int k = 0; k < 4; k++)
      for (int l = 0; l < 4; l++) s += T[k][l] * cn[l * 16 + nu * 4 + k];
    S[UU + nu] = G.gdet * s;
  }
}

void source(const Grid& g, const real P[NV], int i, int j, real S[NV]) {
  source_point(g.gC[g.id2(i, j)], &g.conn[g.id2(i, j) * 64], g.c.gam, P, S);
}

// ------------------------------------------------------------------ U -> P --

// 1D_W inversion (Noble et al. 2006): with D = alpha U_rho/sqrt(-g),
// Q_mu = alpha T^t_mu, Bn^i = alpha B^i and n_mu = (-alpha, 0, 0, 0), solve
//   f(W) = Q.n + W - p(W, v^2) + Bn^2 (1 + v^2)/2 - (Q.Bn)^2/(2 W^2) = 0
// with v^2(W) = [Qt^2 W^2 + (Q.Bn)^2 (Bn^2 + 2W)] / [(Bn^2 + W)^2 W^2] and
// p = (gam-1)/gam [W (1 - v^2) - D sqrt(1 - v^2)], by Newton from the guess's
// W = (rho + gam u) gamma^2, to |dW/W| < tol (at most maxit iterations) and
// one further iteration.  A starting W with v^2 >= 1 is doubled until
// v^2 < 1, and steps that would leave W > 0, v^2 < 1 are halved.  Returns 0 on success; on failure the hydro prims
// are the guess.  B^i = U_B^i / sqrt(-g) in every case.
int u_to_p(const orc_cfg& c, const Geom& G, const real U[NV], const real guess[NV], real P[NV]) {
  const real gam = c.gam;
  for (int k = 0; k < 3; k++) P[B1 + k] = U[B1 + k] / G.gdet;
  real alpha = G.alpha;
  real D = alpha * U[RHO] / G.gdet;
  real Qcov[4];
  Qcov[0] = alpha * (U[UU] / G.gdet - U[RHO] / G.gdet);
  for (int i = 1; i < 4; i++) Qcov[i] = alpha * U[UU + i] / G.gdet;
  real Bn[4] = {0.0, alpha * P[B1], alpha * P[B2], alpha * P[B3]};
  real ncov[4] = {-alpha, 0.0, 0.0, 0.0};
  real ncon[4], Qcon[4];
  for (int m = 0; m < 4; m++) {
    ncon[m] = 0.0;
    Qcon[m] = 0.0;
    for (int n = 0; n < 4; n++) {
      ncon[m] += G.gcon[m][n] * ncov[n];
      Qcon[m] += G.gcon[m][n] * Qcov[n];
    }
  }
  real Qdotn = 0.0, QdotQ = 0.0, QdotB = 0.0, Bsq = 0.0;
  for (int m = 0; m < 4; m++) {
    Qdotn += Qcov[m] * ncon[m];
    QdotQ += Qcov[m] * Qcon[m];
  }
  for (int i = 1; i < 4; i++) {
    QdotB += Qcov[i] * Bn[i];
    for (int j = 1; j < 4; j++) Bsq += G.gcov[i][j] * Bn[i] * Bn[j];
  }
  // Qt is the projection of Q orthogonal to n, a spacelike vector: a negative
  // square can only be roundoff (a fluid at rest with the normal observer).
  real Qtsq = QdotQ + Qdotn * Qdotn;
  if (Qtsq < 0.0) Qtsq = 0.0;
  real QB2 = QdotB * QdotB;
  const real gfac = (gam - 1.0) / gam;

  auto failed = [&]() {
    for (int v = 0; v < 5; v++) P[v] = guess[v];
    return 1;
  };
  auto vsq_of = [&](real W) {
    return (Qtsq * W * W + QB2 * (Bsq + 2.0 * W)) / ((Bsq + W) * (Bsq + W) * W * W);
  };
  auto newton_step = [&](real W) {
    real v2 = vsq_of(W);
    real sq = sqrt(1.0 - v2);
    real p = gfac * (W * (1.0 - v2) - D * sq);
    real f = Qdotn + W - p + 0.5 * Bsq * (1.0 + v2) - QB2 / (2.0 * W * W);
    real dv2 = -2.0 * (Qtsq + QB2 * (3.0 * W * W + 3.0 * W * Bsq + Bsq * Bsq) / (W * W * W)) /
               ((W + Bsq) * (W + Bsq) * (W + Bsq));
    real dpdW = gfac * (1.0 - v2);
    real dpdv2 = gfac * (-W + D / (2.0 * sq));
    real df = 1.0 - (dpdW + dpdv2 * dv2) + 0.5 * Bsq * dv2 + QB2 / (W * W * W);
    return -f / df;
  };

  // initial W from the guess prims
  real qsq = 0.0;
  for (int i = 1; i < 4; i++)
    for (int j = 1; j < 4; j++) qsq += G.gcov[i][j] * guess[U1 + i - 1] * guess[U1 + j - 1];
  real W = (guess[RHO] + gam * guess[UU]) * (1.0 + qsq);
  // v^2(W) falls with W: a guess below the physical range is doubled into it.
  for (int b = 0; b < 60 && !(vsq_of(W) < 1.0); b++) W = 2.0 * W;
  bool conv = false;
  for (int it = 0; it < c.newton_maxit; it++) {
    real dW = newton_step(W);
    real Wn = W + dW;
    // A step that leaves the physical range (W <= 0 or v^2 >= 1) is halved
    // until it is back inside, at most 20 times.
    for (int b = 0; b < 20 && !(Wn > 0.0 && vsq_of(Wn) < 1.0); b++) {
      dW = 0.5 * dW;
      Wn = W + dW;
    }
    if (!isfinite((real)Wn) || Wn <= 0.0) return failed();
    W = Wn;
    if (fabs(dW) < c.newton_tol * fabs(W)) { conv = true; break; }
  }
  if (!conv) return failed();
  W = W + newton_step(W);
  if (!isfinite((real)W) || W <= 0.0) return failed();

  real v2 = vsq_of(W);
  if (!(v2 >= 0.0 && v2 < 1.0)) return failed();
  real gamma = 1.0 / sqrt(1.0 - v2);
  real rho = D / gamma;
  real u = (W * (1.0 - v2) - rho) / gam;
  if (!(rho > 0.0) || !(u > 0.0)) return failed();
  real pre = gamma / (W + Bsq);
  real ut[3];
  for (int i = 1; i < 4; i++) {
    real Qt = Qcon[i] + ncon[i] * Qdotn;
    ut[i - 1] = pre * (Qt + QdotB * Bn[i] / W);
    if (!isfinite((real)ut[i - 1])) return failed();
  }
  P[RHO] = rho;
  P[UU] = u;
  P[U1] = ut[0];
  P[U2] = ut[1];
  P[U3] = ut[2];
  return 0;
}

// Kastaun et al. (2021) recovery, the robust alternative to 1D_W the
// Algorithm section names.  With the same normal-frame quantities as above
// (D, the spatial projection S of Q, E = -Q.n, Bn), scaled by D:
//   r^2 = S.S / D^2,  b^2 = Bn.Bn / D,  rb = S.Bn / D^(3/2),  q = E/D - 1,
// every fluid quantity follows from mu = 1/(h W) (h the specific enthalpy,
// W the normal-frame Lorentz factor):
//   x = 1/(1 + mu b^2),  rbar^2 = x^2 r^2 + mu x (1 + x) rb^2,
//   qbar = q - b^2/2 - mu^2 x^2 (b^2 r^2 - rb^2)/2,
//   v^2 = min(mu^2 rbar^2, vmax^2),  W = 1/sqrt(1 - v^2),  rho = D/W,
//   eps = max(W (qbar - mu rbar^2) + v^2 W^2/(1 + W), 0),
//   a = p/(rho (1 + eps)) = (gam - 1) eps/(1 + eps),
//   nu = max((1 + a)(1 + eps)/W, (1 + a)(1 + qbar - mu rbar^2)),
// and mu is the root of f(mu) = mu - 1/(nu + mu rbar^2).  Since h >= 1,
// mu <= mu+ with mu+ sqrt(1 + rbar^2(mu+)) = 1; f < 0 at 0 and f >= 0 at mu+,
// so both roots are bracketed and found by the Illinois (modified regula
// falsi) iteration, to |d mu| <= tol mu.  Then u = rho eps and
// u~^i = W v^i with v^i = mu x (S^i/D + mu rb b^i).  No guess is needed; a
// failure (no bracket, no convergence, eps <= 0, non-finite) keeps the
// guess's hydro prims as 1D_W does.
int u_to_p_kastaun(const orc_cfg& c, const Geom& G, const real U[NV], const real guess[NV],
                   real P[NV]) {
  const real gam = c.gam;
  for (int k = 0; k < 3; k++) P[B1 + k] = U[B1 + k] / G.gdet;
  auto failed = [&]() {
    for (int v = 0; v < 5; v++) P[v] = guess[v];
    return 1;
  };
  real alpha = G.alpha;
  real D = alpha * U[RHO] / G.gdet;
  if (!(D > 0.0) || !isfinite((real)D)) return failed();
  real Qcov[4];
  Qcov[0] = alpha * (U[UU] / G.gdet - U[RHO] / G.gdet);
  for (int i = 1; i < 4; i++) Qcov[i] = alpha * U[UU + i] / G.gdet;
  real Bn[4] = {0.0, alpha * P[B1], alpha * P[B2], alpha * P[B3]};
  real ncov[4] = {-alpha, 0.0, 0.0, 0.0};
  real ncon[4], Qcon[4];
  for (int m = 0; m < 4; m++) {
    ncon[m] = 0.0;
    Qcon[m] = 0.0;
    for (int n = 0; n < 4; n++) {
      ncon[m] += G.gcon[m][n] * ncov[n];
      Qcon[m] += G.gcon[m][n] * Qcov[n];
    }
  }
  real Qdotn = 0.0, QdotQ = 0.0, QdotB = 0.0, Bsq = 0.0;
  for (int m = 0; m < 4; m++) {
    Qdotn += Qcov[m] * ncon[m];
    QdotQ += Qcov[m] * Qcon[m];
  }
  for (int i = 1; i < 4; i++) {
    QdotB += Qcov[i] * Bn[i];
    for (int j = 1; j < 4; j++) Bsq += G.gcov[i][j] * Bn[i] * Bn[j];
  }
  real Ssq = QdotQ + Qdotn * Qdotn;
  if (Ssq < 0.0) Ssq = 0.0;
  const real r2 = Ssq / (D * D), b2 = Bsq / D, rb = QdotB / (D * sqrt(D)), q = -Qdotn / D - 1.0;
  const real rb2 = rb * rb;
  const real vmax2 = 1.0 - 1.0 / (c.kastaun_wmax * c.kastaun_wmax);

  struct State { real x, rbar2, qbar, v2, W, eps, nu; };
  auto state = [&](real mu) {
    State s;
    s.x = 1.0 / (1.0 + mu * b2);
    s.rbar2 = s.x * s.x * r2 + mu * s.x * (1.0 + s.x) * rb2;
    s.qbar = q - 0.5 * b2 - 0.5 * (mu * mu) * (s.x * s.x) * (b2 * r2 - rb2);
    s.v2 = mu * mu * s.rbar2;
    if (s.v2 > vmax2) s.v2 = vmax2;
    s.W = 1.0 / sqrt(1.0 - s.v2);
    s.eps = s.W * (s.qbar - mu * s.rbar2) + s.v2 * s.W * s.W / (1.0 + s.W);
    if (s.eps < 0.0) s.eps = 0.0;
    real a = (gam - 1.0) * s.eps / (1.0 + s.eps);
    real nuA = (1.0 + a) * (1.0 + s.eps) / s.W, nuB = (1.0 + a) * (1.0 + s.qbar - mu * s.rbar2);
    s.nu = nuA > nuB ? nuA : nuB;
    return s;
  };
  auto f = [&](real mu) {
    State s = state(mu);
    return mu - 1.0 / (s.nu + mu * s.rbar2);
  };
  auto fa = [&](real mu) {
    real x = 1.0 / (1.0 + mu * b2);
    real rbar2 = x * x * r2 + mu * x * (1.0 + x) * rb2;
    return mu * sqrt(1.0 + rbar2) - 1.0;
  };
  // Illinois iteration for a root of g in [a, b] with g(a) < 0 < g(b): stop
  // when an iterate moves by at most tol times itself or hits g = 0.
  auto illinois = [&](auto g, real a, real b, real ga, real gb, real tol, real& root) {
    int side = 0;
    real prev = b;
    for (int it = 0; it < 4 * c.newton_maxit; it++) {
      real m = (a * gb - b * ga) / (gb - ga);
      if (!(m > a && m < b)) m = 0.5 * (a + b);
      real gm = g(m);
      if (gm == 0.0 || fabs(m - prev) <= tol * m) { root = m; return true; }
      prev = m;
      if (gm < 0.0) {
        a = m; ga = gm;
        if (side == -1) gb = 0.5 * gb;
        side = -1;
      } else {
        b = m; gb = gm;
        if (side == 1) ga = 0.5 * ga;
        side = 1;
      }
    }
    return false;
  };
  real mup;
  if (!illinois(fa, 0.0, 1.0, -1.0, fa(1.0), 1e-12, mup)) return failed();
  mup = mup * (1.0 + 1e-10);
  if (mup > 1.0) mup = 1.0;
  real f0 = f(0.0), f1 = f(mup);
  if (!(f0 < 0.0) || !(f1 >= 0.0)) return failed();
  real mu;
  if (f1 == 0.0)
    mu = mup;
  else if (!illinois(f, 0.0, mup, f0, f1, c.newton_tol, mu))
    return failed();
  State s = state(mu);
  real rho = D / s.W;
  real u = rho * s.eps;
  // eps clamped at 0 is the method's own answer for an energy below the
  // cold state; with floors on it stands, and the energy floor raises u
  if (!(rho > 0.0) || !(u > 0.0 || (c.floors && u == 0.0)) || !isfinite((real)u)) return failed();
  real pre = s.W * mu * s.x / D;
  real ut[3];
  for (int i = 1; i < 4; i++) {
    real St = Qcon[i] + ncon[i] * Qdotn;
    ut[i - 1] = pre * (St + mu * QdotB * Bn[i] / D);
    if (!isfinite((real)ut[i - 1])) return failed();
  }
  P[RHO] = rho;
  P[UU] = u;
  P[U1] = ut[0];
  P[U2] = ut[1];
  P[U3] = ut[2];
  return 0;
}

// The implicit solver's Newton-Raphson used as the recovery (Implicit Solver
// section: with all fluid variables implicit and only ideal sources it
// solves U(P) = U* zone by zone).  Unknowns x = (rho, u, u~1, u~2, u~3), B
// from U*; residual R(x) = (U(x) - U*)_{0..4} / s, s the largest |U*_k|;
// Jacobian by forward differences (secant) with steps h_k = 1e-7 max(|x_k|,
// f_k), f = (0, 0, 1e-3, 1e-3, 1e-3); the step solves J dx = -R by a QR
// decomposition with column pivoting (Householder reflections, the column
// of largest remaining norm first, ties to the lower index); backtracking
// line search: lambda = 1, 1/2, ... (at most 8 halvings) until rho and u
// stay positive and |R| decreases (the last try is taken if none does, if
// rho and u are positive).  Stop when every |lambda dx_k| <= tol max(|x_k|,
// f_k), tol = max(newton_tol, 1e-12), or after maxit iterations (failure);
// failure (also non-finite, rho <= 0, u <= 0) keeps the guess's hydro
// prims.  The 1e-12 floor: near the root the residual's roundoff makes
// steps of ~1e-13 relative, so a smaller tolerance is never met; the step
// that meets it has already brought x to roundoff (the secant Jacobian is
// accurate to ~1e-7, so each step shrinks the error by about that much).
void implicit_residual(const orc_cfg& c, const Geom& G, const real x[5], const real B[3], const real Us[NV],
                       real scale, real R[5]) {
  real P[NV] = {x[0], x[1], x[2], x[3], x[4], B[0], B[1], B[2]};
  FluidState S;
  fluid_state(P, G, S);
  real U[NV];
  prim_to_flux(P, S, G, c.gam, 0, U);
  for (int k = 0; k < 5; k++) R[k] = (U[k] - Us[k]) / scale;
}

// Solve A y = b (5 x 5) by Householder QR with column pivoting; false if
// the matrix is numerically singular or non-finite.
bool qr_pivot_solve(real A[5][5], real b[5], real y[5]) {
  int perm[5] = {0, 1, 2, 3, 4};
  real cn[5];
  for (int j = 0; j < 5; j++) {
    cn[j] = 0.0;
    for (int i = 0; i < 5; i++) cn[j] += A[i][j] * A[i][j];
  }
  for (int k = 0; k < 5; k++) {
    // pivot: the column of largest remaining norm (rows k..4)
    int best = k;
    for (int j = k + 1; j < 5; j++)
      if (cn[j] > cn[best]) best = j;
    if (best != k) {
      for (int i = 0; i < 5; i++) std::swap(A[i][k], A[i][best]);
      std::swap(cn[k], cn[best]);
      std::swap(perm[k], perm[best]);
    }
    real nrm = 0.0;
    for (int i = k; i < 5; i++) nrm += A[i][k] * A[i][k];
    nrm = sqrt(nrm);
    if (!(nrm > 0.0) || !isfinite((real)nrm)) return false;
    real alpha = A[k][k] > 0.0 ? -nrm : nrm;
    // v = a_k - alpha e_k; H = I - 2 v v^T / (v^T v)
    real v[5];
    for (int i = 0; i < 5; i++) v[i] = i < k ? 0.0 : A[i][k];
    v[k] = v[k] - alpha;
    real vv = 0.0;
    for (int i = k; i < 5; i++) vv += v[i] * v[i];
    if (!(vv > 0.0)) return false;
    for (int j = k; j < 5; j++) {
      real d = 0.0;
      for (int i = k; i < 5; i++) d += v[i] * A[i][j];
      real f = 2.0 * d / vv;
      for (int i = k; i < 5; i++) A[i][j] = A[i][j] - f * v[i];
    }
    real d = 0.0;
    for (int i = k; i < 5; i++) d += v[i] * b[i];
    real f = 2.0 * d / vv;
    for (int i = k; i < 5; i++) b[i] = b[i] - f * v[i];
    // remaining column norms (rows k+1..4)
    for (int j = k + 1; j < 5; j++) {
      cn[j] = 0.0;
      for (int i = k + 1; i < 5; i++) cn[j] += A[i][j] * A[i][j];
    }
  }
  real z[5];
  for (int i = 4; i >= 0; i--) {
    real t = b[i];
    for (int j = i + 1; j < 5; j++) t = t - A[i][j] * z[j];
    if (!(fabs(A[i][i]) > 0.0)) return false;
    z[i] = t / A[i][i];
  }
  for (int k = 0; k < 5; k++) y[perm[k]] = z[k];
  for (int k = 0; k < 5; k++)
    if (!isfinite((real)y[k])) return false;
  return true;
}

// The Newton iteration of the implicit solver on the five hydro prims x
// from the guess x0 (both positive in rho and u): residual(x, R) fills the
// scaled residual R[5].  Returns 0 with the root in x, 1 on failure.
template <typename Res>
int newton_hydro(const orc_cfg& c, const real x0[5], Res residual, real x[5]) {
  const real fl[5] = {0.0, 0.0, 1e-3, 1e-3, 1e-3};
  for (int k = 0; k < 5; k++) x[k] = x0[k];
  if (!(x[0] > 0.0) || !(x[1] > 0.0)) return 1;
  real R[5];
  residual(x, R);
  real r2 = 0.0;
  for (int k = 0; k < 5; k++) r2 += R[k] * R[k];
  bool conv = false;
  const real tol = c.newton_tol > 1e-12 ? c.newton_tol : 1e-12;
  for (int it = 0; it < c.newton_maxit && !conv; it++) {
    real J[5][5];
    for (int k = 0; k < 5; k++) {
      real ax = fabs(x[k]);
      real h = 1e-7 * (ax > fl[k] ? ax : fl[k]);
      real xp[5];
      for (int m = 0; m < 5; m++) xp[m] = x[m];
      xp[k] = x[k] + h;
      real Rp[5];
      residual(xp, Rp);
      real hh = xp[k] - x[k];
      for (int m = 0; m < 5; m++) J[m][k] = (Rp[m] - R[m]) / hh;
    }
    real rhs[5], dx[5];
    for (int m = 0; m < 5; m++) rhs[m] = -R[m];
    if (!qr_pivot_solve(J, rhs, dx)) return 1;
    real lam = 1.0, xn[5], Rn[5], rn2 = 0.0;
    bool ok = false;
    for (int ls = 0; ls <= 8; ls++) {
      for (int m = 0; m < 5; m++) xn[m] = x[m] + lam * dx[m];
      if (xn[0] > 0.0 && xn[1] > 0.0) {
        residual(xn, Rn);
        rn2 = 0.0;
        for (int m = 0; m < 5; m++) rn2 += Rn[m] * Rn[m];
        ok = isfinite((real)rn2);
        if (ok && rn2 < r2) break;
      } else {
        ok = false;
      }
      if (ls < 8) lam = 0.5 * lam;
    }
    if (!ok) return 1;
    conv = true;
    for (int m = 0; m < 5; m++) {
      real ax = fabs(xn[m]);
      if (fabs(xn[m] - x[m]) > tol * (ax > fl[m] ? ax : fl[m])) conv = false;
      x[m] = xn[m];
      R[m] = Rn[m];
    }
    r2 = rn2;
  }
  if (!conv) return 1;
  for (int k = 0; k < 5; k++)
    if (!isfinite((real)x[k])) return 1;
  return 0;
}

int u_to_p_implicit(const orc_cfg& c, const Geom& G, const real U[NV], const real guess[NV], real P[NV]) {
  for (int k = 0; k < 3; k++) P[B1 + k] = U[B1 + k] / G.gdet;
  auto failed = [&]() {
    for (int v = 0; v < 5; v++) P[v] = guess[v];
    return 1;
  };
  const real B[3] = {P[B1], P[B2], P[B3]};
  real scale = 0.0;
  for (int k = 0; k < 5; k++)
    if (fabs(U[k]) > scale) scale = fabs(U[k]);
  if (!(scale > 0.0) || !isfinite((real)scale)) return failed();
  real x[5];
  auto res = [&](const real xx[5], real R[5]) { implicit_residual(c, G, xx, B, U, scale, R); };
  if (newton_hydro(c, guess, res, x)) return failed();
  for (int k = 0; k < 5; k++) P[k] = x[k];
  return 0;
}

int invert(const orc_cfg& c, const Geom& G, const real U[NV], const real guess[NV], real P[NV]) {
  if (c.inverter == 2) return u_to_p_implicit(c, G, U, guess, P);
  return c.inverter == 1 ? u_to_p_kastaun(c, G, U, guess, P) : u_to_p(c, G, U, guess, P);
}

// ---------------------------------------------------------------- floors --
// Floors and ceilings (Physics section: when the density or internal energy
// falls below set values, or too far below the magnetic pressure, material
// and energy are injected, most commonly in the drift frame).  The paper
// gives no values or formulas; the readings here:
//   rho_fl = max(rho_min_geom r^-3/2, b^2/bsq_over_rho_max),
//   u_fl   = max(u_min_geom r^-5/2,   b^2/bsq_over_u_max),
// r = exp(x1) in modified KS and 1 in flat space.  A zone below either gets
// drho = max(rho_fl - rho, 0), du = max(u_fl - u, 0) of new material that
// moves with the drift velocity, the part of the fluid's normal-frame
// velocity v perpendicular to B (v_D = v - (v.B) B/B.B, spatial metric; the
// fluid velocity itself where B = 0): the new material's conserved variables
// are added to the zone's and the sum is inverted with the floored prims as
// the guess (the field is kept as it was).  If that inversion fails, the
// floored prims themselves are kept (fluid-frame injection).  Then the
// ceilings: a normal-frame Lorentz factor above gamma_max scales u~ down to
// it, and u/rho above u_over_rho_max lowers u.  Returns a mask of what acted.
enum { FL_RHO = 1, FL_U = 2, FL_FLUID_FRAME = 4, FL_GAMMA = 8, FL_TEMP = 16 };

real spatial_dot(const Geom& G, const real a[3], const real b[3]) {
  real s = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) s += G.gcov[i + 1][j + 1] * a[i] * b[j];
  return s;
}

int apply_floors(const orc_cfg& c, const Geom& G, real x1, real P[NV]) {
  const real r = c.metric == KERR_MKS ? exp(x1) : 1.0;
  const real sr = sqrt(r);
  FluidState S;
  fluid_state(P, G, S);
  real rho_fl = c.rho_min_geom / (r * sr);
  real u_fl = c.u_min_geom / (r * r * sr);
  real rb = S.bsq / c.bsq_over_rho_max, ub = S.bsq / c.bsq_over_u_max;
  if (rb > rho_fl) rho_fl = rb;
  if (ub > u_fl) u_fl = ub;
  real drho = rho_fl - P[RHO], du = u_fl - P[UU];
  if (drho < 0.0) drho = 0.0;
  if (du < 0.0) du = 0.0;
  int mask = 0;
  if (drho > 0.0 || du > 0.0) {
    mask |= (drho > 0.0 ? FL_RHO : 0) | (du > 0.0 ? FL_U : 0);
    real ut[3] = {P[U1], P[U2], P[U3]}, B[3] = {P[B1], P[B2], P[B3]};
    real gamma = sqrt(1.0 + spatial_dot(G, ut, ut));
    real v[3], vd[3];
    for (int i = 0; i < 3; i++) v[i] = ut[i] / gamma;
    real BB = spatial_dot(G, B, B);
    if (BB > 0.0) {
      real vB = spatial_dot(G, v, B);
      for (int i = 0; i < 3; i++) vd[i] = v[i] - vB * B[i] / BB;
    } else {
      for (int i = 0; i < 3; i++) vd[i] = v[i];
    }
    real gd = 1.0 / sqrt(1.0 - spatial_dot(G, vd, vd));
    real Pd[NV] = {drho, du, gd * vd[0], gd * vd[1], gd * vd[2], 0.0, 0.0, 0.0};
    real U[NV], dU[NV], guess[NV], Pn[NV];
    FluidState Sd;
    fluid_state(Pd, G, Sd);
    prim_to_flux(P, S, G, c.gam, 0, U);
    prim_to_flux(Pd, Sd, G, c.gam, 0, dU);
    for (int v = 0; v < NV; v++) {
      U[v] = U[v] + dU[v];
      guess[v] = P[v];
    }
    guess[RHO] = P[RHO] + drho;
    guess[UU] = P[UU] + du;
    if (invert(c, G, U, guess, Pn) == 0) {
      for (int v = 0; v < 5; v++) P[v] = Pn[v];
    } else {
      for (int v = 0; v < 5; v++) P[v] = guess[v];
      mask |= FL_FLUID_FRAME;
    }
  }
  real ut[3] = {P[U1], P[U2], P[U3]};
  real gamma = sqrt(1.0 + spatial_dot(G, ut, ut));
  if (gamma > c.gamma_max) {
    real f = sqrt((c.gamma_max * c.gamma_max - 1.0) / (gamma * gamma - 1.0));
    for (int i = 0; i < 3; i++) P[U1 + i] = ut[i] * f;
    mask |= FL_GAMMA;
  }
  if (P[UU] > c.u_over_rho_max * P[RHO]) {
    P[UU] = c.u_over_rho_max * P[RHO];
    mask |= FL_TEMP;
  }
  return mask;
}

// ------------------------------------------------------------------ step --

void cons_at(const Grid& g, const real P[NV], int i, int j, real U[NV]) {
  const Geom& G = g.gC[g.id2(i, j)];
  FluidState S;
  fluid_state(P, G, S);
  prim_to_flux(P, S, G, g.c.gam, 0, U);
}

// dU/dt = -[(dF1/dx1 + dF2/dx2) + dF3/dx3] + S at zone (i, j, k).
void rhs(const Grid& g, const std::vector<real> F[3], const real P[NV], int i, int j, int k, real L[NV]) {
  real S[NV];
  source(g, P, i, j, S);
  for (int v = 0; v < NV; v++) {
    real d1 = (Vc(F[0], g, v, i + 1, j, k) - Vc(F[0], g, v, i, j, k)) / g.dx[0];
    real d2 = (Vc(F[1], g, v, i, j + 1, k) - Vc(F[1], g, v, i, j, k)) / g.dx[1];
    real d3 = (Vc(F[2], g, v, i, j, k + 1) - Vc(F[2], g, v, i, j, k)) / g.dx[2];
    L[v] = -((d1 + d2) + d3) + S[v];
  }
}

// Counters of the last orc_run: failed inversions, zones floors acted on,
// zones whose fluxes the first-order correction replaced, floor injections
// that fell back to the fluid frame.
struct RunStats { long fails, floor_hits, fofc_zones, fluid_frame; };
RunStats g_stats;

// Update every interior zone of one stage from the Flux-CT fluxes F:
// U = U(Pin) + dt L (stage 1; Un and U1v keep U(Pin) and U) or
// U = (Un + U1v)/2 + dt L/2 (stage 2), then U_to_P with the stage input as the
// guess, then floors (stage 1 stores the floored prims' U in U1v).  mark (if
// not null) gets 1 where the inversion failed or floors acted; the counters
// add only when count is set.
void update_pass(const Grid& g, const std::vector<real>& Pin, const std::vector<real> F[3], int stage,
                 real dt, std::vector<real>& Un, std::vector<real>& U1v, std::vector<real>& Pout,
                 int* flags, std::vector<char>* mark, bool count,
                 const std::vector<real>* phi_new = nullptr) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  long fails = 0, hits = 0, fluid = 0;
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads) reduction(+ : fails, hits, fluid)
  for (int k = 0; k < n3; k++)
    for (int j = 0; j < n2; j++)
      for (int i = 0; i < n1; i++) {
        real p[NV], L[NV], Unew[NV], guess[NV], pn[NV];
        for (int v = 0; v < NV; v++) p[v] = Vc(Pin, g, v, i, j, k);
        rhs(g, F, p, i, j, k, L);
        if (stage == 0) {
          real u0[NV];
          cons_at(g, p, i, j, u0);
          const real h = g.c.integrator == 1 ? 0.5 * dt : dt;  // the predictor takes half a step
          for (int v = 0; v < NV; v++) {
            Unew[v] = u0[v] + h * L[v];
            V(Un, g, v, i, j, k) = u0[v];
          }
        } else if (g.c.integrator == 1) {  // corrector: U^n + dt L(P*)
          for (int v = 0; v < NV; v++) Unew[v] = Vc(Un, g, v, i, j, k) + dt * L[v];
        } else {
          for (int v = 0; v < NV; v++)
            Unew[v] = 0.5 * (Vc(Un, g, v, i, j, k) + Vc(U1v, g, v, i, j, k)) + 0.5 * (dt * L[v]);
        }
        if (phi_new) {  // face-centred CT: the zone's field is the mean of its new faces
          real UB[3];
          cell_field(g, phi_new, i, j, k, UB);
          for (int d = 0; d < 3; d++) Unew[B1 + d] = UB[d];
        }
        if (stage == 0)
          for (int v = 0; v < NV; v++) V(U1v, g, v, i, j, k) = Unew[v];
        for (int v = 0; v < NV; v++) guess[v] = p[v];
        int f = invert(g.c, g.gC[g.id2(i, j)], Unew, guess, pn);
        int fl = 0;
        if (g.c.floors) {
          fl = apply_floors(g.c, g.gC[g.id2(i, j)], g.xmin[0] + (i + 0.5) * g.dx[0], pn);
          if (fl && stage == 0) {
            real u1[NV];
            cons_at(g, pn, i, j, u1);
            for (int v = 0; v < NV; v++) V(U1v, g, v, i, j, k) = u1[v];
          }
        }
        if (mark) (*mark)[g.id(i, j, k)] = (f || fl) ? 1 : 0;
        if (count) {
          fails += f;
          hits += fl != 0;
          fluid += (fl & FL_FLUID_FRAME) != 0;
          if (flags && f) flags[g.id(i, j, k)] += 1 << stage;
        }
        for (int v = 0; v < NV; v++) V(Pout, g, v, i, j, k) = pn[v];
      }
  if (count) {
    g_stats.fails += fails;
    g_stats.floor_hits += hits;
    g_stats.fluid_frame += fluid;
  }
}

// Mark of the zone at padded index (i, j, k) for the flux correction:
// interior zones their own; on a periodic axis a ghost index wraps to the
// interior zone it copies; other ghosts are never marked.
bool marked(const Grid& g, const std::vector<char>& mark, int i, int j, int k) {
  int idx[3] = {i, j, k};
  for (int a = 0; a < 3; a++) {
    if (idx[a] >= 0 && idx[a] < g.n[a]) continue;
    if (g.c.bc[2 * a] != BC_PERIODIC) return false;
    idx[a] = ((idx[a] % g.n[a]) + g.n[a]) % g.n[a];
  }
  return mark[g.id(idx[0], idx[1], idx[2])] != 0;
}

// One SSPRK2 (Heun) step:
//   U1 = Un + dt L(Pn);                  P1   = U_to_P(U1; guess Pn)
//   Un+1 = (Un + U1)/2 + (dt L(P1))/2;   Pn+1 = U_to_P(Un+1; guess P1)
// Ghosts are refilled from each stage's prims before it runs.  The other
// integrators the Solvers section lists change only the combination of the
// stages: predictor-corrector (a half step gives P*, then the full step from
// U^n with the rates of P*) and RK1 (one forward-Euler stage).
//
// First-order flux correction (Algorithm section, after Beckwith & Stone
// 2011): each stage is first taken with the high-order fluxes; the zones
// where it would fail the inversion or call on the floors are marked, every
// face of a marked zone gets the local Lax-Friedrichs flux of donor-cell
// states instead, Flux-CT is redone on the corrected fluxes and the stage is
// taken again.  (Stages that mark nothing keep their first result.)
//
// With face-centred CT (phi not null: the face fields, advanced alongside)
// each stage takes the edge EMFs from the fluxes, advances the faces
// (phi1 = phin + dt R(Pn); phin+1 = (phin + phi1)/2 + dt R(P1)/2) and sets
// every zone's conserved field to the mean of its new faces before U_to_P.
long step_ssprk54(const Grid& g, std::vector<real>& P, real dt, int* flags);

long step(const Grid& g, std::vector<real>& P, real dt, int* flags, std::vector<real>* phi = nullptr) {
  if (g.c.integrator == 3) {  // the plain Flux-CT path only
    if (phi || g.c.floors || g.c.fofc) {
      fprintf(stderr, "oracle: SSPRK(5,4) takes the plain Flux-CT step only\n");
      abort();
    }
    return step_ssprk54(g, P, dt, flags);
  }
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  std::vector<real> F[3], Fct[3];
  for (int d = 0; d < 3; d++) F[d].assign(NV * g.nz, 0.0);
  std::vector<real> Un(NV * g.nz, 0.0), U1v(NV * g.nz, 0.0);
  std::vector<real> P1 = P;
  std::vector<char> mark;
  long fails0 = g_stats.fails;
  std::vector<real> phi1[3], phiV[3], phiOut[3], E[3];

  const int nstages = g.c.integrator == 2 ? 1 : 2;
  for (int stage = 0; stage < nstages; stage++) {
    std::vector<real>& Pin = stage == 0 ? P : P1;
    std::vector<real>* phiIn = stage == 0 ? phi : phi1;
    fill_ghosts(g, Pin);
    if (phi) fill_face_ghosts(g, phiIn);
    compute_fluxes(g, Pin, F, phi ? phiIn : nullptr);
    std::vector<real> Pout = Pin;
    // the magnetic part of a stage from fluxes Fx: Flux-CT fluxes (in Fc), or
    // new face fields (in phiOut) from the edge EMFs
    auto magnetic = [&](std::vector<real> Fx[3], std::vector<real> Fc[3]) {
      if (!phi) {
        for (int d = 0; d < 3; d++) Fc[d] = Fx[d];
        flux_ct(g, Fc);
        return;
      }
      for (int d = 0; d < 3; d++) Fc[d] = Fx[d];
      edge_emfs(g, Pin, Fx, g.c.ct, E);
      if (stage == 0) {
        face_update(g, E, phi, dt, phiOut);
        for (int d = 0; d < 3; d++) {
          phiV[d].resize(g.nz);
          for (long q = 0; q < g.nz; q++) phiV[d][q] = 0.5 * (phi[d][q] + phiOut[d][q]);
        }
      } else {
        face_update(g, E, phiV, 0.5 * dt, phiOut);
      }
    };
    const std::vector<real>* pnew = phi ? phiOut : nullptr;
    if (!g.c.fofc) {
      magnetic(F, Fct);
      update_pass(g, Pin, Fct, stage, dt, Un, U1v, Pout, flags, nullptr, true, pnew);
    } else {
      magnetic(F, Fct);
      mark.assign(g.nz, 0);
      update_pass(g, Pin, Fct, stage, dt, Un, U1v, Pout, flags, &mark, false, pnew);
      long nmark = 0;
      for (long z = 0; z < g.nz; z++) nmark += mark[z];
      if (nmark > 0) {
        g_stats.fofc_zones += nmark;
        // every face the flux pass computed whose either zone is marked
        for (int d = 1; d <= 3; d++) {
          int lo[3] = {-1, -1, -1}, hi[3] = {n1, n2, n3};
          lo[d - 1] = 0;
          int di = d == 1, dj = d == 2, dk = d == 3;
          for (int k = lo[2]; k <= hi[2]; k++)
            for (int j = lo[1]; j <= hi[1]; j++)
              for (int i = lo[0]; i <= hi[0]; i++) {
                if (!marked(g, mark, i, j, k) && !marked(g, mark, i - di, j - dj, k - dk)) continue;
                real f[NV];
                face_flux(g, Pin, RECON_DONOR, d, i, j, k, f, phi ? phiIn : nullptr);
                for (int v = 0; v < NV; v++) V(F[d - 1], g, v, i, j, k) = f[v];
              }
        }
        magnetic(F, Fct);
        Pout = Pin;
        update_pass(g, Pin, Fct, stage, dt, Un, U1v, Pout, flags, nullptr, true, pnew);
      }
    }
    if (nstages == 1) {  // RK1: the one stage is the step
      P = Pout;
    } else if (stage == 0) {
      P1 = Pout;
      if (phi)
        for (int d = 0; d < 3; d++) phi1[d] = phiOut[d];
    } else {
      P = Pout;
      if (phi)
        for (int d = 0; d < 3; d++) phi[d] = phiOut[d];
    }
  }
  return g_stats.fails - fails0;
}

// SSPRK(5,4), the five-stage fourth-order strong-stability-preserving
// Runge-Kutta method of Spiteri & Ruuth (2002) that the Solvers section lists,
// in its Shu-Osher form (coefficients as published, 15 digits):
//   U(1)    = U^n + c1 dt L(P^n)
//   U(k)    = a_k U^n + b_k U(k-1) + c_k dt L(P(k-1)),   k = 2, 3, 4
//   U^{n+1} = d2 U(2) + d3 U(3) + e3 dt L(P(3)) + d4 U(4) + e4 dt L(P(4))
// where every U(k) is followed by U_to_P with the previous stage's prims as
// the guess (P(k) = U_to_P(U(k))), and a zone whose inversion fails keeps its
// stage-input prims, as in the other integrators.  The stages take the plain
// Flux-CT path (no floors, correction or face-centred CT).
const real SSP54_C1 = 0.391752226571890;
const real SSP54_A[5] = {0.0, 0.0, 0.444370493651235, 0.620101851488403, 0.178079954393132};
const real SSP54_B[5] = {0.0, 0.0, 0.555629506348765, 0.379898148511597, 0.821920045606868};
const real SSP54_C[5] = {0.0, 0.0, 0.368410593050371, 0.251891774271694, 0.544974750228521};
const real SSP54_D2 = 0.517231671970585, SSP54_D3 = 0.096059710526147, SSP54_E3 = 0.063692468666290,
           SSP54_D4 = 0.386708617503269, SSP54_E4 = 0.226007483236906;

long step_ssprk54(const Grid& g, std::vector<real>& P, real dt, int* flags) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  std::vector<real> F[3];
  for (int d = 0; d < 3; d++) F[d].assign(NV * g.nz, 0.0);
  std::vector<real> Us[5];  // U^n, U(1) .. U(4)
  for (int s = 0; s < 5; s++) Us[s].assign(NV * g.nz, 0.0);
  std::vector<real> dtL3(NV * g.nz, 0.0);  // dt L(P(3)), for the last stage
  std::vector<real> Pin = P;
  long fails = 0;
  for (int stage = 0; stage < 5; stage++) {
    fill_ghosts(g, Pin);
    compute_fluxes(g, Pin, F);
    flux_ct(g, F);
    std::vector<real> Pout = Pin;
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads) reduction(+ : fails)
    for (int k = 0; k < n3; k++)
      for (int j = 0; j < n2; j++)
        for (int i = 0; i < n1; i++) {
          real p[NV], L[NV], Unew[NV], pn[NV];
          for (int v = 0; v < NV; v++) p[v] = Vc(Pin, g, v, i, j, k);
          rhs(g, F, p, i, j, k, L);
          if (stage == 0) {
            real u0[NV];
            cons_at(g, p, i, j, u0);
            for (int v = 0; v < NV; v++) V(Us[0], g, v, i, j, k) = u0[v];
          }
          for (int v = 0; v < NV; v++) {
            const real dtl = dt * L[v];
            const real un = Vc(Us[0], g, v, i, j, k);
            if (stage == 0) {
              Unew[v] = un + SSP54_C1 * dtl;
            } else if (stage < 4) {
              const int s = stage + 1;
              Unew[v] = SSP54_A[s] * un + SSP54_B[s] * Vc(Us[stage], g, v, i, j, k) + SSP54_C[s] * dtl;
              if (stage == 3) V(dtL3, g, v, i, j, k) = dtl;
            } else {
              Unew[v] = SSP54_D2 * Vc(Us[2], g, v, i, j, k) + SSP54_D3 * Vc(Us[3], g, v, i, j, k) +
                        SSP54_E3 * Vc(dtL3, g, v, i, j, k) + SSP54_D4 * Vc(Us[4], g, v, i, j, k) +
                        SSP54_E4 * dtl;
            }
            if (stage < 4) V(Us[stage + 1], g, v, i, j, k) = Unew[v];
          }
          int f = invert(g.c, g.gC[g.id2(i, j)], Unew, p, pn);
          fails += f;
          if (flags && f) flags[g.id(i, j, k)] += 1 << stage;
          for (int v = 0; v < NV; v++) V(Pout, g, v, i, j, k) = pn[v];
        }
    Pin.swap(Pout);
  }
  P.swap(Pin);
  g_stats.fails += fails;
  return fails;
}

// CFL time step: cfl / max over interior zones of sum_d max(|c+|, |c-|)/dx_d,
// over the directions that have more than one zone.  A zone whose rate is
// not finite leaves the minimum over zones undefined: the result is NaN.
real estimate_dt(const Grid& g, std::vector<real>& P) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  real smax = 0.0;
  bool bad = false;
  for (int k = 0; k < n3; k++)
    for (int j = 0; j < n2; j++)
      for (int i = 0; i < n1; i++) {
        real p[NV];
        for (int v = 0; v < NV; v++) p[v] = Vc(P, g, v, i, j, k);
        const Geom& G = g.gC[g.id2(i, j)];
        FluidState S;
        fluid_state(p, G, S);
        real s = 0.0;
        for (int d = 1; d <= 3; d++) {
          if (g.n[d - 1] == 1) continue;
          real cp, cm;
          vchar(p, S, G, g.c.gam, d, cp, cm);
          real cmx = fabs(cp) > fabs(cm) ? fabs(cp) : fabs(cm);
          s += cmx / g.dx[d - 1];
        }
        if (!isfinite(s)) bad = true;
        if (s > smax) smax = s;
      }
  if (bad) return real(NAN);
  return g.c.cfl / smax;
}

// Corner-centred divergence of B from the conserved field sqrt(-g) B^d:
// sum_d [sum of the four zones on the + side - the four on the - side]/(4 dx_d),
// divided by sqrt(-g) at the corner.  Corners on non-periodic boundaries
// (and so on the poles) are excluded.
void divb(const Grid& g, std::vector<real>& P, real* out_max, real* out_mean, real* field) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  fill_ghosts(g, P);
  int ilo = g.c.bc[0] == BC_PERIODIC ? 0 : 1, ihi = g.c.bc[1] == BC_PERIODIC ? n1 - 1 : n1 - 1;
  int jlo = g.c.bc[2] == BC_PERIODIC ? 0 : 1, jhi = n2 - 1;
  int klo = g.c.bc[4] == BC_PERIODIC ? 0 : 1, khi = n3 - 1;
  (void)ihi;
  real mx = 0.0, sum = 0.0;
  long cnt = 0;
  auto UB = [&](int d, int i, int j, int k) -> real {
    return g.gC[g.id2(i, j)].gdet * Vc(P, g, B1 + d, i, j, k);
  };
  for (int k = klo; k <= khi; k++)
    for (int j = jlo; j <= jhi; j++)
      for (int i = ilo; i <= n1 - 1; i++) {
        real dv = 0.0;
        dv += (UB(0, i, j, k) + UB(0, i, j - 1, k) + UB(0, i, j, k - 1) + UB(0, i, j - 1, k - 1) -
               UB(0, i - 1, j, k) - UB(0, i - 1, j - 1, k) - UB(0, i - 1, j, k - 1) - UB(0, i - 1, j - 1, k - 1)) /
              (4.0 * g.dx[0]);
        dv += (UB(1, i, j, k) + UB(1, i - 1, j, k) + UB(1, i, j, k - 1) + UB(1, i - 1, j, k - 1) -
               UB(1, i, j - 1, k) - UB(1, i - 1, j - 1, k) - UB(1, i, j - 1, k - 1) - UB(1, i - 1, j - 1, k - 1)) /
              (4.0 * g.dx[1]);
        dv += (UB(2, i, j, k) + UB(2, i - 1, j, k) + UB(2, i, j - 1, k) + UB(2, i - 1, j - 1, k) -
               UB(2, i, j, k - 1) - UB(2, i - 1, j, k - 1) - UB(2, i, j - 1, k - 1) - UB(2, i - 1, j - 1, k - 1)) /
              (4.0 * g.dx[2]);
        real val = fabs(dv) / g.gCorner[g.id2(i, j)].gdet;
        if (field) field[g.id(i, j, k)] = val;
        if (val > mx) mx = val;
        sum += val;
        cnt++;
      }
  *out_max = mx;
  *out_mean = cnt ? sum / (real)(double)cnt : 0.0;
}

void load(const Grid& g, const double* src, std::vector<real>& dst) {
  dst.resize(NV * g.nz);
  for (long q = 0; q < NV * g.nz; q++) dst[q] = src[q];
}
void store(const Grid& g, const std::vector<real>& src, double* dst) {
  for (long q = 0; q < NV * g.nz; q++) dst[q] = (double)src[q];
}

}  // namespace

// ------------------------------------------------------- Extended GRMHD --
//
// Extended GRMHD (Implicit Solver and Extended Theory section, EGRMHD
// subsection, after Chandra et al. 2015 in the variables of Foucart et al.
// 2016): two more zone-centred variables, the rescaled heat flux and
// pressure anisotropy
//   X0 = qt  = q  (tau_R / (chi rho Theta^2))^(1/2),
//   X1 = dPt = dP (tau_R / (nu rho Theta))^(1/2),     Theta = p / rho.
// The stress-energy tensor gains q^mu u_nu + q_nu u^mu + Pi^mu_nu with
// q^mu = q bh^mu, bh = b / |b|, Pi^mu_nu = -dP (bh^mu bh_nu - h^mu_nu / 3),
// h^mu_nu = delta^mu_nu + u^mu u_nu (both taken as zero where b^2 = 0), and
//   d_mu(sqrt(-g) X u^mu) = sqrt(-g) [-(X - Xtarget) / tau_R + (X / 2) div u].
// Readings where the paper defers to the cited papers:
//   * tau_R, chi, nu are constants;
//   * the targets are the Chandra et al. closure
//       q0  = -rho chi bh^mu (d_mu Theta + Theta a_mu),  a_mu = u^nu nabla_nu u_mu,
//       dP0 = 3 rho nu (bh^mu bh^nu nabla_mu u_nu - div u / 3),
//     rescaled like the variables, from the stage's explicit state with
//     centred spatial differences, the time derivatives in them left out;
//   * div u = d_t u^t + d_i(sqrt(-g) u^i) / sqrt(-g): the spatial part from
//     the explicit state, the time part (u^t(new) - u^t(step start)) / h in
//     the new state, like the relaxation -X / tau_R and the X multiplying
//     div u (the implicit terms);
//   * the LLF signal speeds are the ideal fast-magnetosonic ones.
// The step is the predictor-corrector, the integrator the paper allows for
// a semi-implicit theory: h = dt/2 from the step's state, then h = dt from
// it again with the explicit rates of the predicted state.  Per zone each
// stage solves U(P, X) = U^n + h (explicit rate) + h (implicit sources) with
// the implicit solver's Newton on the five hydro prims: given the hydro
// state the two X equations are linear in X and are solved for X within
// every residual evaluation (the root of the joint seven-variable system).
const int NX = 2;

struct EmhdPar {
  real tau, chi, nu;
};

// Physical q and dP of the rescaled variables X.
void emhd_unscale(const real P[NV], real gam, const EmhdPar& e, const real X[NX], real& q, real& dP) {
  const real theta = (gam - 1.0) * P[UU] / P[RHO];
  q = X[0] * theta * sqrt(e.chi * P[RHO] / e.tau);
  dP = X[1] * sqrt(e.nu * P[RHO] * theta / e.tau);
}

// Mixed T^mu_nu of Extended GRMHD.
real tmunu_emhd(const real P[NV], const FluidState& S, real gam, real q, real dP, int mu, int nu) {
  const real t = tmunu(P, S, gam, mu, nu);
  if (!(S.bsq > 0.0) || (q == 0.0 && dP == 0.0)) return t;
  const real bm = S.bcon[mu] / sqrt(S.bsq), bn = S.bcov[nu] / sqrt(S.bsq);
  const real h = (mu == nu ? 1.0 : 0.0) + S.ucon[mu] * S.ucov[nu];
  return t + q * bm * S.ucov[nu] + q * bn * S.ucon[mu] - dP * (bm * bn - h / 3.0);
}

// Conserved variables (d = 0) or fluxes along x^d of the ten variables:
// sqrt(-g) (rho u^d, T^d_t + rho u^d, T^d_i, b^k u^d - b^d u^k, X u^d).
void prim_to_flux_emhd(const real P[NV], const real X[NX], const FluidState& S, const Geom& G, real gam,
                       const EmhdPar& e, int d, real F[NV + NX]) {
  real q, dP;
  emhd_unscale(P, gam, e, X, q, dP);
  F[RHO] = G.gdet * P[RHO] * S.ucon[d];
  F[UU] = G.gdet * (tmunu_emhd(P, S, gam, q, dP, d, 0) + P[RHO] * S.ucon[d]);
  for (int i = 1; i < 4; i++) F[U1 + i - 1] = G.gdet * tmunu_emhd(P, S, gam, q, dP, d, i);
  for (int k = 1; k < 4; k++) {
    if (d == 0)
      F[B1 + k - 1] = G.gdet * P[B1 + k - 1];
    else
      F[B1 + k - 1] = G.gdet * (S.bcon[k] * S.ucon[d] - S.bcon[d] * S.ucon[k]);
  }
  for (int n = 0; n < NX; n++) F[NV + n] = G.gdet * X[n] * S.ucon[d];
}

// Geometric source sqrt(-g) T^k_l Gamma^l_{nu k} with the extended T.
void source_point_emhd(const Geom& G, const real* cn, real gam, const EmhdPar& e, const real P[NV],
                       const real X[NX], real S[NV]) {
  FluidState st;
  fluid_state(P, G, st);
  real q, dP;
  emhd_unscale(P, gam, e, X, q, dP);
  real T[4][4];
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) T[m][n] = tmunu_emhd(P, st, gam, q, dP, m, n);
  for (int v = 0; v < NV; v++) S[v] = 0.0;
  for (int nu = 0; nu < 4; nu++) {
    real s = 0.0;
    for (int k = 0; k < 4; k++)
      for (int l = 0; l < 4; l++) s += T[k][l] * cn[l * 16 + nu * 4 + k];
    S[UU + nu] = G.gdet * s;
  }
}

// LLF flux of the ten variables at the lower d-face of zone (i, j, k).
void face_flux_emhd(const Grid& g, const std::vector<real>& P, const std::vector<real>& X, const EmhdPar& e,
                    int d, int i, int j, int k, real F[NV + NX]) {
  if (g.pole_face(d, j)) {
    for (int v = 0; v < NV + NX; v++) F[v] = 0.0;
    return;
  }
  real qL[NV], qR[NV], xL[NX], xR[NX];
  reconstruct(g, P, g.c.recon, d, i, j, k, qL, qR);
  reconstruct_vars(g, X, NX, g.c.recon, d, i, j, k, xL, xR);
  const Geom& G = g.face_geom(d, i, j);
  FluidState SL, SR;
  fluid_state(qL, G, SL);
  fluid_state(qR, G, SR);
  real FL[NV + NX], FR[NV + NX], UL[NV + NX], UR[NV + NX];
  prim_to_flux_emhd(qL, xL, SL, G, g.c.gam, e, d, FL);
  prim_to_flux_emhd(qR, xR, SR, G, g.c.gam, e, d, FR);
  prim_to_flux_emhd(qL, xL, SL, G, g.c.gam, e, 0, UL);
  prim_to_flux_emhd(qR, xR, SR, G, g.c.gam, e, 0, UR);
  real cpl, cml, cpr, cmr;
  vchar(qL, SL, G, g.c.gam, d, cpl, cml);
  vchar(qR, SR, G, g.c.gam, d, cpr, cmr);
  real cmax = 0.0;
  if (cpl > cmax) cmax = cpl;
  if (cpr > cmax) cmax = cpr;
  if (-cml > cmax) cmax = -cml;
  if (-cmr > cmax) cmax = -cmr;
  for (int v = 0; v < NV + NX; v++) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * cmax * (UR[v] - UL[v]);
}

// Fluxes on the faces of compute_fluxes: the eight ideal slots to F, the
// two X slots to FX.
void compute_fluxes_emhd(const Grid& g, const std::vector<real>& P, const std::vector<real>& X,
                         const EmhdPar& e, std::vector<real> F[3], std::vector<real> FX[3]) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  for (int d = 1; d <= 3; d++) {
    int lo[3] = {-1, -1, -1}, hi[3] = {n1, n2, n3};  // inclusive
    lo[d - 1] = 0;
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads)
    for (int k = lo[2]; k <= hi[2]; k++)
      for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
          real f[NV + NX];
          face_flux_emhd(g, P, X, e, d, i, j, k, f);
          for (int v = 0; v < NV; v++) V(F[d - 1], g, v, i, j, k) = f[v];
          for (int n = 0; n < NX; n++) V(FX[d - 1], g, n, i, j, k) = f[NV + n];
        }
  }
}

// Targets Xtarget and the spatial part of div u at zone (i, j, k) from the
// explicit state P (ghosts filled).
void emhd_targets(const Grid& g, const std::vector<real>& P, const EmhdPar& e, int i, int j, int k,
                  real Xt[NX], real& divu_sp) {
  const real gam = g.c.gam;
  auto state = [&](int ii, int jj, int kk, FluidState& S, real& theta) {
    real p[NV];
    for (int v = 0; v < NV; v++) p[v] = Vc(P, g, v, ii, jj, kk);
    fluid_state(p, g.gC[g.id2(ii, jj)], S);
    theta = (gam - 1.0) * p[UU] / p[RHO];
  };
  FluidState S0;
  real th0;
  state(i, j, k, S0, th0);
  const Geom& G = g.gC[g.id2(i, j)];
  const real* cn = &g.conn[g.id2(i, j) * 64];
  real dth[3], du[3][4], dgu[3];  // d_a Theta, d_a u_nu, d_a (sqrt(-g) u^a)
  for (int a = 0; a < 3; a++) {
    dth[a] = dgu[a] = 0.0;
    for (int nu = 0; nu < 4; nu++) du[a][nu] = 0.0;
    if (g.n[a] == 1) continue;
    const int di = a == 0, dj = a == 1, dk = a == 2;
    FluidState Sp, Sm;
    real thp, thm;
    state(i + di, j + dj, k + dk, Sp, thp);
    state(i - di, j - dj, k - dk, Sm, thm);
    const real h2 = 2.0 * g.dx[a];
    dth[a] = (thp - thm) / h2;
    for (int nu = 0; nu < 4; nu++) du[a][nu] = (Sp.ucov[nu] - Sm.ucov[nu]) / h2;
    dgu[a] = (g.gC[g.id2(i + di, j + dj)].gdet * Sp.ucon[a + 1] -
              g.gC[g.id2(i - di, j - dj)].gdet * Sm.ucon[a + 1]) / h2;
  }
  divu_sp = ((dgu[0] + dgu[1]) + dgu[2]) / G.gdet;
  Xt[0] = Xt[1] = 0.0;
  if (!(S0.bsq > 0.0)) return;
  real bh[4];
  for (int m = 0; m < 4; m++) bh[m] = S0.bcon[m] / sqrt(S0.bsq);
  // a_nu = u^i d_i u_nu - Gamma^l_{m nu} u^m u_l
  real acc[4];
  for (int nu = 0; nu < 4; nu++) {
    real s = 0.0;
    for (int a = 0; a < 3; a++) s += S0.ucon[a + 1] * du[a][nu];
    for (int l = 0; l < 4; l++)
      for (int m = 0; m < 4; m++) s -= cn[l * 16 + m * 4 + nu] * S0.ucon[m] * S0.ucov[l];
    acc[nu] = s;
  }
  real gq = 0.0;  // bh^mu (d_mu Theta + Theta a_mu)
  for (int a = 0; a < 3; a++) gq += bh[a + 1] * dth[a];
  for (int nu = 0; nu < 4; nu++) gq += th0 * bh[nu] * acc[nu];
  real bbu = 0.0;  // bh^mu bh^nu nabla_mu u_nu
  for (int a = 0; a < 3; a++)
    for (int nu = 0; nu < 4; nu++) bbu += bh[a + 1] * bh[nu] * du[a][nu];
  for (int m = 0; m < 4; m++)
    for (int nu = 0; nu < 4; nu++)
      for (int l = 0; l < 4; l++) bbu -= bh[m] * bh[nu] * cn[l * 16 + m * 4 + nu] * S0.ucov[l];
  const real rho = Vc(P, g, RHO, i, j, k);
  if (e.chi > 0.0) Xt[0] = -gq * sqrt(e.chi * rho * e.tau) / th0;
  if (e.nu > 0.0) Xt[1] = 3.0 * (bbu - divu_sp / 3.0) * sqrt(e.nu * rho * e.tau / th0);
}

// One zone's implicit stage solve.  Urhs: U^n + h (explicit rate) for the
// eight ideal slots; UrhsX: U^n_X + h (-flux divergence + sqrt(-g) Xtarget
// / tau_R); ut_n: u^t of the step's starting state.  P, X: the stage input
// in (the guess), the new state out; returns 1 (and keeps the guess's hydro
// prims and X) on failure.  B^i = Urhs_B / sqrt(-g) in every case.
int emhd_solve(const orc_cfg& c, const EmhdPar& e, const Geom& G, const real Urhs[NV], const real UrhsX[NX],
               real divu_sp, real ut_n, real h, real P[NV], real X[NX]) {
  for (int k = 0; k < 3; k++) P[B1 + k] = Urhs[B1 + k] / G.gdet;
  const real B[3] = {P[B1], P[B2], P[B3]};
  real scale = 0.0;
  for (int k = 0; k < 5; k++)
    if (fabs(Urhs[k]) > scale) scale = fabs(Urhs[k]);
  if (!(scale > 0.0) || !isfinite((real)scale)) return 1;
  // the X of hydro state x: gdet X (u^t + h/tau - (h/2) div u) = UrhsX
  auto xsolve = [&](const real Pz[NV], const FluidState& S, real Xz[NX]) {
    const real ut = S.ucon[0];
    const real divu = divu_sp + (ut - ut_n) / h;
    const real coef = G.gdet * ut + h * G.gdet / e.tau - 0.5 * h * G.gdet * divu;
    for (int n = 0; n < NX; n++) Xz[n] = UrhsX[n] / coef;
    (void)Pz;
  };
  auto res = [&](const real x[5], real R[5]) {
    const real Pz[NV] = {x[0], x[1], x[2], x[3], x[4], B[0], B[1], B[2]};
    FluidState S;
    fluid_state(Pz, G, S);
    real Xz[NX], U[NV + NX];
    xsolve(Pz, S, Xz);
    prim_to_flux_emhd(Pz, Xz, S, G, c.gam, e, 0, U);
    for (int k = 0; k < 5; k++) R[k] = (U[k] - Urhs[k]) / scale;
  };
  real x[5];
  if (newton_hydro(c, P, res, x)) return 1;
  real Pn[NV] = {x[0], x[1], x[2], x[3], x[4], B[0], B[1], B[2]};
  FluidState S;
  fluid_state(Pn, G, S);
  real Xn[NX];
  xsolve(Pn, S, Xn);
  for (int n = 0; n < NX; n++)
    if (!isfinite((real)Xn[n])) return 1;
  for (int k = 0; k < 5; k++) P[k] = x[k];
  for (int n = 0; n < NX; n++) X[n] = Xn[n];
  return 0;
}

// One predictor-corrector step of Extended GRMHD (Flux-CT for the field).
long step_emhd(const Grid& g, const EmhdPar& e, std::vector<real>& P, std::vector<real>& X, real dt) {
  const int n1 = g.c.n1, n2 = g.c.n2, n3 = g.c.n3;
  std::vector<real> F[3], FX[3];
  for (int d = 0; d < 3; d++) {
    F[d].assign(NV * g.nz, 0.0);
    FX[d].assign(NX * g.nz, 0.0);
  }
  std::vector<real> Un(NV * g.nz, 0.0), UnX(NX * g.nz, 0.0), utn(g.nz, 0.0);
  std::vector<real> P1 = P, X1 = X;
  long fails = 0;
  for (int stage = 0; stage < 2; stage++) {
    std::vector<real>& Pin = stage == 0 ? P : P1;
    std::vector<real>& Xin = stage == 0 ? X : X1;
    fill_ghosts(g, Pin);
    fill_ghosts_vars(g, Xin, NX, 0u);
    compute_fluxes_emhd(g, Pin, Xin, e, F, FX);
    flux_ct(g, F);
    const real h = stage == 0 ? 0.5 * dt : dt;
    std::vector<real> Pout = Pin, Xout = Xin;
#pragma omp parallel for collapse(2) schedule(static) num_threads(g.c.nthreads) reduction(+ : fails)
    for (int k = 0; k < n3; k++)
      for (int j = 0; j < n2; j++)
        for (int i = 0; i < n1; i++) {
          const Geom& G = g.gC[g.id2(i, j)];
          real p[NV], x[NX];
          for (int v = 0; v < NV; v++) p[v] = Vc(Pin, g, v, i, j, k);
          for (int n = 0; n < NX; n++) x[n] = Vc(Xin, g, n, i, j, k);
          if (stage == 0) {  // U^n and u^t of the step's state
            FluidState S;
            fluid_state(p, G, S);
            real u0[NV + NX];
            prim_to_flux_emhd(p, x, S, G, g.c.gam, e, 0, u0);
            for (int v = 0; v < NV; v++) V(Un, g, v, i, j, k) = u0[v];
            for (int n = 0; n < NX; n++) V(UnX, g, n, i, j, k) = u0[NV + n];
            utn[g.id(i, j, k)] = S.ucon[0];
          }
          real Sg[NV];
          source_point_emhd(G, &g.conn[g.id2(i, j) * 64], g.c.gam, e, p, x, Sg);
          real Xt[NX], divu_sp;
          emhd_targets(g, Pin, e, i, j, k, Xt, divu_sp);
          real Urhs[NV], UrhsX[NX];
          for (int v = 0; v < NV; v++) {
            real d1 = (Vc(F[0], g, v, i + 1, j, k) - Vc(F[0], g, v, i, j, k)) / g.dx[0];
            real d2 = (Vc(F[1], g, v, i, j + 1, k) - Vc(F[1], g, v, i, j, k)) / g.dx[1];
            real d3 = (Vc(F[2], g, v, i, j, k + 1) - Vc(F[2], g, v, i, j, k)) / g.dx[2];
            const real L = -((d1 + d2) + d3) + Sg[v];
            Urhs[v] = Vc(Un, g, v, i, j, k) + h * L;
          }
          for (int n = 0; n < NX; n++) {
            real d1 = (Vc(FX[0], g, n, i + 1, j, k) - Vc(FX[0], g, n, i, j, k)) / g.dx[0];
            real d2 = (Vc(FX[1], g, n, i, j + 1, k) - Vc(FX[1], g, n, i, j, k)) / g.dx[1];
            real d3 = (Vc(FX[2], g, n, i, j, k + 1) - Vc(FX[2], g, n, i, j, k)) / g.dx[2];
            UrhsX[n] = Vc(UnX, g, n, i, j, k) + h * (-((d1 + d2) + d3) + G.gdet * Xt[n] / e.tau);
          }
          const int f = emhd_solve(g.c, e, G, Urhs, UrhsX, divu_sp, utn[g.id(i, j, k)], h, p, x);
          fails += f;
          for (int v = 0; v < NV; v++) V(Pout, g, v, i, j, k) = p[v];
          for (int n = 0; n < NX; n++) V(Xout, g, n, i, j, k) = x[n];
        }
    if (stage == 0) {
      P1 = Pout;
      X1 = Xout;
    } else {
      P = Pout;
      X = Xout;
    }
  }
  return fails;
}

// ---------------------------------------------------------------- C ABI ----

extern "C" {

// Advance the padded prims in place by `nsteps` steps of size dt of the
// configured integrator (dt <= 0: recompute the CFL dt before each step).
// Returns the number of zone inversions that failed; the dt actually used per
// step go to dts and, when flags is not null, failures are added per padded
// zone (1 << s for a failure in stage s, s counted from 0).
long orc_run(const orc_cfg* c, double* prims, double dt, int nsteps, double* dts, int* flags) {
  Grid g(*c);
  g_stats = RunStats{0, 0, 0, 0};
  std::vector<real> P;
  load(g, prims, P);
  long fails = 0;
  for (int s = 0; s < nsteps; s++) {
    real h = dt;
    if (dt <= 0.0) {
      fill_ghosts(g, P);
      h = estimate_dt(g, P);
    }
    if (dts) dts[s] = (double)h;
    fails += step(g, P, h, flags);
  }
  fill_ghosts(g, P);
  store(g, P, prims);
  return fails;
}

// Extended GRMHD (predictor-corrector, Flux-CT): advance the padded prims
// and the padded extra variables x = double[2][padded] (qt, dPt) in place by
// nsteps steps of size dt (dt <= 0: the ideal CFL dt before each step).
// Returns the number of zone solves that failed.
long orc_run_emhd(const orc_cfg* c, double* prims, double* extra, double dt, int nsteps, double* dts) {
  Grid g(*c);
  const EmhdPar e{c->tau_r, c->chi_emhd, c->nu_emhd};
  std::vector<real> P, X(NX * g.nz);
  load(g, prims, P);
  for (long q = 0; q < NX * g.nz; q++) X[q] = extra[q];
  long fails = 0;
  for (int s = 0; s < nsteps; s++) {
    real h = dt;
    if (dt <= 0.0) {
      fill_ghosts(g, P);
      h = estimate_dt(g, P);
    }
    if (dts) dts[s] = (double)h;
    fails += step_emhd(g, e, P, X, h);
  }
  fill_ghosts(g, P);
  fill_ghosts_vars(g, X, NX, 0u);
  store(g, P, prims);
  for (long q = 0; q < NX * g.nz; q++) extra[q] = (double)X[q];
  return fails;
}

// Conserved variables of Extended GRMHD (ten slots: the ideal eight, then
// sqrt(-g) X u^t) at interior zone centres of prims and extra.
void orc_cons_emhd(const orc_cfg* c, const double* prims, const double* extra, double* cons) {
  Grid g(*c);
  const EmhdPar e{c->tau_r, c->chi_emhd, c->nu_emhd};
  for (int k = 0; k < c->n3; k++)
    for (int j = 0; j < c->n2; j++)
      for (int i = 0; i < c->n1; i++) {
        const long q = g.id(i, j, k);
        real p[NV], x[NX], u[NV + NX];
        for (int v = 0; v < NV; v++) p[v] = prims[v * g.nz + q];
        for (int n = 0; n < NX; n++) x[n] = extra[n * g.nz + q];
        const Geom& G = g.gC[g.id2(i, j)];
        FluidState S;
        fluid_state(p, G, S);
        prim_to_flux_emhd(p, x, S, G, g.c.gam, e, 0, u);
        for (int v = 0; v < NV + NX; v++) cons[v * g.nz + q] = (double)u[v];
      }
}

// Extended GRMHD targets at interior zone (i, j, k) of padded prims (ghosts
// filled here on a copy): out[0], out[1] the rescaled heat-flux and
// anisotropy targets, out[2] the spatial part of div u.
void orc_emhd_targets(const orc_cfg* c, const double* prims, int i, int j, int k, double* out) {
  Grid g(*c);
  const EmhdPar e{c->tau_r, c->chi_emhd, c->nu_emhd};
  std::vector<real> P;
  load(g, prims, P);
  fill_ghosts(g, P);
  real Xt[NX], divu_sp;
  emhd_targets(g, P, e, i, j, k, Xt, divu_sp);
  out[0] = (double)Xt[0];
  out[1] = (double)Xt[1];
  out[2] = (double)divu_sp;
}

// Face-centred CT (cfg ct = 1 or 2): as orc_run, with the face fields
// faces = double[3][padded] (sqrt(-g) B^d on the lower d-face of each zone)
// advanced alongside; the interior zones' B prims are set from the faces
// first.  On return the faces' ghosts are filled and the prims' B is the
// faces' mean.
long orc_run_face(const orc_cfg* c, double* prims, double* faces, double dt, int nsteps, double* dts,
                  int* flags) {
  Grid g(*c);
  g_stats = RunStats{0, 0, 0, 0};
  std::vector<real> P, phi[3];
  load(g, prims, P);
  for (int d = 0; d < 3; d++) {
    phi[d].resize(g.nz);
    for (long q = 0; q < g.nz; q++) phi[d][q] = faces[d * g.nz + q];
  }
  for (int k = 0; k < c->n3; k++)
    for (int j = 0; j < c->n2; j++)
      for (int i = 0; i < c->n1; i++) {
        real UB[3];
        cell_field(g, phi, i, j, k, UB);
        for (int d = 0; d < 3; d++) V(P, g, B1 + d, i, j, k) = UB[d] / g.gC[g.id2(i, j)].gdet;
      }
  long fails = 0;
  for (int s = 0; s < nsteps; s++) {
    real h = dt;
    if (dt <= 0.0) {
      fill_ghosts(g, P);
      h = estimate_dt(g, P);
    }
    if (dts) dts[s] = (double)h;
    fails += step(g, P, h, flags, phi);
  }
  fill_ghosts(g, P);
  fill_face_ghosts(g, phi);
  store(g, P, prims);
  for (int d = 0; d < 3; d++)
    for (long q = 0; q < g.nz; q++) faces[d * g.nz + q] = (double)phi[d][q];
  return fails;
}

// Edge EMFs (E1, E2, E3 at the lower corners of every zone, edges 0..n) of
// the face-centred scheme cfg ct from the prims and faces of one state
// (ghosts filled here); out = double[3][padded], other entries zero.
void orc_edge_emfs(const orc_cfg* c, const double* prims, const double* faces, double* out) {
  Grid g(*c);
  std::vector<real> P, phi[3], F[3], E[3];
  load(g, prims, P);
  for (int d = 0; d < 3; d++) {
    phi[d].resize(g.nz);
    for (long q = 0; q < g.nz; q++) phi[d][q] = faces[d * g.nz + q];
    F[d].assign(NV * g.nz, 0.0);
  }
  fill_ghosts(g, P);
  fill_face_ghosts(g, phi);
  compute_fluxes(g, P, F, phi);
  edge_emfs(g, P, F, c->ct, E);
  for (int d = 0; d < 3; d++)
    for (long q = 0; q < g.nz; q++) out[d * g.nz + q] = (double)E[d][q];
}

// Face divergence sum_d (phi_d(+) - phi_d(-))/dx_d over interior zones:
// maximum and mean of its magnitude.
void orc_face_divb(const orc_cfg* c, const double* faces, double* out_max, double* out_mean) {
  Grid g(*c);
  double mx = 0.0, sm = 0.0;
  auto f = [&](int d, int i, int j, int k) { return faces[d * g.nz + g.id(i, j, k)]; };
  for (int k = 0; k < c->n3; k++)
    for (int j = 0; j < c->n2; j++)
      for (int i = 0; i < c->n1; i++) {
        double dv = ((f(0, i + 1, j, k) - f(0, i, j, k)) / (double)g.dx[0] +
                     (f(1, i, j + 1, k) - f(1, i, j, k)) / (double)g.dx[1]) +
                    (f(2, i, j, k + 1) - f(2, i, j, k)) / (double)g.dx[2];
        mx = std::max(mx, std::fabs(dv));
        sm += std::fabs(dv);
      }
  *out_max = mx;
  *out_mean = sm / ((double)c->n1 * c->n2 * c->n3);
}

// Counters of the last orc_run: failed inversions, zones floors acted on,
// zones the flux correction marked, fluid-frame fallbacks of the floors.
void orc_last_stats(long long* out) {
  out[0] = g_stats.fails;
  out[1] = g_stats.floor_hits;
  out[2] = g_stats.fofc_zones;
  out[3] = g_stats.fluid_frame;
}

double orc_estimate_dt(const orc_cfg* c, double* prims) {
  Grid g(*c);
  std::vector<real> P;
  load(g, prims, P);
  fill_ghosts(g, P);
  return (double)estimate_dt(g, P);
}

void orc_fill_ghosts(const orc_cfg* c, double* prims) {
  Grid g(*c);
  std::vector<real> P;
  load(g, prims, P);
  fill_ghosts(g, P);
  store(g, P, prims);
}

void orc_divb(const orc_cfg* c, const double* prims, double* out_max, double* out_mean, double* field) {
  Grid g(*c);
  std::vector<real> P;
  load(g, prims, P);
  real mx, mean;
  std::vector<real> fld;
  if (field) fld.assign(g.nz, 0.0);
  divb(g, P, &mx, &mean, field ? fld.data() : nullptr);
  *out_max = (double)mx;
  *out_mean = (double)mean;
  if (field)
    for (long q = 0; q < g.nz; q++) field[q] = (double)fld[q];
}

// Face fluxes of one stage from the given prims (ghosts filled here), after
// Flux-CT when ct != 0.  F is 3 x 8 x padded zones; entry (i, j, k) of
// direction d is the flux through the lower d-face of zone (i, j, k).
void orc_fluxes(const orc_cfg* c, const double* prims, double* F, int ct) {
  Grid g(*c);
  std::vector<real> P;
  load(g, prims, P);
  fill_ghosts(g, P);
  std::vector<real> Fv[3];
  for (int d = 0; d < 3; d++) Fv[d].assign(NV * g.nz, 0.0);
  compute_fluxes(g, P, Fv);
  if (ct) flux_ct(g, Fv);
  for (int d = 0; d < 3; d++)
    for (long q = 0; q < NV * g.nz; q++) F[d * NV * g.nz + q] = (double)Fv[d][q];
}

// Conserved variables at zone centres of the interior (padded layout).
void orc_prims_to_cons(const orc_cfg* c, const double* prims, double* cons) {
  Grid g(*c);
  for (int k = 0; k < c->n3; k++)
    for (int j = 0; j < c->n2; j++)
      for (int i = 0; i < c->n1; i++) {
        real p[NV], u[NV];
        for (int v = 0; v < NV; v++) p[v] = prims[v * g.nz + g.id(i, j, k)];
        cons_at(g, p, i, j, u);
        for (int v = 0; v < NV; v++) cons[v * g.nz + g.id(i, j, k)] = (double)u[v];
      }
}

// Inversion at zone centres of the interior; returns the failure count and
// writes a per-zone flag (0/1) when flags is not null.
long orc_cons_to_prims(const orc_cfg* c, const double* cons, const double* guess, double* prims,
                       int* flags) {
  Grid g(*c);
  long fails = 0;
  for (int k = 0; k < c->n3; k++)
    for (int j = 0; j < c->n2; j++)
      for (int i = 0; i < c->n1; i++) {
        real u[NV], gs[NV], p[NV];
        long q = g.id(i, j, k);
        for (int v = 0; v < NV; v++) { u[v] = cons[v * g.nz + q]; gs[v] = guess[v * g.nz + q]; }
        int f = invert(*c, g.gC[g.id2(i, j)], u, gs, p);
        fails += f;
        if (flags) flags[q] = f;
        for (int v = 0; v < NV; v++) prims[v * g.nz + q] = (double)p[v];
      }
  return fails;
}

// ---- point functions (pins) ----

void orc_geom(const orc_cfg* c, double x1, double x2, double* gcov, double* gcon, double* gdet,
              double* alpha) {
  Geom G;
  geom_point(*c, x1, x2, G);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) {
      gcov[m * 4 + n] = (double)G.gcov[m][n];
      gcon[m * 4 + n] = (double)G.gcon[m][n];
    }
  *gdet = (double)G.gdet;
  *alpha = (double)G.alpha;
}

void orc_conn(const orc_cfg* c, double x1, double x2, double* conn) {
  real cn[4][4][4];
  conn_point(*c, x1, x2, cn);
  for (int l = 0; l < 4; l++)
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) conn[l * 16 + m * 4 + n] = (double)cn[l][m][n];
}

// d = 0: conserved; d = 1..3: flux.  Also returns c+ and c- along d (d >= 1).
void orc_point_flux(const orc_cfg* c, const double* prims, double x1, double x2, int d, double* out,
                    double* cmax, double* cmin) {
  Geom G;
  geom_point(*c, x1, x2, G);
  real p[NV], f[NV];
  for (int v = 0; v < NV; v++) p[v] = prims[v];
  FluidState S;
  fluid_state(p, G, S);
  prim_to_flux(p, S, G, c->gam, d, f);
  for (int v = 0; v < NV; v++) out[v] = (double)f[v];
  if (d >= 1) {
    real cp, cm;
    vchar(p, S, G, c->gam, d, cp, cm);
    *cmax = (double)cp;
    *cmin = (double)cm;
  }
}

void orc_point_source(const orc_cfg* c, const double* prims, double x1, double x2, double* out) {
  Geom G;
  geom_point(*c, x1, x2, G);
  real cn[4][4][4];
  conn_point(*c, x1, x2, cn);
  real flat[64];
  for (int l = 0; l < 4; l++)
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) flat[l * 16 + m * 4 + n] = cn[l][m][n];
  real p[NV], s[NV];
  for (int v = 0; v < NV; v++) p[v] = prims[v];
  source_point(G, flat, c->gam, p, s);
  for (int v = 0; v < NV; v++) out[v] = (double)s[v];
}

int orc_point_u_to_p(const orc_cfg* c, const double* cons, const double* guess, double x1, double x2,
                     double* prims) {
  Geom G;
  geom_point(*c, x1, x2, G);
  real u[NV], gs[NV], p[NV];
  for (int v = 0; v < NV; v++) { u[v] = cons[v]; gs[v] = guess[v]; }
  int r = invert(*c, G, u, gs, p);
  for (int v = 0; v < NV; v++) prims[v] = (double)p[v];
  return r;
}

// Floors and ceilings of one zone's prims at (x1, x2); returns the mask of
// what acted (1 rho, 2 u, 4 fluid-frame fallback, 8 Lorentz factor, 16 u/rho).
int orc_point_floors(const orc_cfg* c, double* prims, double x1, double x2) {
  Geom G;
  geom_point(*c, x1, x2, G);
  real p[NV];
  for (int v = 0; v < NV; v++) p[v] = prims[v];
  int m = apply_floors(*c, G, x1, p);
  for (int v = 0; v < NV; v++) prims[v] = (double)p[v];
  return m;
}

// The implicit solver's 5 x 5 solve (QR with column pivoting): y = A^-1 b
// for A row-major; returns 0 if the matrix was found singular.
int orc_qr_solve(const double* A, const double* b, double* y) {
  real M[5][5], r[5], z[5];
  for (int i = 0; i < 5; i++) {
    r[i] = b[i];
    for (int j = 0; j < 5; j++) M[i][j] = A[5 * i + j];
  }
  bool ok = qr_pivot_solve(M, r, z);
  for (int i = 0; i < 5; i++) y[i] = (double)z[i];
  return ok ? 1 : 0;
}

double orc_weno5(double a, double b, double c, double d, double e, double eps) {
  return (double)weno5(a, b, c, d, e, eps);
}

double orc_mc_slope(double l, double c, double r) { return (double)mc_slope(l, c, r); }
// The SSPRK(5,4) step's Shu-Osher coefficients as the step uses them:
// c1, (a_k, b_k, c_k) for k = 2, 3, 4, then d2, d3, e3, d4, e4 (15 values).
void orc_ssprk54_coefficients(double* out) {
  int n = 0;
  out[n++] = (double)SSP54_C1;
  for (int k = 2; k <= 4; k++) {
    out[n++] = (double)SSP54_A[k];
    out[n++] = (double)SSP54_B[k];
    out[n++] = (double)SSP54_C[k];
  }
  for (real x : {SSP54_D2, SSP54_D3, SSP54_E3, SSP54_D4, SSP54_E4}) out[n++] = (double)x;
}
double orc_wenoz(double a, double b, double c, double d, double e, double eps) {
  return (double)wenoz(a, b, c, d, e, eps);
}
double orc_vl_slope(double l, double c, double r) { return (double)vl_slope(l, c, r); }
double orc_mp5(double a, double b, double c, double d, double e) { return (double)mp5(a, b, c, d, e); }
void orc_ppmx_edges(double a, double b, double c, double d, double e, double* aL, double* aR) {
  real l, r;
  ppmx_edges(a, b, c, d, e, l, r);
  *aL = (double)l;
  *aR = (double)r;
}
void orc_ppm_edges(double a, double b, double c, double d, double e, double* aL, double* aR) {
  real l, r;
  ppm_edges(a, b, c, d, e, l, r);
  *aL = (double)l;
  *aR = (double)r;
}

// ---- operation counts (counting build; zeros otherwise) ----

static void tally_out(long long* out) {
#ifdef ORACLE_COUNTING
  out[0] = g_flops.add; out[1] = g_flops.mul; out[2] = g_flops.div;
  out[3] = g_flops.sqrt; out[4] = g_flops.trans;
  g_flops = FlopTally();
#else
  for (int q = 0; q < 5; q++) out[q] = 0;
#endif
}

static void tally_reset() {
#ifdef ORACLE_COUNTING
  g_flops = FlopTally();
#endif
}

// Operations of one face flux along d at zone (i, j, k) of the given prims
// (ghosts filled first, outside the count): reconstruction of the 8 prims,
// both face states, fluxes, conserved variables, speeds and the LLF flux.
void orc_count_face(const orc_cfg* c, const double* prims, int d, int i, int j, int k, long long* out) {
  Grid g(*c);
  std::vector<real> P;
  load(g, prims, P);
  fill_ghosts(g, P);
  real f[NV];
  tally_reset();
  face_flux(g, P, g.c.recon, d, i, j, k, f);
  tally_out(out);
}

// Operations of the EMF and corrected-B-flux work of one zone (three edges,
// six rebuilt fluxes) are counted analytically by the caller; this counts
// one zone's update: source, flux divergence, RK combination (stage 1, with
// U(P)) and the inversion.
void orc_count_zone_update(const orc_cfg* c, const double* prims, int i, int j, int k, double dt,
                           long long* out) {
  Grid g(*c);
  std::vector<real> P;
  load(g, prims, P);
  fill_ghosts(g, P);
  std::vector<real> F[3];
  for (int d = 0; d < 3; d++) F[d].assign(NV * g.nz, 0.0);
  compute_fluxes(g, P, F);
  flux_ct(g, F);
  real p[NV], L[NV], u0[NV], U[NV], pn[NV];
  for (int v = 0; v < NV; v++) p[v] = Vc(P, g, v, i, j, k);
  tally_reset();
  rhs(g, F, p, i, j, k, L);
  cons_at(g, p, i, j, u0);
  for (int v = 0; v < NV; v++) U[v] = u0[v] + (real)dt * L[v];
  invert(g.c, g.gC[g.id2(i, j)], U, p, pn);
  tally_out(out);
}

}  // extern "C"
