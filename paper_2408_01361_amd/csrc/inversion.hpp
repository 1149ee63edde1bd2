// Recovery of the primitive variables from the conserved ones, per zone:
// the 1D_W Newton solve, the Kastaun et al. bracketed recovery and the
// implicit solver's Newton-Raphson, with the dispatcher the update calls.
// Device code written so that it also compiles as plain C++ on the host
// (the sanitizer test builds it there): it uses only Dev's scalar fields,
// the per-point physics and <math.h>.
//
// Included inside the anonymous namespace of grmhd.hip.

// ---------------------------------------------------------------- U -> P --

// 1D_W (Noble et al. 2006) Newton solve for W = w gamma^2 with the normal
// observer n_mu = (-alpha, 0, 0, 0): D = alpha U_rho/sqrt(-g),
// Q_mu = alpha T^t_mu, Bn^i = alpha B^i.  Residual
//   Q.n + W - p(W) + Bn^2 (1 + v^2)/2 - (Q.Bn)^2/(2 W^2),
//   v^2 = [Qt^2 W^2 + (Q.Bn)^2 (Bn^2 + 2W)] / [(Bn^2 + W)^2 W^2],
//   p = (gam-1)/gam [W (1 - v^2) - D sqrt(1 - v^2)].
// Start from the guess's W (doubled while v^2 >= 1); steps leaving W > 0,
// v^2 < 1 are halved (at most 20 times); stop at |dW| < tol W or maxit, then
// one more step.  Returns 1 (and the guess's hydro prims) on failure.
__device__ int invert_1dw(const Dev& g, const PointMetric<double>& m, const double U[NVAR],
                          const double guess[NVAR], double P[NVAR]) {
#pragma clang fp contract(off)
  const double gam = g.gam;
  const double gd = m.gdet;
  P[B1] = U[B1] / gd;
  P[B2] = U[B2] / gd;
  P[B3] = U[B3] / gd;
  const double al = m.alpha;
  const double D = al * U[RHO] / gd;
  double Q[4] = {al * (U[UU] / gd - U[RHO] / gd), al * U[U1] / gd, al * U[U2] / gd, al * U[U3] / gd};
  double Bn1 = al * P[B1], Bn2 = al * P[B2], Bn3 = al * P[B3];
  // n^mu = g^{mu t} (-alpha); Q^mu = g^{mu nu} Q_nu
  double ncon[4], Qup[4];
#pragma unroll
  for (int a = 0; a < 4; a++) {
    ncon[a] = -al * m.gcon[sidx(a, 0)];
    Qup[a] = m.gcon[sidx(a, 0)] * Q[0] + m.gcon[sidx(a, 1)] * Q[1] + m.gcon[sidx(a, 2)] * Q[2] +
             m.gcon[sidx(a, 3)] * Q[3];
  }
  double Qn = Q[0] * ncon[0] + Q[1] * ncon[1] + Q[2] * ncon[2] + Q[3] * ncon[3];
  double QQ = Q[0] * Qup[0] + Q[1] * Qup[1] + Q[2] * Qup[2] + Q[3] * Qup[3];
  double QB = Q[1] * Bn1 + Q[2] * Bn2 + Q[3] * Bn3;
  double Bsq = m.gcov[sidx(1, 1)] * Bn1 * Bn1 + m.gcov[sidx(2, 2)] * Bn2 * Bn2 +
               m.gcov[sidx(3, 3)] * Bn3 * Bn3 +
               2.0 * (m.gcov[sidx(1, 2)] * Bn1 * Bn2 + m.gcov[sidx(1, 3)] * Bn1 * Bn3 +
                      m.gcov[sidx(2, 3)] * Bn2 * Bn3);
  // |Q projected orthogonal to n|^2 is non-negative; roundoff below zero is cleared
  double Qt2 = fmax(QQ + Qn * Qn, 0.0);
  double QB2 = QB * QB;
  const double gf = (gam - 1.0) / gam;

  auto vsq = [&](double W) {
    double WB = Bsq + W;
    return (Qt2 * W * W + QB2 * (Bsq + 2.0 * W)) / (WB * WB * W * W);
  };
  auto step = [&](double W) {
    double v2 = vsq(W);
    double sq = sqrt(1.0 - v2);
    double pr = gf * (W * (1.0 - v2) - D * sq);
    double W2 = W * W, WB = W + Bsq;
    double f = Qn + W - pr + 0.5 * Bsq * (1.0 + v2) - QB2 / (2.0 * W2);
    double dv2 = -2.0 * (Qt2 + QB2 * (3.0 * W * W + 3.0 * W * Bsq + Bsq * Bsq) / (W2 * W)) / (WB * WB * WB);
    double dpdW = gf * (1.0 - v2);
    double dpdv2 = gf * (-W + D / (2.0 * sq));
    double df = 1.0 - (dpdW + dpdv2 * dv2) + 0.5 * Bsq * dv2 + QB2 / (W2 * W);
    return -f / df;
  };
  auto fail = [&]() {
#pragma unroll
    for (int v = 0; v < 5; v++) P[v] = guess[v];
    return 1;
  };

  const double g1 = guess[U1], g2 = guess[U2], g3 = guess[U3];
  double qsq = m.gcov[sidx(1, 1)] * g1 * g1 + m.gcov[sidx(2, 2)] * g2 * g2 + m.gcov[sidx(3, 3)] * g3 * g3 +
               2.0 * (m.gcov[sidx(1, 2)] * g1 * g2 + m.gcov[sidx(1, 3)] * g1 * g3 +
                      m.gcov[sidx(2, 3)] * g2 * g3);
  double W = (guess[RHO] + gam * guess[UU]) * (1.0 + qsq);
  for (int b = 0; b < 60 && !(vsq(W) < 1.0); b++) W *= 2.0;
  bool conv = false;
  for (int it = 0; it < g.maxit; it++) {
    double dW = step(W);
    double Wn = W + dW;
    for (int b = 0; b < 20 && !(Wn > 0.0 && vsq(Wn) < 1.0); b++) {
      dW *= 0.5;
      Wn = W + dW;
    }
    if (!isfinite(Wn) || Wn <= 0.0) return fail();
    W = Wn;
    if (fabs(dW) < g.tol * fabs(W)) {
      conv = true;
      break;
    }
  }
  if (!conv) return fail();
  W += step(W);
  if (!isfinite(W) || W <= 0.0) return fail();
  double v2 = vsq(W);
  if (!(v2 >= 0.0 && v2 < 1.0)) return fail();
  double gamma = 1.0 / sqrt(1.0 - v2);
  double rho = D / gamma;
  double u = (W * (1.0 - v2) - rho) / gam;
  if (!(rho > 0.0) || !(u > 0.0)) return fail();
  double pre = gamma / (W + Bsq);
  double ut1 = pre * ((Qup[1] + ncon[1] * Qn) + QB * Bn1 / W);
  double ut2 = pre * ((Qup[2] + ncon[2] * Qn) + QB * Bn2 / W);
  double ut3 = pre * ((Qup[3] + ncon[3] * Qn) + QB * Bn3 / W);
  if (!isfinite(ut1) || !isfinite(ut2) || !isfinite(ut3)) return fail();
  P[RHO] = rho;
  P[UU] = u;
  P[U1] = ut1;
  P[U2] = ut2;
  P[U3] = ut3;
  return 0;
}

// Kastaun et al. (2021) recovery, the bracketed alternative to 1D_W (the
// Algorithm section names it among the robust inversions).  With D, the
// spatial projection S of Q and Bn as in 1D_W, scaled by D:
//   r^2 = S.S/D^2, b^2 = Bn.Bn/D, rb = S.Bn/D^(3/2), q = -Q.n/D - 1,
// all fluid quantities are functions of mu = 1/(h W):
//   x = 1/(1 + mu b^2), rbar^2 = x^2 r^2 + mu x (1 + x) rb^2,
//   qbar = q - b^2/2 - mu^2 x^2 (b^2 r^2 - rb^2)/2,
//   v^2 = min(mu^2 rbar^2, vmax^2), W = (1 - v^2)^(-1/2), rho = D/W,
//   eps = max(W (qbar - mu rbar^2) + v^2 W^2/(1 + W), 0),
//   a = (gam - 1) eps/(1 + eps),
//   nu = max((1 + a)(1 + eps)/W, (1 + a)(1 + qbar - mu rbar^2)),
// and mu solves mu = 1/(nu + mu rbar^2).  h >= 1 bounds mu by mu+, the root
// of mu sqrt(1 + rbar^2(mu)) = 1 (found first, to 1e-12, then widened by
// 1e-10); the root in [0, mu+] is bracketed and taken by the Illinois
// (modified regula falsi) iteration to |d mu| <= tol mu, at most 4 maxit
// iterations each.  No guess is used except as the failure value (the
// guess's hydro prims, as in 1D_W).  Evaluated in the same operation order
// as the CPU reference of the method, without contraction.
__device__ int invert_kastaun(const Dev& g, const PointMetric<double>& m, const double U[NVAR],
                              const double guess[NVAR], double P[NVAR]) {
#pragma clang fp contract(off)
  const double gam = g.gam;
  const double gd = m.gdet;
  P[B1] = U[B1] / gd;
  P[B2] = U[B2] / gd;
  P[B3] = U[B3] / gd;
  auto fail = [&]() {
#pragma unroll
    for (int v = 0; v < 5; v++) P[v] = guess[v];
    return 1;
  };
  const double al = m.alpha;
  const double D = al * U[RHO] / gd;
  if (!(D > 0.0) || !isfinite(D)) return fail();
  double Q[4] = {al * (U[UU] / gd - U[RHO] / gd), al * U[U1] / gd, al * U[U2] / gd, al * U[U3] / gd};
  const double Bn[4] = {0.0, al * P[B1], al * P[B2], al * P[B3]};
  double ncon[4], Qup[4];
#pragma unroll
  for (int a = 0; a < 4; a++) {
    ncon[a] = m.gcon[sidx(a, 0)] * -al;
    Qup[a] = m.gcon[sidx(a, 0)] * Q[0] + m.gcon[sidx(a, 1)] * Q[1] + m.gcon[sidx(a, 2)] * Q[2] +
             m.gcon[sidx(a, 3)] * Q[3];
  }
  const double Qn = Q[0] * ncon[0] + Q[1] * ncon[1] + Q[2] * ncon[2] + Q[3] * ncon[3];
  const double QQ = Q[0] * Qup[0] + Q[1] * Qup[1] + Q[2] * Qup[2] + Q[3] * Qup[3];
  const double QB = Q[1] * Bn[1] + Q[2] * Bn[2] + Q[3] * Bn[3];
  double Bsq = 0.0;
#pragma unroll
  for (int a = 1; a < 4; a++)
#pragma unroll
    for (int b = 1; b < 4; b++) Bsq += m.gcov[sidx(a, b)] * Bn[a] * Bn[b];
  const double Ssq = fmax(QQ + Qn * Qn, 0.0);
  const double r2 = Ssq / (D * D), b2 = Bsq / D, rb = QB / (D * sqrt(D)), q = -Qn / D - 1.0;
  const double rb2 = rb * rb;
  const double vmax2 = g.vmax2;
  const int maxit = 4 * g.maxit;

  struct St {
    double x, rbar2, qbar, W, eps, nu;
  };
  auto state = [&](double mu) {
    St s;
    s.x = 1.0 / (1.0 + mu * b2);
    s.rbar2 = s.x * s.x * r2 + mu * s.x * (1.0 + s.x) * rb2;
    s.qbar = q - 0.5 * b2 - 0.5 * (mu * mu) * (s.x * s.x) * (b2 * r2 - rb2);
    double v2 = fmin(mu * mu * s.rbar2, vmax2);
    s.W = 1.0 / sqrt(1.0 - v2);
    s.eps = fmax(s.W * (s.qbar - mu * s.rbar2) + v2 * s.W * s.W / (1.0 + s.W), 0.0);
    double a = (gam - 1.0) * s.eps / (1.0 + s.eps);
    s.nu = fmax((1.0 + a) * (1.0 + s.eps) / s.W, (1.0 + a) * (1.0 + s.qbar - mu * s.rbar2));
    return s;
  };
  auto f = [&](double mu) {
    St s = state(mu);
    return mu - 1.0 / (s.nu + mu * s.rbar2);
  };
  auto fa = [&](double mu) {
    double x = 1.0 / (1.0 + mu * b2);
    double rbar2 = x * x * r2 + mu * x * (1.0 + x) * rb2;
    return mu * sqrt(1.0 + rbar2) - 1.0;
  };
  // root of h in [lo, hi] with h(lo) < 0 <= h(hi); false after maxit steps
  auto illinois = [&](auto h, double lo, double hi, double hlo, double hhi, double tol, double& root) {
    int side = 0;
    double prev = hi;
    for (int it = 0; it < maxit; it++) {
      double mid = (lo * hhi - hi * hlo) / (hhi - hlo);
      if (!(mid > lo && mid < hi)) mid = 0.5 * (lo + hi);
      double hm = h(mid);
      if (hm == 0.0 || fabs(mid - prev) <= tol * mid) {
        root = mid;
        return true;
      }
      prev = mid;
      if (hm < 0.0) {
        lo = mid;
        hlo = hm;
        if (side == -1) hhi = 0.5 * hhi;
        side = -1;
      } else {
        hi = mid;
        hhi = hm;
        if (side == 1) hlo = 0.5 * hlo;
        side = 1;
      }
    }
    return false;
  };
  double mup;
  if (!illinois(fa, 0.0, 1.0, -1.0, fa(1.0), 1e-12, mup)) return fail();
  mup = fmin(mup * (1.0 + 1e-10), 1.0);
  const double f0 = f(0.0), f1 = f(mup);
  if (!(f0 < 0.0) || !(f1 >= 0.0)) return fail();
  double mu = mup;
  if (f1 != 0.0 && !illinois(f, 0.0, mup, f0, f1, g.tol, mu)) return fail();
  St s = state(mu);
  const double rho = D / s.W;
  const double u = rho * s.eps;
  // eps clamped at 0 stands when floors are on: the energy floor raises u
  if (!(rho > 0.0) || !(u > 0.0 || (g.floors && u == 0.0)) || !isfinite(u)) return fail();
  const double pre = s.W * mu * s.x / D;
  double ut[3];
#pragma unroll
  for (int a = 1; a < 4; a++) {
    ut[a - 1] = pre * ((Qup[a] + ncon[a] * Qn) + mu * QB * Bn[a] / D);
    if (!isfinite(ut[a - 1])) return fail();
  }
  P[RHO] = rho;
  P[UU] = u;
  P[U1] = ut[0];
  P[U2] = ut[1];
  P[U3] = ut[2];
  return 0;
}

// The implicit solver's per-zone Newton-Raphson used as the recovery
// (Implicit Solver section: with every fluid variable implicit and only
// ideal sources it solves U(P) = U* zone by zone).  Unknowns x = (rho, u,
// u~1, u~2, u~3), B from U*; residual R(x) = (U(x) - U*)_{0..4} / s, s the
// largest |U*_k|; Jacobian by forward differences (secant) with steps
// h_k = 1e-7 max(|x_k|, f_k), f = (0, 0, 1e-3, 1e-3, 1e-3); the step from a
// Householder QR of J with column pivoting (largest remaining column norm
// first, ties to the lower index); backtracking line search lambda = 1,
// 1/2, ... (at most 8 halvings) until rho, u > 0 and |R| decreases (the last
// try is taken otherwise, if rho, u > 0); converged when every |lambda dx_k|
// <= max(tol, 1e-12) max(|x_k|, f_k) (near the root the residual's roundoff
// makes ~1e-13 steps), failure after maxit iterations or on non-finite
// values keeps the guess.  Unrolled so that the 5 x 5 system stays in
// registers (no dynamic indexing); same operation order as the CPU
// reference of the method, without contraction.
__device__ __forceinline__ void implicit_residual(const Dev& g, const PointMetric<double>& m, const double x[5],
                                                  const double B[3], const double Us[NVAR], double scale,
                                                  double R[5]) {
#pragma clang fp contract(off)
  const double P[NVAR] = {x[0], x[1], x[2], x[3], x[4], B[0], B[1], B[2]};
  Fluid<double> f;
  fluid_state(P, m, f);
  double U[NVAR];
  prim_to_flux(P, f, m, g.gam, 0, U);
#pragma unroll
  for (int k = 0; k < 5; k++) R[k] = (U[k] - Us[k]) / scale;
}

// A 5 x 5 matrix of one thread held in LDS: element (i, j) at
// base[(5 i + j) BLOCK], base = the workgroup's array + threadIdx.x, so the
// lanes of a wavefront touch consecutive words.  The Newton system lives
// here rather than in registers, which keeps the solver's register budget
// far from the per-wave limit.
struct LdsMat {
  double* base;
  __device__ __forceinline__ double& operator()(int i, int j) const { return base[(i * 5 + j) * BLOCK]; }
};

__device__ __forceinline__ bool qr_pivot_solve(const LdsMat& A, double b[5], double y[5]) {
#pragma clang fp contract(off)
  int perm[5] = {0, 1, 2, 3, 4};
  double cn[5];
#pragma unroll
  for (int j = 0; j < 5; j++) {
    cn[j] = 0.0;
#pragma unroll
    for (int i = 0; i < 5; i++) cn[j] += A(i, j) * A(i, j);
  }
#pragma unroll
  for (int k = 0; k < 5; k++) {
    int best = k;
    double cb = cn[k];
#pragma unroll
    for (int j = k + 1; j < 5; j++)
      if (cn[j] > cb) {
        cb = cn[j];
        best = j;
      }
#pragma unroll
    for (int j = k + 1; j < 5; j++)
      if (j == best) {
#pragma unroll
        for (int i = 0; i < 5; i++) {
          const double t = A(i, k);
          A(i, k) = A(i, j);
          A(i, j) = t;
        }
        const double t = cn[k];
        cn[k] = cn[j];
        cn[j] = t;
        const int tp = perm[k];
        perm[k] = perm[j];
        perm[j] = tp;
      }
    double nrm = 0.0;
#pragma unroll
    for (int i = k; i < 5; i++) nrm += A(i, k) * A(i, k);
    nrm = sqrt(nrm);
    if (!(nrm > 0.0) || !isfinite(nrm)) return false;
    const double alpha = A(k, k) > 0.0 ? -nrm : nrm;
    double v[5];
#pragma unroll
    for (int i = 0; i < 5; i++) v[i] = i < k ? 0.0 : A(i, k);
    v[k] = v[k] - alpha;
    double vv = 0.0;
#pragma unroll
    for (int i = k; i < 5; i++) vv += v[i] * v[i];
    if (!(vv > 0.0)) return false;
#pragma unroll
    for (int j = k; j < 5; j++) {
      double d = 0.0;
#pragma unroll
      for (int i = k; i < 5; i++) d += v[i] * A(i, j);
      const double f = 2.0 * d / vv;
#pragma unroll
      for (int i = k; i < 5; i++) A(i, j) = A(i, j) - f * v[i];
    }
    double d = 0.0;
#pragma unroll
    for (int i = k; i < 5; i++) d += v[i] * b[i];
    const double f = 2.0 * d / vv;
#pragma unroll
    for (int i = k; i < 5; i++) b[i] = b[i] - f * v[i];
#pragma unroll
    for (int j = k + 1; j < 5; j++) {
      cn[j] = 0.0;
#pragma unroll
      for (int i = k + 1; i < 5; i++) cn[j] += A(i, j) * A(i, j);
    }
  }
  double z[5];
#pragma unroll
  for (int i = 4; i >= 0; i--) {
    double t = b[i];
#pragma unroll
    for (int j = i + 1; j < 5; j++) t = t - A(i, j) * z[j];
    if (!(fabs(A(i, i)) > 0.0)) return false;
    z[i] = t / A(i, i);
  }
#pragma unroll
  for (int mm = 0; mm < 5; mm++) {
    double val = 0.0;
#pragma unroll
    for (int k = 0; k < 5; k++)
      if (perm[k] == mm) val = z[k];
    y[mm] = val;
  }
#pragma unroll
  for (int k = 0; k < 5; k++)
    if (!isfinite(y[k])) return false;
  return true;
}

// jac: this thread's 25 LDS words for the Jacobian (LdsMat base).
__device__ __forceinline__ int invert_implicit(const Dev& g, const PointMetric<double>& m, const double U[NVAR],
                                               const double guess[NVAR], double P[NVAR], double* jac) {
#pragma clang fp contract(off)
  const double gd = m.gdet;
  P[B1] = U[B1] / gd;
  P[B2] = U[B2] / gd;
  P[B3] = U[B3] / gd;
  auto fail = [&]() {
#pragma unroll
    for (int v = 0; v < 5; v++) P[v] = guess[v];
    return 1;
  };
  const double B[3] = {P[B1], P[B2], P[B3]};
  double scale = 0.0;
#pragma unroll
  for (int k = 0; k < 5; k++)
    if (fabs(U[k]) > scale) scale = fabs(U[k]);
  if (!(scale > 0.0) || !isfinite(scale)) return fail();
  const double fl[5] = {0.0, 0.0, 1e-3, 1e-3, 1e-3};
  double x[5];
#pragma unroll
  for (int k = 0; k < 5; k++) x[k] = guess[k];
  if (!(x[0] > 0.0) || !(x[1] > 0.0)) return fail();
  double R[5];
  implicit_residual(g, m, x, B, U, scale, R);
  double r2 = 0.0;
#pragma unroll
  for (int k = 0; k < 5; k++) r2 += R[k] * R[k];
  bool conv = false;
  const double tol = g.tol > 1e-12 ? g.tol : 1e-12;
  const LdsMat J{jac};
  for (int it = 0; it < g.maxit && !conv; it++) {
    // secant Jacobian, one column per pass (components picked by compare,
    // so nothing in registers is indexed by the loop counter)
#pragma unroll 1
    for (int k = 0; k < 5; k++) {
      double xk = x[0], flk = fl[0];
#pragma unroll
      for (int mm = 1; mm < 5; mm++)
        if (mm == k) {
          xk = x[mm];
          flk = fl[mm];
        }
      const double ax = fabs(xk);
      const double h = 1e-7 * (ax > flk ? ax : flk);
      const double xkh = xk + h;
      double xp[5];
#pragma unroll
      for (int mm = 0; mm < 5; mm++) xp[mm] = mm == k ? xkh : x[mm];
      double Rp[5];
      implicit_residual(g, m, xp, B, U, scale, Rp);
      const double hh = xkh - xk;
#pragma unroll
      for (int mm = 0; mm < 5; mm++) J(mm, k) = (Rp[mm] - R[mm]) / hh;
    }
    double rhs[5], dx[5];
#pragma unroll
    for (int mm = 0; mm < 5; mm++) rhs[mm] = -R[mm];
    if (!qr_pivot_solve(J, rhs, dx)) return fail();
    double lam = 1.0, xn[5], Rn[5], rn2 = 0.0;
    bool ok = false;
    for (int ls = 0; ls <= 8; ls++) {
#pragma unroll
      for (int mm = 0; mm < 5; mm++) xn[mm] = x[mm] + lam * dx[mm];
      if (xn[0] > 0.0 && xn[1] > 0.0) {
        implicit_residual(g, m, xn, B, U, scale, Rn);
        rn2 = 0.0;
#pragma unroll
        for (int mm = 0; mm < 5; mm++) rn2 += Rn[mm] * Rn[mm];
        ok = isfinite(rn2);
        if (ok && rn2 < r2) break;
      } else {
        ok = false;
      }
      if (ls < 8) lam = 0.5 * lam;
    }
    if (!ok) return fail();
    conv = true;
#pragma unroll
    for (int mm = 0; mm < 5; mm++) {
      const double ax = fabs(xn[mm]);
      if (fabs(xn[mm] - x[mm]) > tol * (ax > fl[mm] ? ax : fl[mm])) conv = false;
      x[mm] = xn[mm];
      R[mm] = Rn[mm];
    }
    r2 = rn2;
  }
  if (!conv) return fail();
#pragma unroll
  for (int k = 0; k < 5; k++) {
    if (!isfinite(x[k])) return fail();
    P[k] = x[k];
  }
  return 0;
}

// The implicit solver's Newton iteration on the five hydro prims x from the
// guess x0 (rho, u > 0), with the steps, Jacobian, pivoted QR, line search
// and stopping rule of invert_implicit: res(x, R) fills the scaled residual
// R[5]; jac is this thread's 25 LDS words for the Jacobian (LdsMat base).
// Returns true with the root in x.  (invert_implicit keeps its own copy of
// the loop: compiled through this template, its kernel produced different
// and wrong states on torus steps, while this template gives parity here.)
template <typename Res>
__device__ __forceinline__ bool newton_hydro(const Dev& g, const double x0[5], Res res, double x[5],
                                             double* jac) {
#pragma clang fp contract(off)
  const double fl[5] = {0.0, 0.0, 1e-3, 1e-3, 1e-3};
#pragma unroll
  for (int k = 0; k < 5; k++) x[k] = x0[k];
  if (!(x[0] > 0.0) || !(x[1] > 0.0)) return false;
  double R[5];
  res(x, R);
  double r2 = 0.0;
#pragma unroll
  for (int k = 0; k < 5; k++) r2 += R[k] * R[k];
  bool conv = false;
  const double tol = g.tol > 1e-12 ? g.tol : 1e-12;
  const LdsMat J{jac};
  for (int it = 0; it < g.maxit && !conv; it++) {
    // secant Jacobian, one column per pass (components picked by compare,
    // so nothing in registers is indexed by the loop counter)
#pragma unroll 1
    for (int k = 0; k < 5; k++) {
      double xk = x[0], flk = fl[0];
#pragma unroll
      for (int mm = 1; mm < 5; mm++)
        if (mm == k) {
          xk = x[mm];
          flk = fl[mm];
        }
      const double ax = fabs(xk);
      const double h = 1e-7 * (ax > flk ? ax : flk);
      const double xkh = xk + h;
      double xp[5];
#pragma unroll
      for (int mm = 0; mm < 5; mm++) xp[mm] = mm == k ? xkh : x[mm];
      double Rp[5];
      res(xp, Rp);
      const double hh = xkh - xk;
#pragma unroll
      for (int mm = 0; mm < 5; mm++) J(mm, k) = (Rp[mm] - R[mm]) / hh;
    }
    double rhs[5], dx[5];
#pragma unroll
    for (int mm = 0; mm < 5; mm++) rhs[mm] = -R[mm];
    if (!qr_pivot_solve(J, rhs, dx)) return false;
    double lam = 1.0, xn[5], Rn[5], rn2 = 0.0;
    bool ok = false;
    for (int ls = 0; ls <= 8; ls++) {
#pragma unroll
      for (int mm = 0; mm < 5; mm++) xn[mm] = x[mm] + lam * dx[mm];
      if (xn[0] > 0.0 && xn[1] > 0.0) {
        res(xn, Rn);
        rn2 = 0.0;
#pragma unroll
        for (int mm = 0; mm < 5; mm++) rn2 += Rn[mm] * Rn[mm];
        ok = isfinite(rn2);
        if (ok && rn2 < r2) break;
      } else {
        ok = false;
      }
      if (ls < 8) lam = 0.5 * lam;
    }
    if (!ok) return false;
    conv = true;
#pragma unroll
    for (int mm = 0; mm < 5; mm++) {
      const double ax = fabs(xn[mm]);
      if (fabs(xn[mm] - x[mm]) > tol * (ax > fl[mm] ? ax : fl[mm])) conv = false;
      x[mm] = xn[mm];
      R[mm] = Rn[mm];
    }
    r2 = rn2;
  }
  if (!conv) return false;
#pragma unroll
  for (int k = 0; k < 5; k++)
    if (!isfinite(x[k])) return false;
  return true;
}

__device__ __forceinline__ int invert(const Dev& g, const PointMetric<double>& m, const double U[NVAR],
                                      const double guess[NVAR], double P[NVAR]) {
  if (g.inverter == GRMHD_INV_KASTAUN) return invert_kastaun(g, m, U, guess, P);
  return invert_1dw(g, m, U, guess, P);
}

