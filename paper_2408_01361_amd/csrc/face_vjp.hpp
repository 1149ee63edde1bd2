// Reverse-mode derivatives for the adjoint, of one face state (its flux
// along D, conserved variables and two fast signal speeds, as fluid_state /
// prim_to_flux / char_speeds form them) and of one zone's local terms (its
// geometric source and conserved variables): given the adjoints of those
// outputs, the adjoint of the prims q and of the adiabatic index.  One
// forward evaluation that keeps its intermediates (FluidTape), then one
// reverse sweep through them in the opposite order: this replaces one
// dual-number evaluation per prim.
//
// Included by adjoint.hpp (and by host tests) after physics.hpp, where the
// library's names are visible.
#pragma once

// The quantities of one state that its reverse sweeps need: four-velocity,
// field four-vector (both components), b^t, the Lorentz factor, b^2, gas
// pressure, enthalpy density w = rho + u + p + b^2 and total pressure.
struct FluidTape {
  double ucon[4], ucov[4], bcon[4], bcov[4], bt, gamma, bsq, pg, w, ptot;
};
// Adjoints accumulated by the reverse sweeps (B_b[0] unused).
struct FluidAdj {
  double ucon[4], ucov[4], bcon[4], bcov[4], B[4], rho, uu, gam, w, ptot, pg, bsq;
};

__device__ __forceinline__ void fluid_fwd(const double q[NVAR], const PointMetric<double>& m, double gam,
                                          FluidTape& t) {
  auto gc = [&](int a, int b) { return m.gcov[sidx(a, b)]; };
  const double v[4] = {0.0, q[U1], q[U2], q[U3]};
  const double Bp[4] = {0.0, q[B1], q[B2], q[B3]};
  double qsq = 0.0;
#pragma unroll
  for (int i = 1; i < 4; i++)
#pragma unroll
    for (int j = 1; j < 4; j++) qsq += gc(i, j) * v[i] * v[j];
  t.gamma = sqrt(1.0 + qsq);
  t.ucon[0] = t.gamma / m.alpha;
#pragma unroll
  for (int i = 1; i < 4; i++) t.ucon[i] = v[i] - t.gamma * m.alpha * m.gcon[sidx(0, i)];
#pragma unroll
  for (int a = 0; a < 4; a++) {
    t.ucov[a] = 0.0;
#pragma unroll
    for (int b = 0; b < 4; b++) t.ucov[a] += gc(a, b) * t.ucon[b];
  }
  t.bt = 0.0;
#pragma unroll
  for (int i = 1; i < 4; i++) t.bt += Bp[i] * t.ucov[i];
  t.bcon[0] = t.bt;
#pragma unroll
  for (int i = 1; i < 4; i++) t.bcon[i] = (Bp[i] + t.bt * t.ucon[i]) / t.ucon[0];
#pragma unroll
  for (int a = 0; a < 4; a++) {
    t.bcov[a] = 0.0;
#pragma unroll
    for (int b = 0; b < 4; b++) t.bcov[a] += gc(a, b) * t.bcon[b];
  }
  t.bsq = 0.0;
#pragma unroll
  for (int a = 0; a < 4; a++) t.bsq += t.bcon[a] * t.bcov[a];
  t.pg = (gam - 1.0) * q[UU];
  t.w = ((q[RHO] + q[UU]) + t.pg) + t.bsq;
  t.ptot = t.pg + 0.5 * t.bsq;
}

__device__ __forceinline__ void adj_zero(FluidAdj& a) {
#pragma unroll
  for (int k = 0; k < 4; k++) a.ucon[k] = a.ucov[k] = a.bcon[k] = a.bcov[k] = a.B[k] = 0.0;
  a.rho = a.uu = a.gam = a.w = a.ptot = a.pg = a.bsq = 0.0;
}

// Adjoint of row e of the stress-energy part, given the adjoints Y of
// Y[RHO] = g rho u^e, Y[UU] = g (T^e_t + rho u^e), Y[U_i] = g T^e_i with
// T^e_nu = w u^e u_nu + ptot delta^e_nu - b^e b_nu.
__device__ __forceinline__ void adj_row(int e, const double Y[NVAR], double g, double rho, const FluidTape& t,
                                        FluidAdj& a) {
  double Xb[4];
  Xb[0] = g * Y[UU];
#pragma unroll
  for (int i = 1; i < 4; i++) Xb[i] = g * Y[U1 + i - 1];
  const double rb = g * (Y[RHO] + Y[UU]);   // adjoint of rho u^e
  a.rho += rb * t.ucon[e];
  a.ucon[e] += rb * rho;
#pragma unroll
  for (int n = 0; n < 4; n++) {
    a.w += Xb[n] * t.ucon[e] * t.ucov[n];
    a.ucon[e] += Xb[n] * t.w * t.ucov[n];
    a.ucov[n] += Xb[n] * t.w * t.ucon[e];
    a.bcon[e] -= Xb[n] * t.bcov[n];
    a.bcov[n] -= Xb[n] * t.bcon[e];
  }
  a.ptot += Xb[e];
}

// The common tail of the reverse sweeps: from the adjoints of the tape's
// quantities to those of the prims (qb) and of the adiabatic index (gamb).
__device__ __forceinline__ void fluid_rev(const double q[NVAR], const PointMetric<double>& m, double gam,
                                          const FluidTape& t, FluidAdj& a, double qb[NVAR], double& gamb) {
  auto gc = [&](int x, int y) { return m.gcov[sidx(x, y)]; };
  const double v[4] = {0.0, q[U1], q[U2], q[U3]};
  const double Bp[4] = {0.0, q[B1], q[B2], q[B3]};
  // ptot = pg + bsq/2, w = rho + u + pg + bsq, pg = (gam - 1) u
  a.pg += a.ptot + a.w;
  a.bsq += 0.5 * a.ptot + a.w;
  a.rho += a.w;
  a.uu += a.w + a.pg * (gam - 1.0);
  a.gam += a.pg * q[UU];
  // bsq = b^a b_a
#pragma unroll
  for (int k = 0; k < 4; k++) {
    a.bcon[k] += a.bsq * t.bcov[k];
    a.bcov[k] += a.bsq * t.bcon[k];
  }
  // b_a = g_ab b^b
#pragma unroll
  for (int y = 0; y < 4; y++)
#pragma unroll
    for (int x = 0; x < 4; x++) a.bcon[y] += gc(x, y) * a.bcov[x];
  // b^i = (B^i + bt u^i) / u^t, b^t = bt
  double bt_b = a.bcon[0];
#pragma unroll
  for (int i = 1; i < 4; i++) {
    const double f = a.bcon[i] / t.ucon[0];
    a.B[i] += f;
    bt_b += f * t.ucon[i];
    a.ucon[i] += f * t.bt;
    a.ucon[0] -= f * t.bcon[i];
  }
  // bt = B^i u_i
#pragma unroll
  for (int i = 1; i < 4; i++) {
    a.B[i] += bt_b * t.ucov[i];
    a.ucov[i] += bt_b * Bp[i];
  }
  // u_a = g_ab u^b
#pragma unroll
  for (int y = 0; y < 4; y++)
#pragma unroll
    for (int x = 0; x < 4; x++) a.ucon[y] += gc(x, y) * a.ucov[x];
  // u^t = gamma / alpha, u^i = v^i - gamma alpha g^{ti}
  double gamma_b = a.ucon[0] / m.alpha;
  double v_b[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 1; i < 4; i++) {
    v_b[i] += a.ucon[i];
    gamma_b -= a.ucon[i] * m.alpha * m.gcon[sidx(0, i)];
  }
  // gamma = sqrt(1 + g_ij v^i v^j)
  const double qsq_b = 0.5 * gamma_b / t.gamma;
#pragma unroll
  for (int i = 1; i < 4; i++)
#pragma unroll
    for (int j = 1; j < 4; j++) v_b[i] += 2.0 * qsq_b * gc(i, j) * v[j];
  qb[RHO] = a.rho;
  qb[UU] = a.uu;
  qb[U1] = v_b[1];
  qb[U2] = v_b[2];
  qb[U3] = v_b[3];
  qb[B1] = a.B[1];
  qb[B2] = a.B[2];
  qb[B3] = a.B[3];
  gamb = a.gam;
}

// One face state: flux along D (adjoint Fb), conserved variables (Ub) and
// the two fast speeds (cpb, cmb).
template <int D>
__device__ __forceinline__ void state_vjp(const double q[NVAR], const PointMetric<double>& m, double gam,
                                          const double Fb[NVAR], const double Ub[NVAR], double cpb,
                                          double cmb, double qb[NVAR], double& gamb) {
  auto gu = [&](int x, int y) { return m.gcon[sidx(x, y)]; };
  const double rho = q[RHO], uu = q[UU], g = m.gdet;
  FluidTape t;
  fluid_fwd(q, m, gam, t);
  FluidAdj a;
  adj_zero(a);
  // the speeds first (forward and reverse), so that their intermediates
  // are dead before the flux part
  {
    // speeds: roots of A v^2 + B v + C = 0
    const double we = rho + gam * uu;
    const double cs2 = gam * t.pg / we;
    const double S = t.bsq + we;
    const double va2 = t.bsq / S;
    const double c2 = (cs2 + va2) - cs2 * va2;
    const double Au = t.ucon[D], Bu = t.ucon[0];
    const double Asq = gu(D, D), Bsq = gu(0, 0), AB = gu(0, D);
    const double A = Bu * Bu - c2 * (Bsq + Bu * Bu);
    const double Bq = -2.0 * (Au * Bu - c2 * (AB + Au * Bu));
    const double C = Au * Au - c2 * (Asq + Au * Au);
    double disc = Bq * Bq - (4.0 * A) * C;
    disc = disc > 0.0 ? disc : 0.0;
    const double sq = sqrt(disc);
    const double r1 = (-Bq + sq) / (2.0 * A), r2 = (-Bq - sq) / (2.0 * A);
    // reverse: cp = max(r1, r2), cm = min(r1, r2)
    const bool first = r1 > r2;
    const double r1b = first ? cpb : cmb, r2b = first ? cmb : cpb;
    const double i2a = 1.0 / (2.0 * A);
    double Ab = -(r1b * r1 + r2b * r2) / A;
    double Bb = -(r1b + r2b) * i2a;
    const double sqb = (r1b - r2b) * i2a;
    const double discb = sq > 0.0 ? 0.5 * sqb / sq : 0.0;
    Bb += discb * 2.0 * Bq;
    Ab -= discb * 4.0 * C;
    const double Cb = -discb * 4.0 * A;
    const double Qb = -2.0 * Bb;   // Bq = -2 Q, Q = Au Bu - c2 (AB + Au Bu)
    const double c2b = -Ab * (Bsq + Bu * Bu) - Qb * (AB + Au * Bu) - Cb * (Asq + Au * Au);
    a.ucon[0] += Ab * (2.0 * Bu - 2.0 * c2 * Bu) + Qb * (Au - c2 * Au);
    a.ucon[D] += Qb * (Bu - c2 * Bu) + Cb * (2.0 * Au - 2.0 * c2 * Au);
    const double cs2b = c2b * (1.0 - va2), va2b = c2b * (1.0 - cs2);
    a.gam += cs2b * t.pg / we;
    a.pg += cs2b * gam / we;
    double web = -cs2b * cs2 / we;
    a.bsq += va2b * we / (S * S);
    web -= va2b * t.bsq / (S * S);
    a.rho += web;
    a.uu += web * gam;
    a.gam += web * uu;
  }
  // flux (row D) and conserved variables (row 0)
  adj_row(D, Fb, g, rho, t, a);
  adj_row(0, Ub, g, rho, t, a);
  // field slots: F[B_k] = g (b^k u^D - b^D u^k), U[B_k] = g B^k
#pragma unroll
  for (int k = 1; k < 4; k++) {
    const double y = g * Fb[B1 + k - 1];
    a.bcon[k] += y * t.ucon[D];
    a.ucon[D] += y * t.bcon[k];
    a.bcon[D] -= y * t.ucon[k];
    a.ucon[k] -= y * t.bcon[D];
    a.B[k] += g * Ub[B1 + k - 1];
  }
  fluid_rev(q, m, gam, t, a, qb, gamb);
}

// One zone: the geometric source sqrt(-g) T^k_l Gamma^l_{nu k} (adjoint Sb,
// nu = 0..3; cn the connection, Gamma^l_{mn} at l * 10 + sidx(m, n)) and,
// when Ub is not null, the conserved variables (adjoint Ub).
__device__ __forceinline__ void zone_vjp(const double q[NVAR], const PointMetric<double>& m, double gam,
                                         const double cn[40], const double Sb[4], const double* Ub,
                                         double qb[NVAR], double& gamb) {
  const double rho = q[RHO], g = m.gdet;
  FluidTape t;
  fluid_fwd(q, m, gam, t);
  FluidAdj a;
  adj_zero(a);
  // T^k_l: adjoint g sum_nu Sb_nu Gamma^l_{nu k}
#pragma unroll
  for (int k = 0; k < 4; k++)
#pragma unroll
    for (int l = 0; l < 4; l++) {
      double Tb = 0.0;
#pragma unroll
      for (int nu = 0; nu < 4; nu++) Tb += Sb[nu] * cn[l * 10 + sidx(nu, k)];
      Tb *= g;
      // T^k_l = w u^k u_l + ptot delta^k_l - b^k b_l
      a.w += Tb * t.ucon[k] * t.ucov[l];
      a.ucon[k] += Tb * t.w * t.ucov[l];
      a.ucov[l] += Tb * t.w * t.ucon[k];
      if (k == l) a.ptot += Tb;
      a.bcon[k] -= Tb * t.bcov[l];
      a.bcov[l] -= Tb * t.bcon[k];
    }
  if (Ub) {
    adj_row(0, Ub, g, rho, t, a);
#pragma unroll
    for (int k = 1; k < 4; k++) a.B[k] += g * Ub[B1 + k - 1];
  }
  fluid_rev(q, m, gam, t, a, qb, gamb);
}
