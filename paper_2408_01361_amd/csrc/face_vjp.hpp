// Reverse-mode derivative of one face state, for the adjoint: the state's
// flux along D, its conserved variables and its two fast signal speeds, as
// fluid_state / prim_to_flux / char_speeds form them from the prims q, the
// metric and the adiabatic index; given the adjoints of those outputs, the
// adjoint of q and of the adiabatic index.  One forward evaluation that keeps
// its intermediates, then one reverse sweep through them in the opposite
// order: this replaces one dual-number evaluation per prim.
//
// Included by adjoint.hpp (and by a host test) after physics.hpp, where the
// library's names are visible.
#pragma once

template <int D>
__device__ __forceinline__ void state_vjp(const double q[NVAR], const PointMetric<double>& m, double gam,
                                          const double Fb[NVAR], const double Ub[NVAR], double cpb,
                                          double cmb, double qb[NVAR], double& gamb) {
  auto gc = [&](int a, int b) { return m.gcov[sidx(a, b)]; };
  auto gu = [&](int a, int b) { return m.gcon[sidx(a, b)]; };
  const double rho = q[RHO], uu = q[UU];
  const double v[4] = {0.0, q[U1], q[U2], q[U3]};
  const double Bp[4] = {0.0, q[B1], q[B2], q[B3]};
  const double g = m.gdet, al = m.alpha;

  // ---- forward, keeping the intermediates
  double qsq = 0.0;
#pragma unroll
  for (int i = 1; i < 4; i++)
#pragma unroll
    for (int j = 1; j < 4; j++) qsq += gc(i, j) * v[i] * v[j];
  const double gamma = sqrt(1.0 + qsq);
  double ucon[4], ucov[4], bcon[4], bcov[4];
  ucon[0] = gamma / al;
#pragma unroll
  for (int i = 1; i < 4; i++) ucon[i] = v[i] - gamma * al * gu(0, i);
#pragma unroll
  for (int a = 0; a < 4; a++) {
    ucov[a] = 0.0;
#pragma unroll
    for (int b = 0; b < 4; b++) ucov[a] += gc(a, b) * ucon[b];
  }
  double bt = 0.0;
#pragma unroll
  for (int i = 1; i < 4; i++) bt += Bp[i] * ucov[i];
  bcon[0] = bt;
#pragma unroll
  for (int i = 1; i < 4; i++) bcon[i] = (Bp[i] + bt * ucon[i]) / ucon[0];
#pragma unroll
  for (int a = 0; a < 4; a++) {
    bcov[a] = 0.0;
#pragma unroll
    for (int b = 0; b < 4; b++) bcov[a] += gc(a, b) * bcon[b];
  }
  double bsq = 0.0;
#pragma unroll
  for (int a = 0; a < 4; a++) bsq += bcon[a] * bcov[a];
  const double pg = (gam - 1.0) * uu;
  const double w = ((rho + uu) + pg) + bsq;
  const double ptot = pg + 0.5 * bsq;
  // ---- reverse
  double ucon_b[4] = {0.0, 0.0, 0.0, 0.0}, ucov_b[4] = {0.0, 0.0, 0.0, 0.0};
  double bcon_b[4] = {0.0, 0.0, 0.0, 0.0}, bcov_b[4] = {0.0, 0.0, 0.0, 0.0};
  double B_b[4] = {0.0, 0.0, 0.0, 0.0};
  double rho_b = 0.0, uu_b = 0.0, gam_b = 0.0, w_b = 0.0, ptot_b = 0.0, pg_b = 0.0, bsq_b = 0.0;
  // the speeds first (forward and reverse), so that their intermediates
  // are dead before the flux part
  {
    // speeds: roots of A v^2 + B v + C = 0
    const double we = rho + gam * uu;
    const double cs2 = gam * pg / we;
    const double S = bsq + we;
    const double va2 = bsq / S;
    const double c2 = (cs2 + va2) - cs2 * va2;
    const double Au = ucon[D], Bu = ucon[0];
    const double Asq = gu(D, D), Bsq = gu(0, 0), AB = gu(0, D);
    const double A = Bu * Bu - c2 * (Bsq + Bu * Bu);
    const double Bq = -2.0 * (Au * Bu - c2 * (AB + Au * Bu));
    const double C = Au * Au - c2 * (Asq + Au * Au);
    double disc = Bq * Bq - (4.0 * A) * C;
    disc = disc > 0.0 ? disc : 0.0;
    const double sq = sqrt(disc);
    const double r1 = (-Bq + sq) / (2.0 * A), r2 = (-Bq - sq) / (2.0 * A);
    // reverse: cp = max(r1, r2), cm = min(r1, r2)
    {
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
      double c2b = -Ab * (Bsq + Bu * Bu) - Qb * (AB + Au * Bu) - Cb * (Asq + Au * Au);
      const double Bub = Ab * (2.0 * Bu - 2.0 * c2 * Bu) + Qb * (Au - c2 * Au);
      const double Aub = Qb * (Bu - c2 * Bu) + Cb * (2.0 * Au - 2.0 * c2 * Au);
      ucon_b[D] += Aub;
      ucon_b[0] += Bub;
      const double cs2b = c2b * (1.0 - va2), va2b = c2b * (1.0 - cs2);
      gam_b += cs2b * pg / we;
      pg_b += cs2b * gam / we;
      double web = -cs2b * cs2 / we;
      bsq_b += va2b * we / (S * S);
      web -= va2b * bsq / (S * S);
      rho_b += web;
      uu_b += web * gam;
      gam_b += web * uu;
    }
  }
  // flux (row D) and conserved variables (row 0):
  // X^e_nu = w u^e u_nu + ptot delta^e_nu - b^e b_nu;
  // Y[RHO] = g rho u^e, Y[UU] = g (X^e_0 + rho u^e), Y[U_i] = g X^e_i
#pragma unroll
  for (int r = 0; r < 2; r++) {
    const int e = r == 0 ? D : 0;
    const double* Y = r == 0 ? Fb : Ub;
    double Xb[4];
    Xb[0] = g * Y[UU];
#pragma unroll
    for (int i = 1; i < 4; i++) Xb[i] = g * Y[U1 + i - 1];
    const double rb = g * (Y[RHO] + Y[UU]);   // adjoint of rho u^e
    rho_b += rb * ucon[e];
    ucon_b[e] += rb * rho;
#pragma unroll
    for (int n = 0; n < 4; n++) {
      w_b += Xb[n] * ucon[e] * ucov[n];
      ucon_b[e] += Xb[n] * w * ucov[n];
      ucov_b[n] += Xb[n] * w * ucon[e];
      bcon_b[e] -= Xb[n] * bcov[n];
      bcov_b[n] -= Xb[n] * bcon[e];
    }
    ptot_b += Xb[e];
    if (r == 0) {
      // Y[B_k] = g (b^k u^D - b^D u^k)
#pragma unroll
      for (int k = 1; k < 4; k++) {
        const double y = g * Y[B1 + k - 1];
        bcon_b[k] += y * ucon[D];
        ucon_b[D] += y * bcon[k];
        bcon_b[D] -= y * ucon[k];
        ucon_b[k] -= y * bcon[D];
      }
    } else {
#pragma unroll
      for (int k = 1; k < 4; k++) B_b[k] += g * Y[B1 + k - 1];   // Y[B_k] = g B^k
    }
  }
  // ptot = pg + bsq/2, w = rho + u + pg + bsq, pg = (gam - 1) u
  pg_b += ptot_b + w_b;
  bsq_b += 0.5 * ptot_b + w_b;
  rho_b += w_b;
  uu_b += w_b + pg_b * (gam - 1.0);
  gam_b += pg_b * uu;
  // bsq = b^a b_a
#pragma unroll
  for (int a = 0; a < 4; a++) {
    bcon_b[a] += bsq_b * bcov[a];
    bcov_b[a] += bsq_b * bcon[a];
  }
  // b_a = g_ab b^b
#pragma unroll
  for (int b = 0; b < 4; b++)
#pragma unroll
    for (int a = 0; a < 4; a++) bcon_b[b] += gc(a, b) * bcov_b[a];
  // b^i = (B^i + bt u^i) / u^t, b^t = bt
  double bt_b = bcon_b[0];
#pragma unroll
  for (int i = 1; i < 4; i++) {
    const double f = bcon_b[i] / ucon[0];
    B_b[i] += f;
    bt_b += f * ucon[i];
    ucon_b[i] += f * bt;
    ucon_b[0] -= f * bcon[i];
  }
  // bt = B^i u_i
#pragma unroll
  for (int i = 1; i < 4; i++) {
    B_b[i] += bt_b * ucov[i];
    ucov_b[i] += bt_b * Bp[i];
  }
  // u_a = g_ab u^b
#pragma unroll
  for (int b = 0; b < 4; b++)
#pragma unroll
    for (int a = 0; a < 4; a++) ucon_b[b] += gc(a, b) * ucov_b[a];
  // u^t = gamma / alpha, u^i = v^i - gamma alpha g^{ti}
  double gamma_b = ucon_b[0] / al;
  double v_b[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 1; i < 4; i++) {
    v_b[i] += ucon_b[i];
    gamma_b -= ucon_b[i] * al * gu(0, i);
  }
  // gamma = sqrt(1 + g_ij v^i v^j)
  const double qsq_b = 0.5 * gamma_b / gamma;
#pragma unroll
  for (int i = 1; i < 4; i++)
#pragma unroll
    for (int j = 1; j < 4; j++) v_b[i] += 2.0 * qsq_b * gc(i, j) * v[j];
  qb[RHO] = rho_b;
  qb[UU] = uu_b;
  qb[U1] = v_b[1];
  qb[U2] = v_b[2];
  qb[U3] = v_b[3];
  qb[B1] = B_b[1];
  qb[B2] = B_b[2];
  qb[B3] = B_b[3];
  gamb = gam_b;
}
