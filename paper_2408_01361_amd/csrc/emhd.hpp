// Extended GRMHD (Implicit Solver and Extended Theory section, EGRMHD
// subsection, after Chandra et al. 2015 in the rescaled variables of Foucart
// et al. 2016).  Two zone-centred variables join the eight of ideal GRMHD:
//   X0 = q  (tau_R / (chi rho Theta^2))^(1/2),   the rescaled heat flux,
//   X1 = dP (tau_R / (nu rho Theta))^(1/2),      the rescaled anisotropy,
// Theta = (gam - 1) u / rho.  The stress-energy tensor gains
//   q bh^mu u_nu + q bh_nu u^mu - dP (bh^mu bh_nu - h^mu_nu / 3),
// bh = b / |b|, h^mu_nu = delta^mu_nu + u^mu u_nu (nothing where b^2 = 0),
// and each X obeys
//   d_mu(sqrt(-g) X u^mu) = sqrt(-g) [-(X - X_target) / tau_R + (X / 2) div u],
// with the targets of the Chandra et al. closure
//   q_target  = -rho chi bh^mu (d_mu Theta + Theta a_mu),  a_mu = u^nu nabla_nu u_mu,
//   dP_target = 3 rho nu (bh^mu bh^nu nabla_mu u_nu - div u / 3),
// rescaled like the variables and taken from centred spatial differences of
// the stage's explicit state (time derivatives left out).  div u =
// d_t u^t + d_i(sqrt(-g) u^i) / sqrt(-g): the spatial part explicit, the
// time part (u^t - u^t(step start)) / h implicit like the relaxation and the
// X multiplying div u.
//
// A predictor-corrector stage (h = dt/2, then h = dt from the step's state
// again with the predicted state's explicit rates) runs six launches: the
// ghost fill of X, the face fluxes of all ten variables (ideal LLF speeds),
// the Flux-CT EMFs (the ideal kernel), the targets pass (X targets and the
// spatial div u), the update pass that forms each zone's explicit
// right-hand sides U^n + h L (ten slots), and the implicit pass: per zone
// the implicit solver's Newton on the five hydro prims, with the two X
// equations, linear in X for a given hydro state, solved for X inside
// every residual evaluation.
//
// FP64 throughout, every operation rounded on its own in the order written.
//
// Included inside the anonymous namespace of grmhd.hip.

constexpr int NXV = 2;  // extra variables per zone

// Physical heat flux q and anisotropy dP of the rescaled variables x.
__device__ __forceinline__ void emhd_unscale(const Dev& g, const double p[NVAR], const double x[NXV], double& q,
                                             double& dP) {
#pragma clang fp contract(off)
  const double theta = (g.gam - 1.0) * p[UU] / p[RHO];
  q = x[0] * theta * sqrt(g.chi * p[RHO] / g.tau);
  dP = x[1] * sqrt(g.nu * p[RHO] * theta / g.tau);
}

// Row mu of the extended mixed stress-energy tensor.
__device__ __forceinline__ void tmunu_row_emhd(const double p[NVAR], const Fluid<double>& f, double gam, double q,
                                               double dP, int mu, double T[4]) {
#pragma clang fp contract(off)
  tmunu_row(p, f, gam, mu, T);
  if (!(f.bsq > 0.0) || (q == 0.0 && dP == 0.0)) return;
  const double sb = sqrt(f.bsq);
  const double bm = f.bcon[mu] / sb;
#pragma unroll
  for (int nu = 0; nu < 4; nu++) {
    const double bn = f.bcov[nu] / sb;
    const double h = (mu == nu ? 1.0 : 0.0) + f.ucon[mu] * f.ucov[nu];
    T[nu] = ((T[nu] + q * bm * f.ucov[nu]) + q * bn * f.ucon[mu]) - dP * (bm * bn - h / 3.0);
  }
}

// Conserved variables (d = 0) or fluxes along x^d of the ten variables:
// sqrt(-g) (rho u^d, T^d_t + rho u^d, T^d_i, b^k u^d - b^d u^k, X u^d).
__device__ __forceinline__ void prim_to_flux_emhd(const Dev& g, const double p[NVAR], const double x[NXV],
                                                  const Fluid<double>& f, const PointMetric<double>& m, int d,
                                                  double F[NVAR + NXV]) {
#pragma clang fp contract(off)
  double q, dP;
  emhd_unscale(g, p, x, q, dP);
  double T[4];
  tmunu_row_emhd(p, f, g.gam, q, dP, d, T);
  F[RHO] = (m.gdet * p[RHO]) * f.ucon[d];
  F[UU] = m.gdet * (T[0] + p[RHO] * f.ucon[d]);
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
#pragma unroll
  for (int n = 0; n < NXV; n++) F[NVAR + n] = (m.gdet * x[n]) * f.ucon[d];
}

// Ghost zones of the extra variables: the maps of k_bc, no sign flips (both
// are scalars under the polar reflection).
__global__ void __launch_bounds__(BLOCK) k_bc_extra(Dev g, double* X) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= ghost_count(g)) return;
  int i, j, k;
  ghost_index(g, t, i, j, k);
  bool f1 = false, f2 = false, f3 = false;
  const int si = bc_map(i, g.n1, g.bc[0], g.bc[1], f1);
  const int sj = bc_map(j, g.n2, g.bc[2], g.bc[3], f2);
  const int sk = bc_map(k, g.n3, g.bc[4], g.bc[5], f3);
  if (si == i && sj == j && sk == k) return;  // frozen
  const long src = zid(g, si, sj, sk), dst = zid(g, i, j, k);
#pragma unroll
  for (int n = 0; n < NXV; n++) X[n * g.nz + dst] = X[n * g.nz + src];
}

// Face states of one variable at stride s around padded index c (the face
// between c - s and c), as recon_pair forms them.
template <int RECON>
__device__ __forceinline__ void recon_one(const double* __restrict__ q, long s, double eps, double& l,
                                          double& r) {
  if (RECON == GRMHD_RECON_MC) {
    const double m2 = q[-2 * s], m1 = q[-s], p0 = q[0], p1 = q[s];
    l = mc_left(m2, m1, p0);
    r = mc_right(m1, p0, p1);
  } else {
    const double m3 = q[-3 * s], m2 = q[-2 * s], m1 = q[-s], p0 = q[0], p1 = q[s], p2 = q[2 * s];
    l = weno5(m3, m2, m1, p0, p1, eps);
    r = weno5(p2, p1, p0, m1, m2, eps);
  }
}

// LLF flux of the ten variables through the lower D-face of zone (i, j, k),
// the face metric from tab; pole faces get zero.  The normal field's flux is
// not stored (Flux-CT reads only the tangential ones).
template <int D, int RECON>
__device__ __forceinline__ void emhd_face(const Dev& g, const double* __restrict__ P,
                                          const double* __restrict__ X, const double* __restrict__ tab,
                                          double* __restrict__ F, double* __restrict__ FX, int i, int j,
                                          int k) {
#pragma clang fp contract(off)
  const long c = zid(g, i, j, k);
  if (pole_face<D>(g, j)) {
#pragma unroll
    for (int v = 0; v < NVAR; v++) F[v * g.nz + c] = 0.0;
#pragma unroll
    for (int n = 0; n < NXV; n++) FX[n * g.nz + c] = 0.0;
    return;
  }
  const long s = D == 1 ? 1 : (D == 2 ? (long)g.s1 : g.plane);
  double qL[NVAR], qR[NVAR], xL[NXV], xR[NXV];
  recon_pair<RECON, double>(P, g.nz, c, s, g.weno_eps, qL, qR);
#pragma unroll
  for (int n = 0; n < NXV; n++) recon_one<RECON>(X + n * g.nz + c, s, g.weno_eps, xL[n], xR[n]);
  PointMetric<double> m;
  load_metric<double>(tab, g.plane, pid(g, i, j), m);
  Fluid<double> fl, fr;
  fluid_state(qL, m, fl);
  fluid_state(qR, m, fr);
  double FL[NVAR + NXV], FR[NVAR + NXV], UL[NVAR + NXV], UR[NVAR + NXV];
  prim_to_flux_emhd(g, qL, xL, fl, m, D, FL);
  prim_to_flux_emhd(g, qR, xR, fr, m, D, FR);
  prim_to_flux_emhd(g, qL, xL, fl, m, 0, UL);
  prim_to_flux_emhd(g, qR, xR, fr, m, 0, UR);
  double cpl, cml, cpr, cmr;
  char_speeds(qL, fl, m, g.gam, D, cpl, cml);
  char_speeds(qR, fr, m, g.gam, D, cpr, cmr);
  double cmax = 0.0;
  if (cpl > cmax) cmax = cpl;
  if (cpr > cmax) cmax = cpr;
  if (-cml > cmax) cmax = -cml;
  if (-cmr > cmax) cmax = -cmr;
#pragma unroll
  for (int v = 0; v < NVAR; v++)
    if (v != B1 + D - 1) F[v * g.nz + c] = 0.5 * (FL[v] + FR[v]) - 0.5 * cmax * (UR[v] - UL[v]);
#pragma unroll
  for (int n = 0; n < NXV; n++)
    FX[n * g.nz + c] = 0.5 * (FL[NVAR + n] + FR[NVAR + n]) - 0.5 * cmax * (UR[NVAR + n] - UL[NVAR + n]);
}

// All three face directions in one launch, partitioned as k_flux_all.
template <int RECON>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_flux_emhd(Dev g, Sched b1, Sched b2, Sched b3, unsigned nb1, unsigned nb2, unsigned nb3,
            const double* __restrict__ P, const double* __restrict__ X, const double* __restrict__ tabF1,
            const double* __restrict__ tabF2, const double* __restrict__ tabC, double* __restrict__ F1,
            double* __restrict__ F2, double* __restrict__ F3, double* __restrict__ FX1,
            double* __restrict__ FX2, double* __restrict__ FX3) {
  const unsigned b = blockIdx.x;
  int i, j, k;
  if (b < nb1) {
    if (sched_index(b1, b, nb1, i, j, k)) emhd_face<1, RECON>(g, P, X, tabF1, F1, FX1, i, j, k);
  } else if (b < nb1 + nb2) {
    if (sched_index(b2, b - nb1, nb2, i, j, k)) emhd_face<2, RECON>(g, P, X, tabF2, F2, FX2, i, j, k);
  } else {
    if (sched_index(b3, b - nb1 - nb2, nb3, i, j, k)) emhd_face<3, RECON>(g, P, X, tabC, F3, FX3, i, j, k);
  }
}

// Targets X_target and the spatial part of div u at zone (i, j, k) from the
// ghost-filled prims P; p, f, m: the zone's prims, fluid state and metric.
// Axes with one zone contribute no differences.
__device__ __forceinline__ void emhd_targets(const Dev& g, const double* __restrict__ P,
                                             const double* __restrict__ tabC, const double* __restrict__ conn,
                                             int i, int j, int k, const double p[NVAR], const Fluid<double>& f,
                                             const PointMetric<double>& m, double Xt[NXV], double& divu_sp) {
#pragma clang fp contract(off)
  const long c = zid(g, i, j, k), q2 = pid(g, i, j);
  const double gam = g.gam;
  const double th0 = (gam - 1.0) * p[UU] / p[RHO];
  // d_a Theta, d_a u_nu and d_a (sqrt(-g) u^a)
  double dth[3], du[3][4], dgu[3];
  const int n[3] = {g.n1, g.n2, g.n3};
  const double dx[3] = {g.dx1, g.dx2, g.dx3};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    dth[a] = dgu[a] = 0.0;
#pragma unroll
    for (int nu = 0; nu < 4; nu++) du[a][nu] = 0.0;
    if (n[a] == 1) continue;
    const long s = a == 0 ? 1 : (a == 1 ? (long)g.s1 : g.plane);
    const long qs = a == 0 ? 1 : (a == 1 ? (long)g.s1 : 0);
    double pp[NVAR], pm[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; v++) {
      pp[v] = P[v * g.nz + c + s];
      pm[v] = P[v * g.nz + c - s];
    }
    PointMetric<double> mp, mm;
    load_metric<double>(tabC, g.plane, q2 + qs, mp);
    load_metric<double>(tabC, g.plane, q2 - qs, mm);
    Fluid<double> sp, sm;
    fluid_state(pp, mp, sp);
    fluid_state(pm, mm, sm);
    const double thp = (gam - 1.0) * pp[UU] / pp[RHO];
    const double thm = (gam - 1.0) * pm[UU] / pm[RHO];
    const double h2 = 2.0 * dx[a];
    dth[a] = (thp - thm) / h2;
#pragma unroll
    for (int nu = 0; nu < 4; nu++) du[a][nu] = (sp.ucov[nu] - sm.ucov[nu]) / h2;
    dgu[a] = (mp.gdet * sp.ucon[a + 1] - mm.gdet * sm.ucon[a + 1]) / h2;
  }
  divu_sp = ((dgu[0] + dgu[1]) + dgu[2]) / m.gdet;
  Xt[0] = Xt[1] = 0.0;
  if (!(f.bsq > 0.0)) return;
  auto cn = [&](int l, int mu, int nu) { return conn[(l * 10 + sidx(mu, nu)) * g.plane + q2]; };
  double bh[4];
#pragma unroll
  for (int mu = 0; mu < 4; mu++) bh[mu] = f.bcon[mu] / sqrt(f.bsq);
  // a_nu = u^i d_i u_nu - Gamma^l_{m nu} u^m u_l
  double acc[4];
#pragma unroll
  for (int nu = 0; nu < 4; nu++) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) s += f.ucon[a + 1] * du[a][nu];
#pragma unroll
    for (int l = 0; l < 4; l++)
#pragma unroll
      for (int mu = 0; mu < 4; mu++) s -= cn(l, mu, nu) * f.ucon[mu] * f.ucov[l];
    acc[nu] = s;
  }
  double gq = 0.0;  // bh^mu (d_mu Theta + Theta a_mu)
#pragma unroll
  for (int a = 0; a < 3; a++) gq += bh[a + 1] * dth[a];
#pragma unroll
  for (int nu = 0; nu < 4; nu++) gq += th0 * bh[nu] * acc[nu];
  double bbu = 0.0;  // bh^mu bh^nu nabla_mu u_nu
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int nu = 0; nu < 4; nu++) bbu += bh[a + 1] * bh[nu] * du[a][nu];
#pragma unroll
  for (int mu = 0; mu < 4; mu++)
#pragma unroll
    for (int nu = 0; nu < 4; nu++)
#pragma unroll
      for (int l = 0; l < 4; l++) bbu -= bh[mu] * bh[nu] * cn(l, mu, nu) * f.ucov[l];
  const double rho = p[RHO];
  if (g.chi > 0.0) Xt[0] = -gq * sqrt(g.chi * rho * g.tau) / th0;
  if (g.nu > 0.0) Xt[1] = 3.0 * (bbu - divu_sp / 3.0) * sqrt(g.nu * rho * g.tau / th0);
}

// Targets pass of a stage: X_target of every interior zone to xt (the
// update pass reads them there and overwrites them with the X right-hand
// sides, zone by zone) and the spatial div u to divu.
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_targets_emhd(Dev g, Sched box, const double* __restrict__ Pin, const double* __restrict__ tabC,
               const double* __restrict__ conn, double* __restrict__ xt, double* __restrict__ divu) {
  int i, j, k;
  if (!sched_index(box, blockIdx.x, gridDim.x, i, j, k)) return;
  const long c = zid(g, i, j, k);
  double p[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) p[v] = Pin[v * g.nz + c];
  PointMetric<double> m;
  load_metric<double>(tabC, g.plane, pid(g, i, j), m);
  Fluid<double> f;
  fluid_state(p, m, f);
  double Xt[NXV], dsp;
  emhd_targets(g, Pin, tabC, conn, i, j, k, p, f, m, Xt, dsp);
#pragma unroll
  for (int n = 0; n < NXV; n++) xt[n * g.nz + c] = Xt[n];
  divu[c] = dsp;
}

// Update pass of a stage: per interior zone the explicit right-hand sides
// of the ten variables, U^n + h (-flux divergence + geometric source) for
// the eight ideal slots (the field from the edge EMFs as in update_zone)
// and U^n_X + h (-flux divergence + sqrt(-g) X_target / tau_R) for X (the
// targets as the targets pass left them in xrhs), to ustar and xrhs.
// STAGE 1 (h = dt/2) also keeps U^n of the stage input in V, VX and its u^t
// in utn; STAGE 2 (h = dt) reads them.  dt from dt_dev when given.
template <int STAGE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_update_emhd(Dev g, Sched box, const double* __restrict__ Pin, const double* __restrict__ Xin,
              double* __restrict__ V, double* __restrict__ VX, double* __restrict__ utn,
              const double* __restrict__ F1, const double* __restrict__ F2, const double* __restrict__ F3,
              const double* __restrict__ FX1, const double* __restrict__ FX2, const double* __restrict__ FX3,
              const double* __restrict__ E1, const double* __restrict__ E2, const double* __restrict__ E3,
              const double* __restrict__ tabC, const double* __restrict__ conn, double dt,
              const double* __restrict__ dt_dev, double* __restrict__ ustar, double* __restrict__ xrhs) {
#pragma clang fp contract(off)
  int i, j, k;
  if (!sched_index(box, blockIdx.x, gridDim.x, i, j, k)) return;
  if (dt_dev) dt = *dt_dev;
  const long c = zid(g, i, j, k), nz = g.nz, si = 1, sj = g.s1, sk = g.plane;
  const long q2 = pid(g, i, j);
  double p[NVAR], x[NXV];
#pragma unroll
  for (int v = 0; v < NVAR; v++) p[v] = Pin[v * nz + c];
#pragma unroll
  for (int n = 0; n < NXV; n++) x[n] = Xin[n * nz + c];
  PointMetric<double> m;
  load_metric<double>(tabC, g.plane, q2, m);
  Fluid<double> f;
  fluid_state(p, m, f);
  double qh, dPh;
  emhd_unscale(g, p, x, qh, dPh);

  double L[NVAR];
  {
    // sqrt(-g) T^k_l Gamma^l_{nu k} with the extended T, sums over k, then l
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      double Tk[4];
      tmunu_row_emhd(p, f, g.gam, qh, dPh, kk, Tk);
#pragma unroll
      for (int nu = 0; nu < 4; nu++)
#pragma unroll
        for (int l = 0; l < 4; l++) s[nu] += Tk[l] * conn[(l * 10 + sidx(nu, kk)) * g.plane + q2];
    }
#pragma unroll
    for (int v = 0; v < 5; v++) {
      const double d1 = (F1[v * nz + c + si] - F1[v * nz + c]) / g.dx1;
      const double d2 = (F2[v * nz + c + sj] - F2[v * nz + c]) / g.dx2;
      const double d3 = (F3[v * nz + c + sk] - F3[v * nz + c]) / g.dx3;
      L[v] = -((d1 + d2) + d3) + (v == RHO ? 0.0 : m.gdet * s[v - 1]);
    }
    ct_field_rate(g, E1, E2, E3, c, L);
  }
  double LX[NXV];
#pragma unroll
  for (int n = 0; n < NXV; n++) {
    const double d1 = (FX1[n * nz + c + si] - FX1[n * nz + c]) / g.dx1;
    const double d2 = (FX2[n * nz + c + sj] - FX2[n * nz + c]) / g.dx2;
    const double d3 = (FX3[n * nz + c + sk] - FX3[n * nz + c]) / g.dx3;
    LX[n] = -((d1 + d2) + d3) + m.gdet * xrhs[n * nz + c] / g.tau;
  }
  double U0[NVAR + NXV];
  if (STAGE == 1) {
    prim_to_flux_emhd(g, p, x, f, m, 0, U0);
#pragma unroll
    for (int v = 0; v < NVAR; v++) V[v * nz + c] = U0[v];
#pragma unroll
    for (int n = 0; n < NXV; n++) VX[n * nz + c] = U0[NVAR + n];
    utn[c] = f.ucon[0];
  } else {
#pragma unroll
    for (int v = 0; v < NVAR; v++) U0[v] = V[v * nz + c];
#pragma unroll
    for (int n = 0; n < NXV; n++) U0[NVAR + n] = VX[n * nz + c];
  }
  const double h = STAGE == 1 ? 0.5 * dt : dt;
#pragma unroll
  for (int v = 0; v < NVAR; v++) ustar[v * nz + c] = U0[v] + h * L[v];
#pragma unroll
  for (int n = 0; n < NXV; n++) xrhs[n * nz + c] = U0[NVAR + n] + h * LX[n];
}

// Implicit pass of a stage: per interior zone, the hydro prims and X whose
// ten conserved variables equal the right-hand sides plus h times the
// implicit X sources.  Given the hydro state the X equations read
//   sqrt(-g) X (u^t + h / tau_R - (h / 2) div u) = xrhs,
//   div u = divu + (u^t - u^t_n) / h,
// solved for X inside every residual; the Newton runs on the five hydro
// prims from the stage input (the guess), the field is xrhs's B /
// sqrt(-g).  On failure the zone keeps the guess's hydro prims and X (the
// field still updated) and is counted.  With RATE the CFL-rate partials of
// the new prims (ideal signal speeds), over the update's schedule.
template <int STAGE, bool RATE>
__global__ void __launch_bounds__(BLOCK)
k_implicit_emhd(Dev g, Sched box, const double* __restrict__ Pin, const double* __restrict__ Xin,
                const double* __restrict__ ustar, const double* __restrict__ xrhs,
                const double* __restrict__ divu, const double* __restrict__ utn, double* __restrict__ Pout,
                double* __restrict__ Xout, const double* __restrict__ tabC, double dt,
                const double* __restrict__ dt_dev, unsigned long long* fails,
                double* __restrict__ rate_partial) {
#pragma clang fp contract(off)
  __shared__ double jac[25 * BLOCK];
  int i, j, k;
  const bool in = sched_index(box, blockIdx.x, gridDim.x, i, j, k);
  if (dt_dev) dt = *dt_dev;
  double r = 0.0;
  if (in) {
    const long c = zid(g, i, j, k), nz = g.nz;
    double Us[NVAR], Ux[NXV], gs[NVAR], xg[NXV];
#pragma unroll
    for (int v = 0; v < NVAR; v++) {
      Us[v] = ustar[v * nz + c];
      gs[v] = Pin[v * nz + c];
    }
#pragma unroll
    for (int n = 0; n < NXV; n++) {
      Ux[n] = xrhs[n * nz + c];
      xg[n] = Xin[n * nz + c];
    }
    const double dsp = divu[c], ut_n = utn[c];
    const double h = STAGE == 1 ? 0.5 * dt : dt;
    PointMetric<double> m;
    load_metric<double>(tabC, g.plane, pid(g, i, j), m);
    const double gd = m.gdet;
    double out[NVAR], xo[NXV];
    out[B1] = Us[B1] / gd;
    out[B2] = Us[B2] / gd;
    out[B3] = Us[B3] / gd;
    const double B[3] = {out[B1], out[B2], out[B3]};
    // X of a hydro state with fluid state fz
    auto xsolve = [&](const Fluid<double>& fz, double Xz[NXV]) {
      const double ut = fz.ucon[0];
      const double du = dsp + (ut - ut_n) / h;
      const double coef = gd * ut + h * gd / g.tau - 0.5 * h * gd * du;
#pragma unroll
      for (int n = 0; n < NXV; n++) Xz[n] = Ux[n] / coef;
    };
    double scale = 0.0;
#pragma unroll
    for (int kk = 0; kk < 5; kk++)
      if (fabs(Us[kk]) > scale) scale = fabs(Us[kk]);
    bool ok = scale > 0.0 && isfinite(scale);
    double xs[5];
    if (ok) {
      auto res = [&](const double xx[5], double R[5]) {
        const double Pz[NVAR] = {xx[0], xx[1], xx[2], xx[3], xx[4], B[0], B[1], B[2]};
        Fluid<double> fz;
        fluid_state(Pz, m, fz);
        double Xz[NXV];
        xsolve(fz, Xz);
        double q, dP;
        emhd_unscale(g, Pz, Xz, q, dP);
        double T[4];
        tmunu_row_emhd(Pz, fz, g.gam, q, dP, 0, T);
        double U[5];
        U[RHO] = (gd * Pz[RHO]) * fz.ucon[0];
        U[UU] = gd * (T[0] + Pz[RHO] * fz.ucon[0]);
        U[U1] = gd * T[1];
        U[U2] = gd * T[2];
        U[U3] = gd * T[3];
#pragma unroll
        for (int kk = 0; kk < 5; kk++) R[kk] = (U[kk] - Us[kk]) / scale;
      };
      ok = newton_hydro(g, gs, res, xs, jac + threadIdx.x);
    }
    if (ok) {
      const double Pn[NVAR] = {xs[0], xs[1], xs[2], xs[3], xs[4], B[0], B[1], B[2]};
      Fluid<double> fz;
      fluid_state(Pn, m, fz);
      xsolve(fz, xo);
#pragma unroll
      for (int n = 0; n < NXV; n++)
        if (!isfinite(xo[n])) ok = false;
    }
    if (ok) {
#pragma unroll
      for (int v = 0; v < 5; v++) out[v] = xs[v];
    } else {
#pragma unroll
      for (int v = 0; v < 5; v++) out[v] = gs[v];
#pragma unroll
      for (int n = 0; n < NXV; n++) xo[n] = xg[n];
      atomicAdd(&fails[C_FAILS], 1ull);
    }
#pragma unroll
    for (int v = 0; v < NVAR; v++) Pout[v * nz + c] = out[v];
#pragma unroll
    for (int n = 0; n < NXV; n++) Xout[n * nz + c] = xo[n];
    if (RATE) r = zone_rate(g, out, m);
  }
  if (RATE) {
    double sm = 0.0;
    block_reduce(r, sm);
    if (threadIdx.x == 0) rate_partial[blockIdx.x] = r;
  }
}
