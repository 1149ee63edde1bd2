// Hand-written adjoint (vector-Jacobian product) of one SSPRK2 step.
//
// The reverse sweep is written out stage by stage: the inversion is
// differentiated by the implicit-function theorem (lambda_U = (dU/dP)^-T
// lambda_P at the recovered prims; a zone whose inversion failed passes its
// hydro adjoint to the guess), the RK combination and flux divergence are
// transposed explicitly, Flux-CT is transposed through its edge EMFs, every
// face flux is transposed through its stencil, and ghost fills are transposed
// by gathering each ghost's adjoint back onto the zone it was copied from
// (with the polar sign flips).  The local derivatives of the per-point
// physics: a face flux with respect to its two states' prims by a reverse
// sweep through each state (face_vjp.hpp), chained with the reconstruction's
// derivatives with respect to each stencil slot (the WENO5 and MC gradients
// in closed form); the source and the conserved variables with respect to
// one zone's prims by a reverse sweep through the zone; the inversion's
// Jacobian by forward-mode dual numbers.  Every sum is a gather in a fixed
// order: the result is deterministic.
//
// Included inside the anonymous namespace of grmhd.hip.

template <int RECON>
struct Stencil {
  static constexpr int W = RECON == GRMHD_RECON_MC ? 4 : 6;  // zones per face
  static constexpr int H = W / 2;                            // zones left of the face
  static constexpr int NSLOT = NVAR * W;                     // stencil inputs of one face
};

#include "face_vjp.hpp"

// One face state in plain FP64: its flux along D, conserved variables and
// characteristic speeds.
template <int D>
__device__ __forceinline__ void state_real(const double q[NVAR], const PointMetric<double>& m, double gam,
                                           double Fx[NVAR], double U[NVAR], double& cp, double& cm) {
  Fluid<double> f;
  fluid_state(q, m, f);
  prim_to_flux(q, f, m, gam, D, Fx);
  prim_to_flux(q, f, m, gam, 0, U);
  char_speeds(q, f, m, gam, D, cp, cm);
}

// Adjoint of the Flux-CT EMFs on every padded edge position (zero outside
// the edge box [0, n]^3 and on polar edges), from the stage adjoint lambda_L
// of the field components (zero in ghost zones).  With the rebuilt fluxes
// Ft1(B2) = (E3 + E3_{j+1})/2 etc., lambda_Ft(face f) = (LL(f) - LL(f - e_d))/dx_d.
__global__ void __launch_bounds__(BLOCK) k_adj_emf(Dev g, const double* __restrict__ LL,
                                                   double* __restrict__ LE1, double* __restrict__ LE2,
                                                   double* __restrict__ LE3) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= g.nz) return;
  int i = (int)(t % g.s1) - NG;
  long r = t / g.s1;
  int j = (int)(r % g.s2) - NG, k = (int)(r / g.s2) - NG;
  if (i < 0 || j < 0 || k < 0 || i > g.n1 || j > g.n2 || k > g.n3) {
    LE1[t] = LE2[t] = LE3[t] = 0.0;
    return;
  }
  const long nz = g.nz, si = 1, sj = g.s1, sk = g.plane;
  auto lf = [&](int v, long f, long sd, double dx) { return (LL[v * nz + f] - LL[v * nz + f - sd]) / dx; };
  bool pole = (g.pole_lo && j == 0) || (g.pole_hi && j == g.n2);
  // E3 enters Ft1(B2) at faces (i,j),(i,j-1) with +1/2 and Ft2(B1) at (i,j),(i-1,j) with -1/2
  double e3 = 0.5 * (lf(B2, t, si, g.dx1) + lf(B2, t - sj, si, g.dx1)) -
              0.5 * (lf(B1, t, sj, g.dx2) + lf(B1, t - si, sj, g.dx2));
  // E2 enters Ft3(B1) at (i,k),(i-1,k) with +1/2 and Ft1(B3) at (i,k),(i,k-1) with -1/2
  double e2 = 0.5 * (lf(B1, t, sk, g.dx3) + lf(B1, t - si, sk, g.dx3)) -
              0.5 * (lf(B3, t, si, g.dx1) + lf(B3, t - sk, si, g.dx1));
  // E1 enters Ft2(B3) at (j,k),(j,k-1) with +1/2 and Ft3(B2) at (j,k),(j-1,k) with -1/2
  double e1 = 0.5 * (lf(B3, t, sj, g.dx2) + lf(B3, t - sk, sj, g.dx2)) -
              0.5 * (lf(B2, t, sk, g.dx3) + lf(B2, t - sj, sk, g.dx3));
  LE1[t] = pole ? 0.0 : e1;
  LE2[t] = e2;
  LE3[t] = pole ? 0.0 : e3;
}

// Per face of the forward flux box: the adjoint of the LLF flux (hydro slots
// from the divergence, field slots through the EMF averages), pushed through
// the face's local Jacobian onto its stencil: LS[(v*W + s) * nz + face], and
// the gamma part added to GF[face].
// Waves per SIMD the face adjoint is compiled for (2: 250-254 VGPRs, no
// spills; about 10 % faster than 1 wave).
#ifndef ADJ_FACE_WAVES
#define ADJ_FACE_WAVES 2
#endif
template <int D, int RECON>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(ADJ_FACE_WAVES, 8)))
k_adj_face(Dev g, Box box, const double* __restrict__ P,
                                                    const double* __restrict__ tab,
                                                    const double* __restrict__ LL,
                                                    const double* __restrict__ LE1,
                                                    const double* __restrict__ LE2,
                                                    const double* __restrict__ LE3,
                                                    double* __restrict__ LS, double* __restrict__ GF) {
  using St = Stencil<RECON>;
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (!box_index(box, t, i, j, k)) return;
  const long c = zid(g, i, j, k), nz = g.nz, si = 1, sj = g.s1, sk = g.plane;
  const long s = D == 1 ? si : (D == 2 ? sj : sk);
  const double dx = D == 1 ? g.dx1 : (D == 2 ? g.dx2 : g.dx3);
  double lam[NVAR];
#pragma unroll
  for (int v = 0; v < 5; v++) lam[v] = (LL[v * nz + c] - LL[v * nz + c - s]) / dx;
  const double q = 0.25;
  if (D == 1) {
    lam[B1] = 0.0;
    lam[B2] = q * (LE3[c] + LE3[c + sj]);
    lam[B3] = -q * (LE2[c] + LE2[c + sk]);
  } else if (D == 2) {
    lam[B1] = -q * (LE3[c] + LE3[c + si]);
    lam[B2] = 0.0;
    lam[B3] = q * (LE1[c] + LE1[c + sk]);
  } else {
    lam[B1] = q * (LE2[c] + LE2[c + si]);
    lam[B2] = -q * (LE1[c] + LE1[c + sj]);
    lam[B3] = 0.0;
  }
  bool zero = true;
#pragma unroll
  for (int v = 0; v < NVAR; v++) zero = zero && lam[v] == 0.0;
  if (zero || (D == 2 && ((g.pole_lo && j == 0) || (g.pole_hi && j == g.n2)))) {
    for (int sd = 0; sd < St::NSLOT; sd++) LS[sd * nz + c] = 0.0;
    return;
  }
  // chain rule through the face states: lambda . dF/d(stencil slot) =
  // sum over the two states of (lambda . dF/dq_state[v]) dq_state[v]/dslot;
  // the first factor by a reverse sweep through each state, the second from
  // the reconstruction's derivatives with respect to each slot
  PointMetric<double> m;
  load_metric<double>(tab, g.plane, pid(g, i, j), m);
  double qL[NVAR], qR[NVAR];
  recon_pair<RECON, double>(P, nz, c, s, g.weno_eps, qL, qR);
  const double gam = g.gam;
  // lambda . dF/dq of both states by one reverse sweep per state: the LLF
  // flux F = (FL + FR)/2 - cmax (UR - UL)/2 gives the adjoints lambda/2 of
  // FL and FR, +-cmax lambda/2 of UL and UR, and -lambda.(UR - UL)/2 of
  // cmax, which goes to the speed that attains it (chosen as the dual-number
  // fmax chain chooses: the later operand only when strictly larger)
  double FL[NVAR], UL[NVAR], cpl, cml, FR[NVAR], UR[NVAR], cpr, cmr;
  state_real<D>(qL, m, gam, FL, UL, cpl, cml);
  state_real<D>(qR, m, gam, FR, UR, cpr, cmr);
  const bool s1 = cpr > cpl, s2 = -cmr > -cml;
  const double m1 = s1 ? cpr : cpl, m2 = s2 ? -cmr : -cml;
  const bool s3 = m2 > m1;
  const double m3 = s3 ? m2 : m1;
  const bool pos = !(0.0 > m3);
  const double cmax = pos ? m3 : 0.0;
  double cb = 0.0;
#pragma unroll
  for (int v = 0; v < NVAR; v++) cb += lam[v] * (UR[v] - UL[v]);
  cb = pos ? -0.5 * cb : 0.0;
  const double cplb = !s3 && !s1 ? cb : 0.0, cprb = !s3 && s1 ? cb : 0.0;
  const double cmlb = s3 && !s2 ? -cb : 0.0, cmrb = s3 && s2 ? -cb : 0.0;
  double Fb[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) Fb[v] = 0.5 * lam[v];
  double gL[NVAR], gR[NVAR], gsum = 0.0;
  // one side at a time (a single copy of the sweep: shorter live ranges)
#pragma unroll 1
  for (int side = 0; side < 2; side++) {
    double qs[NVAR], Ub[NVAR], qb[NVAR], gamb;
#pragma unroll
    for (int v = 0; v < NVAR; v++) {
      qs[v] = side == 0 ? qL[v] : qR[v];
      Ub[v] = (side == 0 ? 0.5 : -0.5) * cmax * lam[v];
    }
    state_vjp<D>(qs, m, gam, Fb, Ub, side == 0 ? cplb : cprb, side == 0 ? cmlb : cmrb, qb, gamb);
    gsum += gamb;
#pragma unroll
    for (int v = 0; v < NVAR; v++) {
      gL[v] = side == 0 ? qb[v] : gL[v];
      gR[v] = side == 1 ? qb[v] : gR[v];
    }
  }
  GF[c] += gsum;
#pragma unroll 1
  for (int v = 0; v < NVAR; v++) {
    double qs[St::W];
#pragma unroll
    for (int z = 0; z < St::W; z++) qs[z] = P[v * nz + c + (z - St::H) * s];
    double dL[St::W], dR[St::W];
    if constexpr (RECON == GRMHD_RECON_WENO5) {
      // the left state is weno5(q0, .., q4), the right one weno5(q5, .., q1):
      // both gradients in closed form
      weno5_grad(qs[0], qs[1], qs[2], qs[3], qs[4], g.weno_eps, dL[0], dL[1], dL[2], dL[3], dL[4]);
      weno5_grad(qs[5], qs[4], qs[3], qs[2], qs[1], g.weno_eps, dR[5], dR[4], dR[3], dR[2], dR[1]);
      dL[5] = 0.0;
      dR[0] = 0.0;
    } else {
      // MC: the left state is mc_left(q0, q1, q2), the right one mc_right(q1, q2, q3)
      mc_left_grad(qs[0], qs[1], qs[2], dL[0], dL[1], dL[2]);
      mc_right_grad(qs[1], qs[2], qs[3], dR[1], dR[2], dR[3]);
      dL[3] = 0.0;
      dR[0] = 0.0;
    }
    double gl = 0.0, gr = 0.0;
#pragma unroll
    for (int u = 0; u < NVAR; u++) {   // compare and select: no register array indexed by v
      gl = u == v ? gL[u] : gl;
      gr = u == v ? gR[u] : gr;
    }
#pragma unroll
    for (int z = 0; z < St::W; z++) LS[(v * St::W + z) * nz + c] = gl * dL[z] + gr * dR[z];
  }
}

// Gather of the stencil adjoints onto every padded zone: zone z is slot s of
// the D-face f = z + (H - s) e_D.
template <int RECON>
__device__ __forceinline__ void gather_dir(const Dev& g, const Box& fb, const double* __restrict__ LS,
                                           int D, int i, int j, int k, double acc[NVAR]) {
  using St = Stencil<RECON>;
  for (int s = 0; s < St::W; s++) {
    int o = St::H - s;
    int fi = i + (D == 1 ? o : 0), fj = j + (D == 2 ? o : 0), fk = k + (D == 3 ? o : 0);
    if (fi < fb.lo1 || fi >= fb.lo1 + fb.n1 || fj < fb.lo2 || fj >= fb.lo2 + fb.n2 || fk < fb.lo3 ||
        fk >= fb.lo3 + fb.n3)
      continue;
    long f = zid(g, fi, fj, fk);
#pragma unroll
    for (int v = 0; v < NVAR; v++) acc[v] += LS[(v * St::W + s) * g.nz + f];
  }
}

template <int RECON>
__global__ void __launch_bounds__(BLOCK) k_adj_gather(Dev g, Box b1, Box b2, Box b3,
                                                      const double* __restrict__ LS1,
                                                      const double* __restrict__ LS2,
                                                      const double* __restrict__ LS3,
                                                      double* __restrict__ LPh) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= g.nz) return;
  int i = (int)(t % g.s1) - NG;
  long r = t / g.s1;
  int j = (int)(r % g.s2) - NG, k = (int)(r / g.s2) - NG;
  double acc[NVAR] = {0, 0, 0, 0, 0, 0, 0, 0};
  gather_dir<RECON>(g, b1, LS1, 1, i, j, k, acc);
  gather_dir<RECON>(g, b2, LS2, 2, i, j, k, acc);
  gather_dir<RECON>(g, b3, LS3, 3, i, j, k, acc);
#pragma unroll
  for (int v = 0; v < NVAR; v++) LPh[v * g.nz + t] = acc[v];
}


// Per interior zone: the ghost-fill transpose of the gathered stencil
// adjoint, plus the local terms: source^T lambda_L, (stage 1) U^T lambda_U0,
// and the guess adjoint of a failed inversion.  Gamma parts go to GZ.
template <bool STAGE1>
__global__ void __launch_bounds__(BLOCK) k_adj_zone(Dev g, Box box, const double* __restrict__ Pin,
                                                    const double* __restrict__ tabC,
                                                    const double* __restrict__ conn,
                                                    const double* __restrict__ LPh,
                                                    const double* __restrict__ LL,
                                                    const double* __restrict__ LU0,
                                                    const double* __restrict__ LG,
                                                    double* __restrict__ LP, double* __restrict__ GZ) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (!box_index(box, t, i, j, k)) return;
  const long c = zid(g, i, j, k), nz = g.nz;
  double acc[NVAR];
  int y1[7], y2[7], y3[7];
  bool f1[7], f2[7], f3[7];
  int n1 = bc_preimages(i, g.n1, g.bc[0], g.bc[1], y1, f1);
  int n2 = bc_preimages(j, g.n2, g.bc[2], g.bc[3], y2, f2);
  int n3 = bc_preimages(k, g.n3, g.bc[4], g.bc[5], y3, f3);
#pragma unroll
  for (int v = 0; v < NVAR; v++) acc[v] = 0.0;
  for (int a = 0; a < n1; a++)
    for (int b = 0; b < n2; b++)
      for (int e = 0; e < n3; e++) {
        long q = zid(g, y1[a], y2[b], y3[e]);
        bool flip = f1[a] ^ f2[b] ^ f3[e];
#pragma unroll
        for (int v = 0; v < NVAR; v++) {
          double x = LPh[v * nz + q];
          acc[v] += (flip && (v == U2 || v == B2)) ? -x : x;
        }
      }
  PointMetric<double> m;
  load_metric<double>(tabC, g.plane, pid(g, i, j), m);
  double cn[40];
  load_conn(conn, g.plane, pid(g, i, j), cn);
  double lL[NVAR], lU[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) {
    lL[v] = LL[v * nz + c];
    lU[v] = STAGE1 ? LU0[v * nz + c] : 0.0;
  }
  // the local terms by one reverse sweep: the source (adjoint lambda_L of
  // the energy and momentum rows) and, in stage 1, the conserved variables
  double p[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) p[v] = Pin[v * nz + c];
  const double Sb[4] = {lL[UU], lL[U1], lL[U2], lL[U3]};
  double qb[NVAR], gz;
  zone_vjp(p, m, g.gam, cn, Sb, STAGE1 ? lU : nullptr, qb, gz);
#pragma unroll
  for (int v = 0; v < NVAR; v++) acc[v] += qb[v];
#pragma unroll
  for (int v = 0; v < 5; v++) acc[v] += LG[v * nz + c];
#pragma unroll
  for (int v = 0; v < NVAR; v++) LP[v * nz + c] = acc[v];
  GZ[c] += gz;
}

// Transposed RK combination of one element, from lambda_U of a stage's
// conserved variables.  mode 0 (stage 2, U^{n+1} = V + (dt/2) L(P1)):
// lambda_V = lambda_U, lambda_L = (dt/2) lambda_U.  mode 1 (stage 1,
// U1 = U^n + dt L(P^n), V = (U^n + U1)/2, with lambda_V from stage 2):
// lambda_U1 = lambda_U + lambda_V/2, lambda_Un = lambda_V/2 + lambda_U1 (into
// LV), lambda_L = dt lambda_U1.
__device__ __forceinline__ void rk_transpose(int mode, double dt, double u, double& LV, double& LL) {
  if (mode == 0) {
    LV = u;
    LL = 0.5 * dt * u;
  } else {
    const double lu1 = u + 0.5 * LV;
    const double lu0 = 0.5 * LV + lu1;
    LV = lu0;
    LL = dt * lu1;
  }
}

// Implicit-function adjoint of the inversion at the recovered prims P:
// lambda_U = (dU/dP)^-T lambda_P, and -lambda_U . dU/dgamma into GZ.  A zone
// whose inversion failed kept its guess's hydro prims: lambda goes to the
// guess (LG) and only B^i = U_B^i / sqrt(-g) carries lambda to U.
// Ghost entries of LU and LG are zero.
__global__ void __launch_bounds__(BLOCK) k_adj_ift(Dev g, const double* __restrict__ P,
                                                   const unsigned char* __restrict__ flags,
                                                   const double* __restrict__ tabC,
                                                   const double* __restrict__ LP, int mode, double dt,
                                                   double* __restrict__ LV, double* __restrict__ LL,
                                                   double* __restrict__ LG, double* __restrict__ GZ) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= g.nz) return;
  const long nz = g.nz;
  // lambda_U of variable v, passed through the transposed RK combination
  // (rk_transpose) into the stage register's and the stage rate's adjoints
  auto LU = [&](int v, double u) { rk_transpose(mode, dt, u, LV[v * nz + t], LL[v * nz + t]); };
  int i = (int)(t % g.s1) - NG;
  long r = t / g.s1;
  int j = (int)(r % g.s2) - NG, k = (int)(r / g.s2) - NG;
  if (i < 0 || j < 0 || k < 0 || i >= g.n1 || j >= g.n2 || k >= g.n3) {
#pragma unroll
    for (int v = 0; v < NVAR; v++) LU(v, 0.0);
#pragma unroll
    for (int v = 0; v < 5; v++) LG[v * nz + t] = 0.0;
    return;
  }
  double lp[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) lp[v] = LP[v * nz + t];
  PointMetric<double> m;
  load_metric<double>(tabC, g.plane, pid(g, i, j), m);
  if (flags[t]) {
#pragma unroll
    for (int v = 0; v < 5; v++) {
      LG[v * nz + t] = lp[v];
      LU(v, 0.0);
    }
#pragma unroll
    for (int v = 5; v < NVAR; v++) LU(v, lp[v] / m.gdet);
    return;
  }
  // Rows of the hydro conserved variables of the Jacobian: Jh[a][b] =
  // dU_a / dP_b (a < 5), column NVAR dU_a / dgamma.  The field rows are
  // sqrt(-g) on the diagonal (U_B = sqrt(-g) B, independent of the rest).
  // One seed direction per pass; the column is stored by compare and select,
  // so nothing held in registers is indexed by the pass counter.
  double Jh[5][NVAR + 1];
  double pv[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) pv[v] = P[v * nz + t];
#pragma unroll 1
  for (int sd = 0; sd <= NVAR; sd++) {
    Dual p[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; v++) p[v] = Dual(pv[v], sd == v ? 1.0 : 0.0);
    Dual gam(g.gam, sd == NVAR ? 1.0 : 0.0);
    Fluid<Dual> f;
    fluid_state(p, m, f);
    Dual U[NVAR];
    prim_to_flux(p, f, m, gam, 0, U);
#pragma unroll
    for (int c = 0; c <= NVAR; c++)
      if (c == sd) {
#pragma unroll
        for (int a = 0; a < 5; a++) Jh[a][c] = U[a].d;
      }
  }
  // J^T x = lp with J = [[Jhh, Jhb], [0, sqrt(-g) I]]: first Jhh^T x_h = lp_h
  // (Gaussian elimination with partial pivoting, every index fixed at
  // compile time so the system stays in registers), then
  // x_B = (lp_B - Jhb^T x_h) / sqrt(-g).
  double A[5][5], x[NVAR];
#pragma unroll
  for (int a = 0; a < 5; a++) {
#pragma unroll
    for (int b = 0; b < 5; b++) A[a][b] = Jh[b][a];
    x[a] = lp[a];
  }
#pragma unroll
  for (int col = 0; col < 5; col++) {
    int piv = col;
    double best = fabs(A[col][col]);
#pragma unroll
    for (int rr = col + 1; rr < 5; rr++)
      if (fabs(A[rr][col]) > best) {
        best = fabs(A[rr][col]);
        piv = rr;
      }
#pragma unroll
    for (int rr = col + 1; rr < 5; rr++)
      if (rr == piv) {
#pragma unroll
        for (int b = col; b < 5; b++) {
          const double tmp = A[col][b];
          A[col][b] = A[rr][b];
          A[rr][b] = tmp;
        }
        const double tmp = x[col];
        x[col] = x[rr];
        x[rr] = tmp;
      }
#pragma unroll
    for (int rr = col + 1; rr < 5; rr++) {
      const double fct = A[rr][col] / A[col][col];
#pragma unroll
      for (int b = col; b < 5; b++) A[rr][b] -= fct * A[col][b];
      x[rr] -= fct * x[col];
    }
  }
#pragma unroll
  for (int rr = 4; rr >= 0; rr--) {
    double sum = x[rr];
#pragma unroll
    for (int b = rr + 1; b < 5; b++) sum -= A[rr][b] * x[b];
    x[rr] = sum / A[rr][rr];
  }
#pragma unroll
  for (int k = 0; k < 3; k++) {
    double sum = lp[B1 + k];
#pragma unroll
    for (int a = 0; a < 5; a++) sum -= Jh[a][B1 + k] * x[a];
    x[B1 + k] = sum / m.gdet;
  }
  double gz = 0.0;
#pragma unroll
  for (int v = 0; v < NVAR; v++) LU(v, x[v]);
#pragma unroll
  for (int a = 0; a < 5; a++) gz -= x[a] * Jh[a][NVAR];
#pragma unroll
  for (int v = 0; v < 5; v++) LG[v * nz + t] = 0.0;
  GZ[t] += gz;
}

// Sum of the gamma parts: per-block partial sums of GZ + GF1 + GF2 + GF3.
__global__ void __launch_bounds__(BLOCK) k_adj_gsum(long nz, const double* __restrict__ GZ,
                                                    const double* __restrict__ GF1,
                                                    const double* __restrict__ GF2,
                                                    const double* __restrict__ GF3, double* pmax,
                                                    double* psum) {
  double s = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < nz; t += stride)
    s += ((GZ[t] + GF1[t]) + GF2[t]) + GF3[t];
  double mx = 0.0;
  block_reduce(mx, s);
  if (threadIdx.x == 0) {
    pmax[blockIdx.x] = 0.0;
    psum[blockIdx.x] = s;
  }
}
