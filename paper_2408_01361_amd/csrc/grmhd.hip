// HIP kernels (gfx950) and the C ABI of the HARM ideal-GRMHD step.
//
// Per stage the step runs, on one stream:
//   bc      ghost zones from the stage's prims (index remap per axis)
//   flux    per face, for the x1, x2 and x3 faces in one launch: reconstruct
//           8 prims left/right, evaluate the face state, flux, conserved
//           variables and characteristic speeds for both sides, and form the
//           local Lax-Friedrichs flux (the paper keeps speeds, P->U and the
//           Riemann solve in one kernel, Solvers section)
//   emf     Flux-CT edge EMFs from the transverse B fluxes
//   update  per zone: flux divergence (B fluxes rebuilt from edge EMFs),
//           geometric source, SSPRK2 combination and the 1D_W inversion;
//           stage 2 also reduces the next step's CFL rate per workgroup
// with every intermediate resident in the caller's HBM workspace, and a
// single-workgroup pass over the CFL partials before the step when its dt
// is taken on the device.  Layouts are variable-major and x1-fastest, so
// each wavefront's loads and stores of one variable are contiguous.
//
// Options selected per context add passes to a stage: the Kastaun recovery
// replaces 1D_W inside the update; the implicit solver's recovery runs as a
// pass of its own after an update that stores U*; floors run after each
// update pass; the first-order flux correction repeats the EMF and update
// passes after a donor-cell fix of the marked zones' faces (launches that
// exit at once when nothing was marked); face-centred CT fills ghost faces,
// reads the face field in the flux pass, forms edge EMFs (averaged, or
// upwinded from zone-centre EMFs) and advances the faces before the update.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <mutex>
#include <vector>
#include <new>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/grmhd.h"
#include "geometry.hpp"
#include "physics.hpp"

using namespace grmhd;

namespace {

constexpr int NG = 3;
constexpr int BLOCK = 256;
constexpr int MAX_PARTIALS = 65536;

// Waves per SIMD the update kernel is compiled for (its register budget):
// without and with the CFL-rate evaluation of the new state.
#ifndef UPDATE_WAVES
#define UPDATE_WAVES 3
#endif
#ifndef UPDATE_WAVES_RATE
#define UPDATE_WAVES_RATE 3
#endif

// Everything a kernel needs to know about the grid, passed by value.
struct Dev {
  int n1, n2, n3;
  int s1, s2, s3;     // padded extents
  long nz;            // padded zones per variable
  long plane;         // s1 * s2
  double dx1, dx2, dx3;
  double idx1, idx2, idx3;  // 1 / dx_d (the update's differences multiply by them)
  double x1min, x2min;
  int bc[6];
  int pole_lo, pole_hi;
  double gam, weno_eps, tol;
  int maxit;
  int inverter;       // GRMHD_INV_*
  double vmax2;       // 1 - 1/W_max^2, the Kastaun recovery's speed cap
  int ct;             // GRMHD_CT_*: Flux-CT, or face-centred CT (averaged / upwinded EMFs)
  int floors;         // floors and ceilings after every inversion of a stage
  double rho_min_geom, u_min_geom, bsq_over_rho_max, bsq_over_u_max, u_over_rho_max, gamma_max;
  double tau, chi, nu;  // Extended GRMHD closure constants
  SpaceTime st;
};

__device__ __forceinline__ long zid(const Dev& g, int i, int j, int k) {
  return ((long)(k + NG) * g.s2 + (j + NG)) * g.s1 + (i + NG);
}
__device__ __forceinline__ long pid(const Dev& g, int i, int j) {
  return (long)(j + NG) * g.s1 + (i + NG);
}

// Box of (i, j, k), inclusive bounds, enumerated x1-fastest by a 1-D grid.
struct Box {
  int lo1, lo2, lo3, n1, n2, n3;
  __host__ __device__ long count() const { return (long)n1 * n2 * n3; }
};
__device__ __forceinline__ bool box_index(const Box& b, long t, int& i, int& j, int& k) {
  if (t >= (long)b.n1 * b.n2 * b.n3) return false;
  int n12 = b.n1 * b.n2;
  int kk = (int)(t / n12);
  int r = (int)(t - (long)kk * n12);
  int jj = r / b.n1;
  i = b.lo1 + (r - jj * b.n1);
  j = b.lo2 + jj;
  k = b.lo3 + kk;
  return true;
}

inline Box make_box(int lo1, int hi1, int lo2, int hi2, int lo3, int hi3) {
  return Box{lo1, lo2, lo3, hi1 - lo1 + 1, hi2 - lo2 + 1, hi3 - lo3 + 1};
}

inline unsigned blocks_for(long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

// Scheduled enumeration of a box for the heavy kernels.  A workgroup covers
// BLOCK consecutive (x1, x2) positions of one x3 plane.  Workgroups are
// dispatched round-robin over the 8 XCDs, so workgroup b is renumbered to
// give each XCD one contiguous range of work; within it kg consecutive x3
// planes of the same (x1, x2) chunk follow each other, so that chunk's 2-D
// geometry and the x3 stencil stay in that XCD's L2.  Any kg >= 1 covers the
// box exactly once.
struct Sched {
  Box b;
  int kg;       // x3 planes per chunk run
  int nchunk;   // workgroups per plane
  int kgroups;  // ceil(n3 / kg)
};
inline Sched make_sched(const Box& b, int kg) {
  if (kg < 1) kg = 1;
  if (kg > b.n3) kg = b.n3;
  long nij = (long)b.n1 * b.n2;
  return Sched{b, kg, (int)((nij + BLOCK - 1) / BLOCK), (b.n3 + kg - 1) / kg};
}
inline unsigned blocks_for(const Sched& s) { return (unsigned)((long)s.nchunk * s.kgroups * s.kg); }

// Logical workgroup index of dispatched workgroup b of nb: workgroups go to
// the 8 XCDs round-robin, so this gives each XCD one contiguous range.
__device__ __forceinline__ unsigned xcd_order(unsigned b, unsigned nb) {
  const unsigned x = b & 7u, slot = b >> 3;
  const unsigned q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + slot;
}

// bid / nb: this workgroup's index and the workgroup count of the launch (or
// of its part that covers this box, when the part starts at a multiple of 8).
__device__ __forceinline__ bool sched_index(const Sched& s, unsigned bid, unsigned nb, int& i, int& j,
                                            int& k) {
  const unsigned w = xcd_order(bid, nb);
  const int kin = (int)(w % (unsigned)s.kg);
  const unsigned rest = w / (unsigned)s.kg;
  const int chunk = (int)(rest % (unsigned)s.nchunk);
  const int kgrp = (int)(rest / (unsigned)s.nchunk);
  const int kk = kgrp * s.kg + kin;
  const int ij = chunk * BLOCK + (int)threadIdx.x;
  if (kk >= s.b.n3 || ij >= s.b.n1 * s.b.n2) return false;
  const int jj = ij / s.b.n1;
  i = s.b.lo1 + (ij - jj * s.b.n1);
  j = s.b.lo2 + jj;
  k = s.b.lo3 + kk;
  return true;
}

// ------------------------------------------------------------- geometry --

// Tables over the padded (x1, x2) plane: metric at zone centres, x1 faces,
// x2 faces; sqrt(-g) at (x1, x2) corners; connection and the geometric
// source's metric-derivative rows at centres.  x3 faces share the centre
// values (nothing depends on x3).  Pole faces and corners are left zero:
// nothing reads them.
__global__ void k_geometry(Dev g, double* tabC, double* tabF1, double* tabF2, double* corner,
                           double* conn, double* dgs) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= g.plane) return;
  int i = (int)(t % g.s1) - NG, j = (int)(t / g.s1) - NG;
  double xc1 = g.x1min + (i + 0.5) * g.dx1, xc2 = g.x2min + (j + 0.5) * g.dx2;
  double xf1 = g.x1min + i * g.dx1, xf2 = g.x2min + j * g.dx2;
  bool pole = (g.pole_lo && j == 0) || (g.pole_hi && j == g.n2);
  double gcov[10], gcon[10], gdet, alpha;
  auto put = [&](double* tab) {
    for (int f = 0; f < 10; f++) {
      tab[(G_COV + f) * g.plane + t] = gcov[f];
      tab[(G_CON + f) * g.plane + t] = gcon[f];
    }
    tab[G_DET * g.plane + t] = gdet;
    tab[G_ALPHA * g.plane + t] = alpha;
  };
  metric_point(g.st, xc1, xc2, gcov, gcon, gdet, alpha);
  put(tabC);
  metric_point(g.st, xf1, xc2, gcov, gcon, gdet, alpha);
  put(tabF1);
  if (!pole) {
    metric_point(g.st, xc1, xf2, gcov, gcon, gdet, alpha);
    put(tabF2);
    metric_point(g.st, xf1, xf2, gcov, gcon, gdet, alpha);
    corner[t] = gdet;
  } else {
    for (int f = 0; f < G_NF; f++) tabF2[f * g.plane + t] = 0.0;
    corner[t] = 0.0;
  }
  if (conn) {  // (blocks of a pack have no connection table: nothing there reads it)
    double cn[40];
    connection_point(g.st, xc1, xc2, cn);
    for (int q = 0; q < 40; q++) conn[q * g.plane + t] = cn[q];
  }
  double D[NDG];
  source_metric_point(g.st, xc1, xc2, D);
  for (int q = 0; q < NDG; q++) dgs[q * g.plane + t] = D[q];
}

// ------------------------------------------------------------ boundaries --

// Source index along one axis of a ghost coordinate, or the coordinate itself
// when the axis is interior there or frozen.  Sets flip for a polar mirror.
__device__ __forceinline__ int bc_map(int x, int n, int bclo, int bchi, bool& flip) {
  if (x < 0) {
    if (bclo == GRMHD_BC_PERIODIC) return ((x % n) + n) % n;
    if (bclo == GRMHD_BC_OUTFLOW) return 0;
    if (bclo == GRMHD_BC_POLAR) { flip = true; return -x - 1; }
    return x;
  }
  if (x >= n) {
    if (bchi == GRMHD_BC_PERIODIC) return x % n;
    if (bchi == GRMHD_BC_OUTFLOW) return n - 1;
    if (bchi == GRMHD_BC_POLAR) { flip = true; return 2 * n - 1 - x; }
    return x;
  }
  return x;
}

// Padded positions along one axis whose ghost fill copies interior x (x
// itself included), with the polar sign.
__device__ __forceinline__ int bc_preimages(int x, int n, int bclo, int bchi, int ys[7], bool fl[7]) {
  int cnt = 0;
  ys[cnt] = x;
  fl[cnt++] = false;
  for (int y = -NG; y < 0; y++) {
    bool f = false;
    if (bclo == GRMHD_BC_FROZEN) continue;
    if (bc_map(y, n, bclo, bchi, f) == x) { ys[cnt] = y; fl[cnt++] = f; }
  }
  for (int y = n; y < n + NG; y++) {
    bool f = false;
    if (bchi == GRMHD_BC_FROZEN) continue;
    if (bc_map(y, n, bclo, bchi, f) == x) { ys[cnt] = y; fl[cnt++] = f; }
  }
  return cnt;
}

// Ghost shell of the padded grid, enumerated without touching interior
// zones: the 6 x3 ghost planes (all x1, x2), then the 6 x2 ghost rows of every
// interior x3 plane (all x1), then the 6 x1 ghost zones of every interior
// (x2, x3) row.  Count = 6 s1 s2 + 6 n3 s1 + 6 n3 n2 = s1 s2 s3 - n1 n2 n3.
__host__ __device__ inline long ghost_count(const Dev& g) {
  return 6L * g.plane + 6L * g.n3 * g.s1 + 6L * g.n3 * g.n2;
}
__device__ __forceinline__ void ghost_index(const Dev& g, long t, int& i, int& j, int& k) {
  auto side = [](int l, int n) { return l < NG ? l - NG : n + (l - NG); };
  if (t < 6L * g.plane) {
    int l = (int)(t / g.plane);
    long r = t - (long)l * g.plane;
    k = side(l, g.n3);
    j = (int)(r / g.s1) - NG;
    i = (int)(r - (long)(j + NG) * g.s1) - NG;
    return;
  }
  t -= 6L * g.plane;
  const long row6 = 6L * g.s1;
  if (t < (long)g.n3 * row6) {
    k = (int)(t / row6);
    long r = t - (long)k * row6;
    int l = (int)(r / g.s1);
    j = side(l, g.n2);
    i = (int)(r - (long)l * g.s1) - NG;
    return;
  }
  t -= (long)g.n3 * row6;
  const int col6 = 6 * g.n2;
  k = (int)(t / col6);
  int r = (int)(t - (long)k * col6);
  j = r / 6;
  i = side(r - 6 * j, g.n1);
}

// One thread per ghost zone; ghost zones of non-frozen axes copy from the
// zone their per-axis maps point to (always interior along those axes, so
// nothing read here is written here).  Polar mirrors flip u~2 and B2.
__global__ void __launch_bounds__(BLOCK) k_bc(Dev g, double* P) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= ghost_count(g)) return;
  int i, j, k;
  ghost_index(g, t, i, j, k);
  bool f1 = false, f2 = false, f3 = false;
  int si = bc_map(i, g.n1, g.bc[0], g.bc[1], f1);
  int sj = bc_map(j, g.n2, g.bc[2], g.bc[3], f2);
  int sk = bc_map(k, g.n3, g.bc[4], g.bc[5], f3);
  if (si == i && sj == j && sk == k) return;  // frozen
  const long src = zid(g, si, sj, sk), dst = zid(g, i, j, k);
#pragma unroll
  for (int v = 0; v < NVAR; v++) {
    double x = P[v * g.nz + src];
    if (f2 && (v == U2 || v == B2)) x = -x;
    P[v * g.nz + dst] = x;
  }
}

// ----------------------------------------------------------------- fluxes --

template <int RECON, typename R>
__device__ __forceinline__ void recon_pair(const double* __restrict__ P, long nz, long c, long s,
                                           R eps, R qL[NVAR], R qR[NVAR]) {
#pragma unroll
  for (int v = 0; v < NVAR; v++) {
    const double* q = P + v * nz + c;
    if (RECON == GRMHD_RECON_DONOR) {
      qL[v] = (R)q[-s];
      qR[v] = (R)q[0];
    } else if (RECON == GRMHD_RECON_MC) {
      R m2 = (R)q[-2 * s], m1 = (R)q[-s], p0 = (R)q[0], p1 = (R)q[s];
      qL[v] = mc_left(m2, m1, p0);
      qR[v] = mc_right(m1, p0, p1);
    } else if (RECON == GRMHD_RECON_VL) {
      R m2 = (R)q[-2 * s], m1 = (R)q[-s], p0 = (R)q[0], p1 = (R)q[s];
      qL[v] = vl_left(m2, m1, p0);
      qR[v] = vl_right(m1, p0, p1);
    } else if (RECON == GRMHD_RECON_WENOZ) {
      R m3 = (R)q[-3 * s], m2 = (R)q[-2 * s], m1 = (R)q[-s], p0 = (R)q[0], p1 = (R)q[s],
        p2 = (R)q[2 * s];
      qL[v] = wenoz(m3, m2, m1, p0, p1, eps);
      qR[v] = wenoz(p2, p1, p0, m1, m2, eps);
    } else if (RECON == GRMHD_RECON_MP5) {
      R m3 = (R)q[-3 * s], m2 = (R)q[-2 * s], m1 = (R)q[-s], p0 = (R)q[0], p1 = (R)q[s],
        p2 = (R)q[2 * s];
      qL[v] = mp5(m3, m2, m1, p0, p1);
      qR[v] = mp5(p2, p1, p0, m1, m2);
    } else if (RECON == GRMHD_RECON_PPM) {
      R m3 = (R)q[-3 * s], m2 = (R)q[-2 * s], m1 = (R)q[-s], p0 = (R)q[0], p1 = (R)q[s],
        p2 = (R)q[2 * s];
      R l, r;
      ppm_edges(m3, m2, m1, p0, p1, l, r);  // zone i-1: its right edge
      qL[v] = r;
      ppm_edges(m2, m1, p0, p1, p2, l, r);  // zone i: its left edge
      qR[v] = l;
    } else if (RECON == GRMHD_RECON_PPMX) {
      R m3 = (R)q[-3 * s], m2 = (R)q[-2 * s], m1 = (R)q[-s], p0 = (R)q[0], p1 = (R)q[s],
        p2 = (R)q[2 * s];
      R l, r;
      ppmx_edges(m3, m2, m1, p0, p1, l, r);  // zone i-1: its right edge
      qL[v] = r;
      ppmx_edges(m2, m1, p0, p1, p2, l, r);  // zone i: its left edge
      qR[v] = l;
    } else {
      R m3 = (R)q[-3 * s], m2 = (R)q[-2 * s], m1 = (R)q[-s], p0 = (R)q[0], p1 = (R)q[s],
        p2 = (R)q[2 * s];
      qL[v] = weno5(m3, m2, m1, p0, p1, eps);
      qR[v] = weno5(p2, p1, p0, m1, m2, eps);
    }
  }
}

// Local Lax-Friedrichs flux of one face from its left and right states qL,
// qR, with the face metric at table position q2; stored at padded index c.
template <int D, typename R, typename FT>
__device__ __forceinline__ void face_llf(const Dev& g, const R qL[NVAR], const R qR[NVAR],
                                         const double* __restrict__ tab, long q2, FT* __restrict__ F,
                                         long c) {
  FaceMetric<R> m;
  load_face_metric<R>(tab, g.plane, q2, m);
  const R gam = (R)g.gam;
  R FL[NVAR], UL[NVAR], cpl, cml;
  face_side<D, R>(qL, m, gam, FL, UL, cpl, cml);
  R FR[NVAR], UR[NVAR], cpr, cmr;
  face_side<D, R>(qR, m, gam, FR, UR, cpr, cmr);
  R cmax = fmax(fmax(cpl, cpr), fmax(-cml, -cmr));
  cmax = fmax(cmax, (R)0);
  // the normal field component's flux is not stored: Flux-CT replaces it by
  // zero and nothing reads it
#pragma unroll
  for (int v = 0; v < NVAR; v++)
    if (v != B1 + D - 1)
      F[v * g.nz + c] = (FT)(m.gdet * fma((R)-0.5 * cmax, UR[v] - UL[v], (R)0.5 * (FL[v] + FR[v])));
}

template <int D>
__device__ __forceinline__ bool pole_face(const Dev& g, int j) {
  return D == 2 && ((g.pole_lo && j == 0) || (g.pole_hi && j == g.n2));
}

// Local Lax-Friedrichs flux through the lower d-face of zone (i, j, k); pole
// faces get zero flux.  FT is the stored type.
// With face fields (face-centred CT, phi not null: sqrt(-g) B^D on the lower
// D-faces), the normal field of both states is phi / sqrt(-g) at the face.
template <int D, int RECON, typename R, typename FT>
__device__ __forceinline__ void flux_face(const Dev& g, const double* __restrict__ P,
                                          const double* __restrict__ tab, FT* __restrict__ F, int i,
                                          int j, int k, const double* __restrict__ phi = nullptr) {
  long c = zid(g, i, j, k);
  if (pole_face<D>(g, j)) {
#pragma unroll
    for (int v = 0; v < NVAR; v++) F[v * g.nz + c] = (FT)0;
    return;
  }
  const long s = D == 1 ? 1 : (D == 2 ? (long)g.s1 : g.plane);
  R qL[NVAR], qR[NVAR];
  recon_pair<RECON, R>(P, g.nz, c, s, (R)g.weno_eps, qL, qR);
  const long q2 = pid(g, i, j);
  if (phi) {
    const R bn = (R)(phi[c] / tab[G_DET * g.plane + q2]);
    qL[B1 + D - 1] = bn;
    qR[B1 + D - 1] = bn;
  }
  face_llf<D, R, FT>(g, qL, qR, tab, q2, F, c);
}

#ifndef FLUX_WAVES
#define FLUX_WAVES 3
#endif
// The LDS-tiled x2 and x3 face sweeps of WENO5 (below; FLUX_TILE 0
// evaluates those faces one by one, with the same results bit for bit):
// steps of four zone rows per segment, faces per segment, right-edge row
// buffers.
#ifndef TILE_STEPS
#define TILE_STEPS 4
#endif
#ifndef FLUX_TILE
#define FLUX_TILE 1
#endif
constexpr int TILE_FACES = 4 * TILE_STEPS - 1;
constexpr int TILE_NBUF = 3;

// All three face directions in one launch: workgroups [0, nb1) take x1
// faces, [nb1, nb1 + nb2) x2 faces, the rest x3 faces (nb1 and nb2 are
// multiples of 8, so each part keeps the XCD-aware order of its schedule).
// For MC and WENO5 the x1 part is the shared-edge sweep, for WENO5 the x2
// and x3 parts are the LDS-tiled sweeps (below); other schemes and parts
// evaluate face by face.
template <int RECON, typename R, typename FT, bool FACE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(FACE ? 3 : FLUX_WAVES, 8)))
k_flux_all(Dev g, Sched b1, Sched b2, Sched b3, unsigned nb1, unsigned nb2, unsigned nb3,
           const double* __restrict__ P, const double* __restrict__ tabF1,
           const double* __restrict__ tabF2, const double* __restrict__ tabC, FT* __restrict__ F1,
           FT* __restrict__ F2, FT* __restrict__ F3, const double* __restrict__ ph1,
           const double* __restrict__ ph2, const double* __restrict__ ph3) {
  constexpr bool shared = RECON == GRMHD_RECON_MC || RECON == GRMHD_RECON_WENO5;
  // (WENO5 only: for MC the pair saves little arithmetic and the tile's
  // registers and LDS cost a wave per SIMD)
  constexpr bool tiled = RECON == GRMHD_RECON_WENO5 && FLUX_TILE;
  __shared__ R rows[tiled ? TILE_NBUF * 4 * NVAR * 64 : 1];
  const unsigned b = blockIdx.x;
  int i, j, k;
  if (b < nb1) {
    if (shared)
      sweep_x1<RECON, R, FT, FACE>(g, xcd_order(b, nb1), P, tabF1, F1, ph1);
    else if (sched_index(b1, b, nb1, i, j, k))
      flux_face<1, RECON, R, FT>(g, P, tabF1, F1, i, j, k, FACE ? ph1 : nullptr);
  } else if (b < nb1 + nb2) {
    if (tiled)
      sweep_tile<2, RECON, R, FT, FACE>(g, xcd_order(b - nb1, nb2), P, tabF2, F2, ph2, rows);
    else if (sched_index(b2, b - nb1, nb2, i, j, k))
      flux_face<2, RECON, R, FT>(g, P, tabF2, F2, i, j, k, FACE ? ph2 : nullptr);
  } else {
    if (tiled)
      sweep_tile<3, RECON, R, FT, FACE>(g, xcd_order(b - nb1 - nb2, nb3), P, tabC, F3, ph3, rows);
    else if (sched_index(b3, b - nb1 - nb2, nb3, i, j, k))
      flux_face<3, RECON, R, FT>(g, P, tabC, F3, i, j, k, FACE ? ph3 : nullptr);
  }
}

// ------------------------------------------- x1 faces with shared edges --
//
// MC and WENO5 give both edge values of a zone from one slope (MC) or one
// set of smoothness indicators and weight products (WENO5): the indicators
// of a stencil are symmetric under reversing it, so the left edge, the
// reversed-stencil evaluation, reuses them bit for bit.  For the x1 faces of
// these two schemes every lane reconstructs one zone of the box i in
// [-1, n1], j in [-1, n2], k in [-1, n3] (linearised x1-fastest); each
// wavefront starts one zone before the last zone of the previous one, and a
// face takes its left state, the right edge of the zone below it, from the
// lane below (a cross-lane shift).  Lane 0 and the zones i = -1 give no
// face.  The face values are those of the per-face evaluation bit for bit.

// Both edges of the zone c of stencil (a, b, c, d, e) along the axis.
template <int RECON>
__device__ __forceinline__ void edge_pair(double a, double b, double c, double d, double e, double eps,
                                          double& left, double& right) {
  if (RECON == GRMHD_RECON_MC) {
    (void)a;
    (void)e;
    (void)eps;
    left = mc_right(b, c, d);   // the per-face forms, rounded alike
    right = mc_left(b, c, d);
  } else {
    weno5_pair(a, b, c, d, e, eps, left, right);
  }
}
template <int RECON>
__device__ __forceinline__ void edge_pair(float a, float b, float c, float d, float e, float eps,
                                          float& left, float& right) {
  if (RECON == GRMHD_RECON_MC) {
    (void)a;
    (void)e;
    (void)eps;
    left = mc_right(b, c, d);
    right = mc_left(b, c, d);
  } else {
    weno5_pair(a, b, c, d, e, eps, left, right);
  }
}

// Both edges of every prim of the zone at padded index c along x1.
template <int RECON, typename R>
__device__ __forceinline__ void zone_edges_x1(const double* __restrict__ P, long nz, long c, R eps,
                                              R left[NVAR], R right[NVAR]) {
#pragma unroll
  for (int v = 0; v < NVAR; v++) {
    const double* q = P + v * nz + c;
    const R m1 = (R)q[-1], p0 = (R)q[0], p1 = (R)q[1];
    const R m2 = RECON == GRMHD_RECON_MC ? p0 : (R)q[-2];
    const R p2 = RECON == GRMHD_RECON_MC ? p0 : (R)q[2];
    edge_pair<RECON>(m2, m1, p0, p1, p2, eps, left[v], right[v]);
  }
}

// Workgroups of the shared-edge x1 part for a box of n1z zones (4 wavefronts
// of 63 new zones each), rounded up to a multiple of 8.
inline unsigned x1_sweep_blocks(long n1z) {
  const long waves = (n1z + 62) / 63;
  return (unsigned)(((waves + 3) / 4 + 7) / 8 * 8);
}

// lb: this workgroup's place in the part (XCD-ordered).
template <int RECON, typename R, typename FT, bool FACE>
__device__ __forceinline__ void sweep_x1(const Dev& g, unsigned lb, const double* __restrict__ P,
                                         const double* __restrict__ tabF1, FT* __restrict__ F1,
                                         const double* __restrict__ ph1) {
  const int lane = (int)(threadIdx.x & 63u);
  const int wave = (int)(lb * (BLOCK / 64) + (threadIdx.x >> 6));
  const unsigned m1 = (unsigned)g.n1 + 2u, m12 = m1 * ((unsigned)g.n2 + 2u);
  const int t = wave * 63 + lane - 1;
  const bool valid = t >= 0 && t < (int)(m12 * ((unsigned)g.n3 + 2u));
  const unsigned tt = valid ? (unsigned)t : 0u;
  const unsigned kk = tt / m12, r = tt - kk * m12;
  const unsigned jj = r / m1;
  const int i = (int)(r - jj * m1) - 1, j = (int)jj - 1, k = (int)kk - 1;
  const long c = zid(g, i, j, k);
  R left[NVAR], right[NVAR];
  zone_edges_x1<RECON, R>(P, g.nz, c, (R)g.weno_eps, left, right);
  // left state of this zone's lower face: the right edge of the zone below,
  // held by the lane below (every lane takes part in the shift)
  R qL[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) qL[v] = __shfl_up(right[v], 1);
  if (!valid || lane == 0 || i < 0) return;
  const long q2 = pid(g, i, j);
  if (FACE) {
    const R bn = (R)(ph1[c] / tabF1[G_DET * g.plane + q2]);
    qL[B1] = bn;
    left[B1] = bn;
  }
  face_llf<1, R, FT>(g, qL, left, tabF1, q2, F1, c);
}

// ------------------------------- x2 and x3 faces with shared edges (LDS) --
//
// The same sharing along x2 and x3, where the zone below a face is not in the
// lane below: a workgroup takes 64 columns of the face box (one per lane:
// (x1, x3) positions for x2 faces, (x1, x2) for x3 faces, linearised
// x1-fastest) and marches along the face axis over a segment of faces.  In
// each step its four wavefronts reconstruct four consecutive zone rows (both
// edges of all prims, edge_pair), each wavefront's right edges go through
// LDS to the wavefront of the row above, and every wavefront forms the lower
// face of its row from that left state and its own left edge.  The first row
// of a segment is the zone below its first face (reconstructed, no face).
// The right-edge rows are triple-buffered, so one barrier per step orders
// everything: the buffer a step writes was last read in the step before the
// previous one, and every wavefront has passed the barrier in between.
// The face values are those of the per-face evaluation bit for bit.

// Columns and faces of the tiled part for direction D (2 or 3).
__host__ __device__ inline long tile_columns(const Dev& g, int D) {
  return (long)(g.n1 + 2) * ((D == 2 ? g.n3 : g.n2) + 2);
}
__host__ __device__ inline int tile_faces(const Dev& g, int D) { return (D == 2 ? g.n2 : g.n3) + 1; }
// Workgroups of the tiled part: column groups of 64 times segments, rounded
// up to a multiple of 8.
inline unsigned tile_blocks(const Dev& g, int D) {
  const long ncg = (tile_columns(g, D) + 63) / 64;
  const long nseg = (tile_faces(g, D) + TILE_FACES - 1) / TILE_FACES;
  return (unsigned)((ncg * nseg + 7) / 8 * 8);
}

// Both edges of every prim of the zone at padded index c along the axis of
// stride s: the left edges into left[], the right edges stored to
// rows[v * 64] as they are formed.
template <int RECON, typename R>
__device__ __forceinline__ void zone_edges(const double* __restrict__ P, long nz, long c, long s, R eps,
                                           R left[NVAR], R* rows) {
#pragma unroll
  for (int v = 0; v < NVAR; v++) {
    const double* q = P + v * nz + c;
    const R m1 = (R)q[-s], p0 = (R)q[0], p1 = (R)q[s];
    const R m2 = RECON == GRMHD_RECON_MC ? p0 : (R)q[-2 * s];
    const R p2 = RECON == GRMHD_RECON_MC ? p0 : (R)q[2 * s];
    R right;
    edge_pair<RECON>(m2, m1, p0, p1, p2, eps, left[v], right);
    rows[v * 64] = right;
  }
}

// lb: this workgroup's place in the part (XCD-ordered); nb: workgroups in
// the part; rows: the LDS right-edge buffers (TILE_NBUF x 4 x NVAR x 64).
template <int D, int RECON, typename R, typename FT, bool FACE>
__device__ __forceinline__ void sweep_tile(const Dev& g, unsigned lb, const double* __restrict__ P,
                                           const double* __restrict__ tab, FT* __restrict__ F,
                                           const double* __restrict__ ph, R* rows) {
  const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
  const long ncol = tile_columns(g, D);
  const int nface = tile_faces(g, D);
  const unsigned nseg = (unsigned)((nface + TILE_FACES - 1) / TILE_FACES);
  const unsigned cg = lb / nseg, sg = lb - cg * nseg;
  const long col = (long)cg * 64 + lane;
  const bool colvalid = col < ncol;
  const long cc = colvalid ? col : 0;
  const int m1 = g.n1 + 2;
  const int i = (int)(cc % m1) - 1, o = (int)(cc / m1) - 1;   // o: the other transverse index
  const int fs = (int)sg * TILE_FACES;
  const int fe = fs + TILE_FACES < nface ? fs + TILE_FACES : nface;
  // a workgroup past the last segment (rounding) runs no step
  const int nsteps = fs < nface ? (fe - fs + 1 + 3) / 4 : 0;
  const long s = D == 2 ? (long)g.s1 : g.plane;
  for (int t = 0; t < nsteps; t++) {
    const int r = fs - 1 + 4 * t + w;            // zone row along the face axis
    const bool rowvalid = r <= fe - 1;
    const int rr = rowvalid ? r : fe - 1;        // rows past the segment load an in-range stencil
    const long c = D == 2 ? zid(g, i, rr, o) : zid(g, i, o, rr);
    R left[NVAR];
    zone_edges<RECON, R>(P, g.nz, c, s, (R)g.weno_eps, left, rows + ((t % TILE_NBUF) * 4 + w) * NVAR * 64 + lane);
    __syncthreads();
    if (!colvalid || !rowvalid || r < fs) continue;
    // left state: the right edge of the row below (for the first wavefront,
    // the last row of the previous step)
    const R* rd = w > 0 ? rows + ((t % TILE_NBUF) * 4 + (w - 1)) * NVAR * 64
                        : rows + (((t + TILE_NBUF - 1) % TILE_NBUF) * 4 + 3) * NVAR * 64;
    R qL[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; v++) qL[v] = rd[v * 64 + lane];
    if (pole_face<D>(g, r)) {
#pragma unroll
      for (int v = 0; v < NVAR; v++) F[v * g.nz + c] = (FT)0;
      continue;
    }
    long q2 = D == 2 ? pid(g, i, r) : pid(g, i, o);
    // x3 faces: the face metric is the same for the whole column; keep its
    // loads in the step (hoisted out of the loop it would be held through
    // the reconstruction and spilled)
    if (D == 3) asm volatile("" : "+v"(q2));
    if (FACE) {
      const R bn = (R)(ph[c] / tab[G_DET * g.plane + q2]);
      qL[B1 + D - 1] = bn;
      left[B1 + D - 1] = bn;
    }
    face_llf<D, R, FT>(g, qL, left, tab, q2, F, c);
  }
}

// Flux-CT edge EMFs at the lower (x1, x2, x3) corner of zone (i, j, k):
//   E3 = [F1(B2) + F1(B2)_{j-1} - F2(B1) - F2(B1)_{i-1}]/4
//   E2 = [F3(B1) + F3(B1)_{i-1} - F1(B3) - F1(B3)_{k-1}]/4
//   E1 = [F2(B3) + F2(B3)_{k-1} - F3(B2) - F3(B2)_{j-1}]/4
// E1 and E3 vanish on polar edges (sqrt(-g) = 0 there).
template <typename FT>
__device__ __forceinline__ void emf_edge(const Dev& g, const FT* __restrict__ F1, const FT* __restrict__ F2,
                                         const FT* __restrict__ F3, FT* __restrict__ E1,
                                         FT* __restrict__ E2, FT* __restrict__ E3, int i, int j, int k) {
  long c = zid(g, i, j, k);
  const long nz = g.nz, si = 1, sj = g.s1, sk = g.plane;
  bool pole = (g.pole_lo && j == 0) || (g.pole_hi && j == g.n2);
  const FT q = (FT)0.25;
  FT e3 = q * (F1[B2 * nz + c] + F1[B2 * nz + c - sj] - F2[B1 * nz + c] - F2[B1 * nz + c - si]);
  FT e2 = q * (F3[B1 * nz + c] + F3[B1 * nz + c - si] - F1[B3 * nz + c] - F1[B3 * nz + c - sk]);
  FT e1 = q * (F2[B3 * nz + c] + F2[B3 * nz + c - sk] - F3[B2 * nz + c] - F3[B2 * nz + c - sj]);
  E1[c] = pole ? (FT)0 : e1;
  E2[c] = e2;
  E3[c] = pole ? (FT)0 : e3;
}

// With gate, runs only when *gate is non-zero (the flux correction's second
// EMF pass); with zero, its first workgroup clears *zero (the mark count of
// the stage about to be taken).
template <typename FT>
__global__ void __launch_bounds__(BLOCK) k_emf(Dev g, Sched box, const FT* __restrict__ F1,
                                               const FT* __restrict__ F2, const FT* __restrict__ F3,
                                               FT* __restrict__ E1, FT* __restrict__ E2,
                                               FT* __restrict__ E3, const unsigned long long* gate,
                                               unsigned long long* zero) {
  if (gate && *gate == 0) return;
  if (zero && blockIdx.x == 0 && threadIdx.x == 0) *zero = 0;
  int i, j, k;
  if (!sched_index(box, blockIdx.x, gridDim.x, i, j, k)) return;
  emf_edge<FT>(g, F1, F2, F3, E1, E2, E3, i, j, k);
}

// Mark of the zone at (i, j, k) for the flux correction: interior zones
// their own; a ghost index on a periodic axis wraps to the zone it copies;
// other ghosts are never marked.
__device__ __forceinline__ bool marked(const Dev& g, const unsigned char* __restrict__ mark, int i, int j,
                                       int k) {
  int idx[3] = {i, j, k};
  const int n[3] = {g.n1, g.n2, g.n3};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (idx[a] >= 0 && idx[a] < n[a]) continue;
    if (g.bc[2 * a] != GRMHD_BC_PERIODIC) return false;
    idx[a] = ((idx[a] % n[a]) + n[a]) % n[a];
  }
  return mark[zid(g, idx[0], idx[1], idx[2])] != 0;
}

// First-order flux correction: every face of the flux boxes (the same faces
// the flux launch computes) whose either zone is marked gets the local
// Lax-Friedrichs flux of donor-cell states.  Runs only when *gate (the mark
// count) is non-zero; one thread per face, faces of unmarked zones return
// after two byte loads.
template <typename R, typename FT>
__global__ void __launch_bounds__(BLOCK) k_fofc_flux(Dev g, Box b1, Box b2, Box b3, const double* __restrict__ P,
                                                     const double* __restrict__ tabF1,
                                                     const double* __restrict__ tabF2,
                                                     const double* __restrict__ tabC, FT* __restrict__ F1,
                                                     FT* __restrict__ F2, FT* __restrict__ F3,
                                                     const unsigned char* __restrict__ mark,
                                                     const unsigned long long* gate,
                                                     const double* __restrict__ ph1,
                                                     const double* __restrict__ ph2,
                                                     const double* __restrict__ ph3) {
  if (*gate == 0) return;
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long c1 = b1.count(), c2 = b2.count();
  int i, j, k;
  if (t < c1) {
    box_index(b1, t, i, j, k);
    if (marked(g, mark, i, j, k) || marked(g, mark, i - 1, j, k))
      flux_face<1, GRMHD_RECON_DONOR, R, FT>(g, P, tabF1, F1, i, j, k, ph1);
  } else if (t < c1 + c2) {
    box_index(b2, t - c1, i, j, k);
    if (marked(g, mark, i, j, k) || marked(g, mark, i, j - 1, k))
      flux_face<2, GRMHD_RECON_DONOR, R, FT>(g, P, tabF2, F2, i, j, k, ph2);
  } else {
    if (!box_index(b3, t - c1 - c2, i, j, k)) return;
    if (marked(g, mark, i, j, k) || marked(g, mark, i, j, k - 1))
      flux_face<3, GRMHD_RECON_DONOR, R, FT>(g, P, tabC, F3, i, j, k, ph3);
  }
}

// ------------------------------------------------------- face-centred CT --
// Face-centred constrained transport (Algorithm section: the scheme of Stone
// & Gardiner; edge EMFs with or without upwinding).  The magnetic state is
// phi_d = sqrt(-g) B^d on the lower d-face of every zone; a zone's field is
// the mean of its two faces.  Edge EMFs E3 = F^1(B^2) = -F^2(B^1) on x1-x2
// edges and cyclically: the averaged scheme is the Flux-CT average of the
// four face values (k_emf); the upwinded one (Gardiner & Stone 2005) adds,
// along each in-plane direction, a quarter of (lower minus upper) gradient
// across the edge, each the difference of a face value and a zone-centre EMF
// taken in the zone the mass flux through the adjoining face comes from (the
// mean of both zones where it is zero), so that flow along one grid
// direction gets its face EMF.  A face mass flux within 1e-10 (FP64; 1e-5
// for the FP32 fluxes) of its two zones' mass-current scale, sqrt(-g) rho
// (|u^t| + sum_d |u^d|) each, counts as zero: its sign would be roundoff.
// Faces evolve by Stokes' theorem (face divergence kept to roundoff).

// Ghost faces: the per-axis maps composed (equal to axis-by-axis passes).
// Along a face array's own axis (faces 0..n evolve): periodic wraps modulo n,
// outflow copies the boundary face, polar mirrors about the axis face with
// the sign flipped; across it the zone maps (polar mirror without flip).
// Frozen ghosts keep their values.  One thread per padded position of each
// of the three arrays; interior positions return at once.
__device__ __forceinline__ void face_map(int x, int n, bool normal, int bc_lo, int bc_hi, int& src,
                                         bool& flip) {
  const int last = normal ? n : n - 1;
  src = x;
  if (x >= 0 && x <= last) return;
  const int bc = x < 0 ? bc_lo : bc_hi;
  if (bc == GRMHD_BC_PERIODIC) {
    src = ((x % n) + n) % n;  // faces n and 0 coincide
  } else if (bc == GRMHD_BC_OUTFLOW) {
    src = x < 0 ? 0 : last;
  } else if (bc == GRMHD_BC_POLAR) {
    if (normal) {
      src = x < 0 ? -x : 2 * n - x;
      flip = !flip;
    } else {
      src = x < 0 ? -1 - x : 2 * n - 1 - x;
    }
  }  // frozen: the position keeps its own value
}

__global__ void __launch_bounds__(BLOCK) k_bc_faces(Dev g, double* __restrict__ ph1, double* __restrict__ ph2,
                                                    double* __restrict__ ph3) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= 3 * g.nz) return;
  const int d = (int)(t / g.nz);
  const long q = t - d * g.nz;
  const int i = (int)(q % g.s1) - NG, j = (int)((q / g.s1) % g.s2) - NG, k = (int)(q / g.plane) - NG;
  const int idx[3] = {i, j, k}, n[3] = {g.n1, g.n2, g.n3};
  int src[3];
  bool flip = false;
#pragma unroll
  for (int a = 0; a < 3; a++) face_map(idx[a], n[a], a == d, g.bc[2 * a], g.bc[2 * a + 1], src[a], flip);
  if (src[0] == i && src[1] == j && src[2] == k) return;  // interior, or frozen
  double* ph = d == 0 ? ph1 : (d == 1 ? ph2 : ph3);
  const double x = ph[zid(g, src[0], src[1], src[2])];
  ph[q] = flip ? -x : x;
}

// Zone-centre EMFs (E1, E2, E3) = (F^2(B^3), F^3(B^1), F^1(B^2)) and the
// mass-current scale |U(rho)| + sum_d |F^d(rho)| from the zone prims, over
// zones -1..n (the upwinded edge EMFs read them).
template <typename R, typename FT>
__global__ void __launch_bounds__(BLOCK) k_cell_emf(Dev g, Box box, const double* __restrict__ P,
                                                    const double* __restrict__ tabC, FT* __restrict__ C1,
                                                    FT* __restrict__ C2, FT* __restrict__ C3,
                                                    FT* __restrict__ S) {
#pragma clang fp contract(off)
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (!box_index(box, t, i, j, k)) return;
  const long c = zid(g, i, j, k);
  R p[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) p[v] = (R)P[v * g.nz + c];
  PointMetric<R> m;
  load_metric<R>(tabC, g.plane, pid(g, i, j), m);
  Fluid<R> f;
  fluid_state(p, m, f);
  // the components prim_to_flux gives for F^d(rho) and F^d(B^k), written
  // out with the same operations: sqrt(-g) rho u^d, sqrt(-g)(b^k u^d - b^d u^k)
  const R gr = m.gdet * p[RHO];
  R sc = fabs(gr * f.ucon[0]);
  C3[c] = (FT)(m.gdet * (f.bcon[2] * f.ucon[1] - f.bcon[1] * f.ucon[2]));
  sc = sc + fabs(gr * f.ucon[1]);
  C1[c] = (FT)(m.gdet * (f.bcon[3] * f.ucon[2] - f.bcon[2] * f.ucon[3]));
  sc = sc + fabs(gr * f.ucon[2]);
  C2[c] = (FT)(m.gdet * (f.bcon[1] * f.ucon[3] - f.bcon[3] * f.ucon[1]));
  sc = sc + fabs(gr * f.ucon[3]);
  S[c] = (FT)sc;
}

// Upwinded (Gardiner & Stone) edge EMFs at the lower corner of zone (i, j,
// k), edges 0..n; gate/zero as in k_emf.  Same operation order as the CPU
// reference of the scheme.
template <typename FT>
__global__ void __launch_bounds__(BLOCK) k_emf_gs(Dev g, Sched box, const FT* __restrict__ F1,
                                                  const FT* __restrict__ F2, const FT* __restrict__ F3,
                                                  const FT* __restrict__ C1, const FT* __restrict__ C2,
                                                  const FT* __restrict__ C3, const FT* __restrict__ S,
                                                  FT* __restrict__ E1,
                                                  FT* __restrict__ E2, FT* __restrict__ E3,
                                                  const unsigned long long* gate, unsigned long long* zero) {
#pragma clang fp contract(off)
  if (gate && *gate == 0) return;
  if (zero && blockIdx.x == 0 && threadIdx.x == 0) *zero = 0;
  int i, j, k;
  if (!sched_index(box, blockIdx.x, gridDim.x, i, j, k)) return;
  const long c = zid(g, i, j, k), nz = g.nz;
  const long st[3] = {1, g.s1, g.plane};
  const bool pole = (g.pole_lo && j == 0) || (g.pole_hi && j == g.n2);
  const FT* Fd[3] = {F1, F2, F3};
  const FT* Cd[3] = {C1, C2, C3};
  FT* Ed[3] = {E1, E2, E3};
  const FT tiny = sizeof(FT) == 8 ? (FT)1e-10 : (FT)1e-5;
  auto up = [&](FT flux, FT scale, FT lower, FT upper) -> FT {
    if (fabs(flux) <= tiny * scale) return (FT)0.5 * (lower + upper);
    return flux > (FT)0 ? lower : upper;
  };
#pragma unroll
  for (int e = 0; e < 3; e++) {
    if (pole && e != 1) {
      Ed[e][c] = (FT)0;
      continue;
    }
    const int a = (e + 1) % 3, b = (e + 2) % 3;  // axes of the edge's plane, cyclic
    const FT* Fa = Fd[a];
    const FT* Fb = Fd[b];
    const FT* C = Cd[e];
    const long sa = st[a], sb = st[b];
    const long p00 = c, p10 = c - sa, p01 = c - sb, p11 = c - sa - sb;
    const FT ea0 = Fa[(B1 + b) * nz + p00], ea1 = Fa[(B1 + b) * nz + p01];
    const FT eb0 = -Fb[(B1 + a) * nz + p00], eb1 = -Fb[(B1 + a) * nz + p10];
    FT ed = (FT)0.25 * (((ea0 + ea1) + eb0) + eb1);
    const FT fa0 = Fa[RHO * nz + p00], fa1 = Fa[RHO * nz + p01];
    const FT sa0 = S[p10] + S[p00], sa1 = S[p11] + S[p01];
    const FT dbp = up(fa0, sa0, C[p10] - eb1, C[p00] - eb0);
    const FT dbm = up(fa1, sa1, eb1 - C[p11], eb0 - C[p01]);
    const FT fb0 = Fb[RHO * nz + p00], fb1 = Fb[RHO * nz + p10];
    const FT sb0 = S[p01] + S[p00], sb1 = S[p11] + S[p10];
    const FT dap = up(fb0, sb0, C[p01] - ea1, C[p00] - ea0);
    const FT dam = up(fb1, sb1, ea1 - C[p11], ea0 - C[p10]);
    ed = ed + (FT)0.25 * (dbm - dbp) + (FT)0.25 * (dam - dap);
    Ed[e][c] = ed;
  }
}

// Face update of one stage over the evolved faces (0..n along a face's
// axis, interior across): stage 1 phi1 = phin + dt R, V = (phin + phi1)/2;
// stage 2 phin+1 = V + (dt/2) R, with R the Stokes rate
//   R1 = dE3/dx2 - dE2/dx3, R2 = dE1/dx3 - dE3/dx1, R3 = dE2/dx1 - dE1/dx2.
// gate as in k_update's final pass.
template <int STAGE, typename FT>
__global__ void __launch_bounds__(BLOCK) k_face_update(Dev g, Box box, const FT* __restrict__ E1,
                                                       const FT* __restrict__ E2, const FT* __restrict__ E3,
                                                       const double* __restrict__ b1, const double* __restrict__ b2,
                                                       const double* __restrict__ b3, double* __restrict__ o1,
                                                       double* __restrict__ o2, double* __restrict__ o3,
                                                       double* __restrict__ v1, double* __restrict__ v2,
                                                       double* __restrict__ v3, double dt,
                                                       const double* __restrict__ dt_dev,
                                                       const unsigned long long* gate) {
#pragma clang fp contract(off)
  if (gate && *gate == 0) return;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (!box_index(box, t, i, j, k)) return;
  if (dt_dev) dt = *dt_dev;
  const double h = STAGE == 1 ? dt : 0.5 * dt;
  const long c = zid(g, i, j, k), si = 1, sj = g.s1, sk = g.plane;
  auto e = [&](const FT* E, long o) { return (double)E[c + o]; };
  if (j < g.n2 && k < g.n3) {
    const double r = (e(E3, sj) - e(E3, 0)) / g.dx2 - (e(E2, sk) - e(E2, 0)) / g.dx3;
    const double x = b1[c] + h * r;
    o1[c] = x;
    if (STAGE == 1) v1[c] = 0.5 * (b1[c] + x);
  }
  if (i < g.n1 && k < g.n3) {
    const double r = (e(E1, sk) - e(E1, 0)) / g.dx3 - (e(E3, si) - e(E3, 0)) / g.dx1;
    const double x = b2[c] + h * r;
    o2[c] = x;
    if (STAGE == 1) v2[c] = 0.5 * (b2[c] + x);
  }
  if (i < g.n1 && j < g.n2) {
    const double r = (e(E2, si) - e(E2, 0)) / g.dx1 - (e(E1, sj) - e(E1, 0)) / g.dx2;
    const double x = b3[c] + h * r;
    o3[c] = x;
    if (STAGE == 1) v3[c] = 0.5 * (b3[c] + x);
  }
}

// Interior zones' B prims from the faces (after faces are loaded).
__global__ void __launch_bounds__(BLOCK) k_cell_b(Dev g, Box box, const double* __restrict__ ph1,
                                                  const double* __restrict__ ph2, const double* __restrict__ ph3,
                                                  const double* __restrict__ tabC, double* __restrict__ P) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (!box_index(box, t, i, j, k)) return;
  const long c = zid(g, i, j, k);
  const double gd = tabC[G_DET * g.plane + pid(g, i, j)];
  P[B1 * g.nz + c] = 0.5 * (ph1[c] + ph1[c + 1]) / gd;
  P[B2 * g.nz + c] = 0.5 * (ph2[c] + ph2[c + g.s1]) / gd;
  P[B3 * g.nz + c] = 0.5 * (ph3[c] + ph3[c + g.plane]) / gd;
}

// Rebuild the B components of interior-face fluxes from the EMFs (as the
// update does on the fly); used by the flux inspection entry point only.
template <typename FT>
__global__ void k_ct_fluxes(Dev g, Box box, FT* F1, FT* F2, FT* F3, const FT* E1, const FT* E2,
                            const FT* E3) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (!box_index(box, t, i, j, k)) return;
  long c = zid(g, i, j, k);
  const long nz = g.nz, si = 1, sj = g.s1, sk = g.plane;
  const FT h = (FT)0.5;
  if (j < g.n2 && k < g.n3) {
    F1[B1 * nz + c] = (FT)0;
    F1[B2 * nz + c] = h * (E3[c] + E3[c + sj]);
    F1[B3 * nz + c] = -h * (E2[c] + E2[c + sk]);
  }
  if (i < g.n1 && k < g.n3) {
    F2[B1 * nz + c] = -h * (E3[c] + E3[c + si]);
    F2[B2 * nz + c] = (FT)0;
    F2[B3 * nz + c] = h * (E1[c] + E1[c + sk]);
  }
  if (i < g.n1 && j < g.n2) {
    F3[B1 * nz + c] = h * (E2[c] + E2[c + si]);
    F3[B2 * nz + c] = -h * (E1[c] + E1[c + sj]);
    F3[B3 * nz + c] = (FT)0;
  }
}

#include "inversion.hpp"

// ---------------------------------------------------------------- floors --

// Floors and ceilings of one zone's prims (the Physics section's injection
// of material and energy where density or internal energy drop below set
// values or too far below the magnetic pressure, in the drift frame):
//   rho_fl = max(rho_min_geom r^-3/2, b^2/bsq_over_rho_max),
//   u_fl   = max(u_min_geom r^-5/2,   b^2/bsq_over_u_max),
// r = exp(x1) in modified KS, 1 in flat space.  drho = max(rho_fl - rho, 0)
// and du = max(u_fl - u, 0) of new material moving with the drift velocity
// v_D = v - (v.B) B/B.B (normal-frame velocity v, spatial metric; v itself
// where B = 0) are added as conserved variables and the sum is inverted
// from the floored prims (B kept as it was); if that fails the floored prims
// stay (fluid-frame injection).  Then a Lorentz factor above gamma_max
// scales u~ down to it and u/rho above u_over_rho_max lowers u.  Returns
// the mask of what acted.  Same operation order as the CPU reference,
// without contraction.
enum { FL_RHO = 1, FL_U = 2, FL_FLUID_FRAME = 4, FL_GAMMA = 8, FL_TEMP = 16 };

__device__ __forceinline__ double spatial_dot(const PointMetric<double>& m, const double a[3],
                                              const double b[3]) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) s += m.gcov[sidx(i + 1, j + 1)] * a[i] * b[j];
  return s;
}

// Injection of drho, du of material moving with the drift velocity into
// the zone's prims P (fluid state f); returns FL_FLUID_FRAME if the inversion
// of the sum failed and the floored prims were kept.  Inlined on purpose: an
// out-of-line call gives the kernel a private (scratch) segment, and the
// scratch every wave then reserves cut the floors pass's speed six-fold.
__device__ __forceinline__ int inject_drift(const Dev& g, const PointMetric<double>& m, const Fluid<double>& f,
                                         double drho, double du, double P[NVAR]) {
#pragma clang fp contract(off)
  const double ut[3] = {P[U1], P[U2], P[U3]}, B[3] = {P[B1], P[B2], P[B3]};
  const double gamma = sqrt(1.0 + spatial_dot(m, ut, ut));
  double v[3], vd[3];
#pragma unroll
  for (int i = 0; i < 3; i++) v[i] = ut[i] / gamma;
  const double BB = spatial_dot(m, B, B);
  if (BB > 0.0) {
    const double vB = spatial_dot(m, v, B);
#pragma unroll
    for (int i = 0; i < 3; i++) vd[i] = v[i] - vB * B[i] / BB;
  } else {
#pragma unroll
    for (int i = 0; i < 3; i++) vd[i] = v[i];
  }
  const double gd = 1.0 / sqrt(1.0 - spatial_dot(m, vd, vd));
  double Pd[NVAR] = {drho, du, gd * vd[0], gd * vd[1], gd * vd[2], 0.0, 0.0, 0.0};
  double U[NVAR], dU[NVAR], guess[NVAR], Pn[NVAR];
  prim_to_flux(P, f, m, g.gam, 0, U);
  Fluid<double> fd;
  fluid_state(Pd, m, fd);
  prim_to_flux(Pd, fd, m, g.gam, 0, dU);
#pragma unroll
  for (int v2 = 0; v2 < NVAR; v2++) {
    U[v2] = U[v2] + dU[v2];
    guess[v2] = P[v2];
  }
  guess[RHO] = P[RHO] + drho;
  guess[UU] = P[UU] + du;
  if (invert(g, m, U, guess, Pn) == 0) {
#pragma unroll
    for (int v2 = 0; v2 < 5; v2++) P[v2] = Pn[v2];
    return 0;
  }
#pragma unroll
  for (int v2 = 0; v2 < 5; v2++) P[v2] = guess[v2];
  return FL_FLUID_FRAME;
}

__device__ __forceinline__ int apply_floors(const Dev& g, const PointMetric<double>& m, double x1,
                                            double P[NVAR]) {
#pragma clang fp contract(off)
  const double r = g.st.kerr ? exp(x1) : 1.0;
  const double sr = sqrt(r);
  Fluid<double> f;
  fluid_state(P, m, f);
  double rho_fl = g.rho_min_geom / (r * sr);
  double u_fl = g.u_min_geom / (r * r * sr);
  const double rb = f.bsq / g.bsq_over_rho_max, ub = f.bsq / g.bsq_over_u_max;
  if (rb > rho_fl) rho_fl = rb;
  if (ub > u_fl) u_fl = ub;
  double drho = rho_fl - P[RHO], du = u_fl - P[UU];
  if (drho < 0.0) drho = 0.0;
  if (du < 0.0) du = 0.0;
  int mask = 0;
  if (drho > 0.0 || du > 0.0)
    mask |= (drho > 0.0 ? FL_RHO : 0) | (du > 0.0 ? FL_U : 0) | inject_drift(g, m, f, drho, du, P);
  const double ut[3] = {P[U1], P[U2], P[U3]};
  const double gamma = sqrt(1.0 + spatial_dot(m, ut, ut));
  if (gamma > g.gamma_max) {
    const double fs = sqrt((g.gamma_max * g.gamma_max - 1.0) / (gamma * gamma - 1.0));
#pragma unroll
    for (int i = 0; i < 3; i++) P[U1 + i] = ut[i] * fs;
    mask |= FL_GAMMA;
  }
  if (P[UU] > g.u_over_rho_max * P[RHO]) {
    P[UU] = g.u_over_rho_max * P[RHO];
    mask |= FL_TEMP;
  }
  return mask;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  return x;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Block-wide max and sum in a fixed order (wavefront butterflies, then the
// wavefront results in index order): deterministic for a given launch shape.
__device__ void block_reduce(double& mx, double& sm) {
  __shared__ double smx[BLOCK / 64], ssm[BLOCK / 64];
  mx = wave_max(mx);
  sm = wave_sum(sm);
  int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) {
    smx[w] = mx;
    ssm[w] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = smx[0], b = ssm[0];
    for (int q = 1; q < BLOCK / 64; q++) {
      a = fmax(a, smx[q]);
      b += ssm[q];
    }
    mx = a;
    sm = b;
  }
}

// Signal-rate bound of one zone for the CFL step: the sum over axes with
// more than one zone of max(|c+|, |c-|)/dx_d at the zone centre.  A zone
// whose rate is not finite (a NaN state) reports +inf, so the max-reductions
// (fmax drops NaN operands) carry it and the step size comes out unusable.
__device__ __forceinline__ double zone_rate(const Dev& g, const double p[NVAR],
                                            const PointMetric<double>& m) {
  Fluid<double> f;
  fluid_state(p, m, f);
  double cp, cm, z = 0.0;
  if (g.n1 > 1) {
    char_speeds(p, f, m, g.gam, 1, cp, cm);
    z += fmax(fabs(cp), fabs(cm)) / g.dx1;
  }
  if (g.n2 > 1) {
    char_speeds(p, f, m, g.gam, 2, cp, cm);
    z += fmax(fabs(cp), fabs(cm)) / g.dx2;
  }
  if (g.n3 > 1) {
    char_speeds(p, f, m, g.gam, 3, cp, cm);
    z += fmax(fabs(cp), fabs(cm)) / g.dx3;
  }
  return isfinite(z) ? z : (double)INFINITY;
}

// ----------------------------------------------------------------- update --

__device__ __forceinline__ void load_conn(const double* __restrict__ conn, long plane, long q,
                                          double cn[40]) {
#pragma unroll
  for (int f = 0; f < 40; f++) cn[f] = conn[f * plane + q];
}

// Geometric source of the x1 and x2 momentum equations, S[0] and S[1], from
// the zone's metric-derivative rows (the energy and x3-momentum sources
// vanish identically in a metric independent of x0 and x3).
__device__ __forceinline__ void geometric_source(const double p[NVAR], const Fluid<double>& f,
                                                 const PointMetric<double>& m,
                                                 const double* __restrict__ dgs, long plane, long q,
                                                 double gam, double S[2]) {
  double D[NDG];
#pragma unroll
  for (int r = 0; r < NDG; r++) D[r] = x2_offdiag(r % 10) ? 0.0 : dgs[r * plane + q];
  metric_source(p, f, m, gam, D, S);
}

// One stage for every interior zone.  STAGE 1: V = (Un + U1)/2 with
// Un = U(Pin), U1 = Un + dt L(Pin); STAGE 2: U = V + dt L(Pin)/2.  Then
// Pout = U_to_P(U; guess Pin).  B fluxes come from the edge EMFs.
// Update modes: PLAIN, and the two passes of a stage under the first-order
// flux correction: PROVISIONAL (marks zones whose inversion fails, counts
// nothing else) and FINAL (the same update from the corrected fluxes,
// counted).  Floors run in a kernel of their own after each update pass
// (k_floors), with the same modes.
enum { U_PLAIN = 0, U_PROVISIONAL = 2, U_FINAL = 3, U_STORE = 4 };
// Counter slots of the context's counter array.
enum { C_FAILS = 0, C_C2P = 1, C_FLOORS = 2, C_FOFC = 3, C_FLUID = 4, C_MARKS = 5 };

// Rate of the zone field at padded index c from the edge EMFs (Flux-CT):
// F1(B2) = (E3 + E3_{j+1})/2, F1(B3) = -(E2 + E2_{k+1})/2,
// F2(B1) = -(E3 + E3_{i+1})/2, F2(B3) = (E1 + E1_{k+1})/2,
// F3(B1) = (E2 + E2_{i+1})/2, F3(B2) = -(E1 + E1_{j+1})/2; normal ones zero.
template <typename FT>
__device__ __forceinline__ void ct_field_rate(const Dev& g, const FT* __restrict__ E1, const FT* __restrict__ E2,
                                              const FT* __restrict__ E3, long c, double L[NVAR]) {
#pragma clang fp contract(off)
  const long si = 1, sj = g.s1, sk = g.plane;
  auto e = [&](const FT* E, long o) { return (double)E[c + o]; };
  double f1b2_p = 0.5 * (e(E3, si) + e(E3, si + sj)), f1b2_m = 0.5 * (e(E3, 0) + e(E3, sj));
  double f1b3_p = -0.5 * (e(E2, si) + e(E2, si + sk)), f1b3_m = -0.5 * (e(E2, 0) + e(E2, sk));
  double f2b1_p = -0.5 * (e(E3, sj) + e(E3, sj + si)), f2b1_m = -0.5 * (e(E3, 0) + e(E3, si));
  double f2b3_p = 0.5 * (e(E1, sj) + e(E1, sj + sk)), f2b3_m = 0.5 * (e(E1, 0) + e(E1, sk));
  double f3b1_p = 0.5 * (e(E2, sk) + e(E2, sk + si)), f3b1_m = 0.5 * (e(E2, 0) + e(E2, si));
  double f3b2_p = -0.5 * (e(E1, sk) + e(E1, sk + sj)), f3b2_m = -0.5 * (e(E1, 0) + e(E1, sj));
  L[B1] = -((f2b1_p - f2b1_m) * g.idx2 + (f3b1_p - f3b1_m) * g.idx3);
  L[B2] = -((f1b2_p - f1b2_m) * g.idx1 + (f3b2_p - f3b2_m) * g.idx3);
  L[B3] = -((f1b3_p - f1b3_m) * g.idx1 + (f2b3_p - f2b3_m) * g.idx2);
}

// SSPRK(5,4) of Spiteri & Ruuth (2002), Shu-Osher form, coefficients as
// published (15 digits): stage k (k = 2, 3, 4) takes A_k U^n + B_k U(k-1) +
// C_k dt L; the last stage D2 U(2) + D3 U(3) + E3 dt L(P(3)) + D4 U(4) +
// E4 dt L(P(4)).
constexpr double SSP54_C1 = 0.391752226571890;
constexpr double SSP54_A2 = 0.444370493651235, SSP54_B2 = 0.555629506348765, SSP54_C2 = 0.368410593050371;
constexpr double SSP54_A3 = 0.620101851488403, SSP54_B3 = 0.379898148511597, SSP54_C3 = 0.251891774271694;
constexpr double SSP54_A4 = 0.178079954393132, SSP54_B4 = 0.821920045606868, SSP54_C4 = 0.544974750228521;
constexpr double SSP54_D2 = 0.517231671970585, SSP54_D3 = 0.096059710526147, SSP54_E3 = 0.063692468666290,
                 SSP54_D4 = 0.386708617503269, SSP54_E4 = 0.226007483236906;

template <int STAGE, typename FT, bool RATE = false, int MODE = U_PLAIN, bool FACE = false,
          int INTEG = GRMHD_INTEG_SSPRK2>
__device__ __forceinline__ void update_zone(const Dev& g, const double* __restrict__ Pin,
                                            double* __restrict__ Pout, double* __restrict__ V,
                                            const FT* __restrict__ F1, const FT* __restrict__ F2,
                                            const FT* __restrict__ F3, const FT* __restrict__ E1,
                                            const FT* __restrict__ E2, const FT* __restrict__ E3,
                                            const double* __restrict__ tabC,
                                            const double* __restrict__ dgs, double dt,
                                            unsigned long long* fails, unsigned char* __restrict__ flags,
                                            int i, int j, int k, double* rate = nullptr,
                                            unsigned char* __restrict__ mark = nullptr,
                                            const double* __restrict__ ph1 = nullptr,
                                            const double* __restrict__ ph2 = nullptr,
                                            const double* __restrict__ ph3 = nullptr,
                                            double* __restrict__ ustar = nullptr) {
  // the FP64 update is rounded operation by operation, in the order written
#pragma clang fp contract(off)
  const long c = zid(g, i, j, k), nz = g.nz, si = 1, sj = g.s1, sk = g.plane;
  const long q2 = pid(g, i, j);
  double p[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) p[v] = Pin[v * nz + c];
  PointMetric<double> m;
  load_metric<double>(tabC, g.plane, q2, m);
  Fluid<double> f;
  fluid_state(p, m, f);

  double L[NVAR];
  {
    double S[2];
    geometric_source(p, f, m, dgs, g.plane, q2, g.gam, S);
#pragma unroll
    for (int v = 0; v < 5; v++) {
      double d1 = ((double)F1[v * nz + c + si] - (double)F1[v * nz + c]) * g.idx1;
      double d2 = ((double)F2[v * nz + c + sj] - (double)F2[v * nz + c]) * g.idx2;
      double d3 = ((double)F3[v * nz + c + sk] - (double)F3[v * nz + c]) * g.idx3;
      L[v] = -((d1 + d2) + d3);
      if (v == U1 || v == U2) L[v] += S[v - U1];
    }
    if constexpr (!FACE) {
      ct_field_rate(g, E1, E2, E3, c, L);
    } else {
      L[B1] = L[B2] = L[B3] = 0.0;
    }
  }

  // SSPRK2: U1 = U^n + dt L(P^n), V = (U^n + U1)/2, U^{n+1} = V + dt L(P1)/2;
  // predictor-corrector: U* = U^n + (dt/2) L(P^n), V = U^n, U^{n+1} = V + dt L(P*);
  // RK1: the first stage alone, no register.
  // SSPRK(5,4): three registers, R0 = U^n, R1 = the next stage's part
  // without its rate, R2 = the last stage's, each summed in the order the
  // method writes its terms:
  //   1: R0 = U^n,  U(1) = R0 + C1 dtL,  R1 = A2 R0 + B2 U(1)
  //   2: U(2) = R1 + C2 dtL,  R1 = A3 R0 + B3 U(2),  R2 = D2 U(2)
  //   3: U(3) = R1 + C3 dtL,  R1 = A4 R0 + B4 U(3),  R2 = R2 + D3 U(3)
  //   4: U(4) = R1 + C4 dtL,  R2 = (R2 + E3 dtL) + D4 U(4)
  //   5: U^{n+1} = R2 + E4 dtL
  double U[NVAR];
  if constexpr (INTEG == GRMHD_INTEG_SSPRK54) {
    double* R0 = V;
    double* R1 = V + NVAR * nz;
    double* R2 = V + 2 * NVAR * nz;
    double U0[NVAR];
    if constexpr (STAGE == 1) prim_to_flux(p, f, m, g.gam, 0, U0);
#pragma unroll
    for (int v = 0; v < NVAR; v++) {
      const double dtl = dt * L[v];
      const long o = v * nz + c;
      if constexpr (STAGE == 1) {
        U[v] = U0[v] + SSP54_C1 * dtl;
        R0[o] = U0[v];
        R1[o] = SSP54_A2 * U0[v] + SSP54_B2 * U[v];
      } else if constexpr (STAGE == 2) {
        U[v] = R1[o] + SSP54_C2 * dtl;
        R1[o] = SSP54_A3 * R0[o] + SSP54_B3 * U[v];
        R2[o] = SSP54_D2 * U[v];
      } else if constexpr (STAGE == 3) {
        U[v] = R1[o] + SSP54_C3 * dtl;
        R1[o] = SSP54_A4 * R0[o] + SSP54_B4 * U[v];
        R2[o] = R2[o] + SSP54_D3 * U[v];
      } else if constexpr (STAGE == 4) {
        U[v] = R1[o] + SSP54_C4 * dtl;
        R2[o] = (R2[o] + SSP54_E3 * dtl) + SSP54_D4 * U[v];
      } else {
        U[v] = R2[o] + SSP54_E4 * dtl;
      }
    }
  } else if (STAGE == 1) {
    double U0[NVAR];
    prim_to_flux(p, f, m, g.gam, 0, U0);
    const double h = INTEG == GRMHD_INTEG_PC ? 0.5 * dt : dt;
#pragma unroll
    for (int v = 0; v < NVAR; v++) {
      U[v] = U0[v] + h * L[v];
      if (INTEG == GRMHD_INTEG_SSPRK2) V[v * nz + c] = 0.5 * (U0[v] + U[v]);
      if (INTEG == GRMHD_INTEG_PC) V[v * nz + c] = U0[v];
    }
  } else {
#pragma unroll
    for (int v = 0; v < NVAR; v++)
      U[v] = INTEG == GRMHD_INTEG_PC ? V[v * nz + c] + dt * L[v] : V[v * nz + c] + 0.5 * (dt * L[v]);
  }
  if constexpr (FACE) {  // face-centred CT: the zone's field is the mean of its new faces
    U[B1] = 0.5 * (ph1[c] + ph1[c + si]);
    U[B2] = 0.5 * (ph2[c] + ph2[c + sj]);
    U[B3] = 0.5 * (ph3[c] + ph3[c + sk]);
  }
  if constexpr (MODE == U_STORE) {  // the implicit solver recovers the prims in its own pass
#pragma unroll
    for (int v = 0; v < NVAR; v++) ustar[v * nz + c] = U[v];
    return;
  }
  double out[NVAR];
  int bad = invert(g, m, U, p, out);
#pragma unroll
  for (int v = 0; v < NVAR; v++) Pout[v * nz + c] = out[v];
  if (flags) flags[c] = (unsigned char)bad;
  if (MODE == U_PROVISIONAL) {
    mark[c] = (unsigned char)bad;
    if (bad) atomicAdd(&fails[C_MARKS], 1ull);
  } else if (bad) {
    atomicAdd(&fails[C_FAILS], 1ull);
  }
  if (RATE) *rate = zone_rate(g, out, m);
}

// One stage over the interior.  With RATE (stage 2) every workgroup also
// writes the maximum CFL rate of the prims it produced to rate_partial[], so
// the next step's dt needs only the final pass over the partials.
// fails is the context's counter array (C_* slots).  The FINAL pass of the
// flux correction runs only when the PROVISIONAL pass marked a zone (a
// grid-uniform test of the mark count), and then adds that count to the
// correction's running total.
template <int STAGE, typename FT, bool RATE, int MODE, bool FACE, int INTEG = GRMHD_INTEG_SSPRK2>
__global__ void __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(RATE ? UPDATE_WAVES_RATE : UPDATE_WAVES, 8)))
k_update(Dev g, Sched box, const double* __restrict__ Pin, double* __restrict__ Pout,
         double* __restrict__ V, const FT* __restrict__ F1, const FT* __restrict__ F2,
         const FT* __restrict__ F3, const FT* __restrict__ E1, const FT* __restrict__ E2,
         const FT* __restrict__ E3, const double* __restrict__ tabC, const double* __restrict__ dgs,
         double dt, const double* __restrict__ dt_dev, unsigned long long* fails,
         unsigned char* __restrict__ flags, double* __restrict__ rate_partial,
         unsigned char* __restrict__ mark, const double* __restrict__ ph1,
         const double* __restrict__ ph2, const double* __restrict__ ph3, double* __restrict__ ustar) {
  if (MODE == U_FINAL) {
    const unsigned long long nmark = fails[C_MARKS];
    if (nmark == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&fails[C_FOFC], nmark);
  }
  int i, j, k;
  const bool in = sched_index(box, blockIdx.x, gridDim.x, i, j, k);
  if (dt_dev) dt = *dt_dev;
  if (!RATE) {
    if (in)
      update_zone<STAGE, FT, false, MODE, FACE, INTEG>(g, Pin, Pout, V, F1, F2, F3, E1, E2, E3, tabC, dgs,
                                                       dt, fails, flags, i, j, k, nullptr, mark, ph1, ph2,
                                                       ph3, ustar);
    return;
  }
  double r = 0.0, sm = 0.0;
  if (in)
    update_zone<STAGE, FT, true, MODE, FACE, INTEG>(g, Pin, Pout, V, F1, F2, F3, E1, E2, E3, tabC, dgs, dt,
                                                    fails, flags, i, j, k, &r, mark, ph1, ph2, ph3, ustar);
  block_reduce(r, sm);
  if (threadIdx.x == 0) rate_partial[blockIdx.x] = r;
}

// Floors over the prims one update pass wrote (Pout), zone by zone as the
// update left them: where they act, the new prims are stored and, in stage
// 1, the stage register V gets the floored state's conserved variables
// (recomputed from the stage input Pin).  PROVISIONAL marks the zones floors
// act on (counting each newly marked zone), PLAIN and FINAL count floor
// activations; FINAL runs only when the provisional passes marked a zone.
// With RATE the CFL-rate partials of the final prims are written here (the
// update then writes none), over the update's schedule.
template <int STAGE, bool RATE, int MODE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3, 8))) k_floors(Dev g, Sched box, const double* __restrict__ Pin,
                                                  double* __restrict__ Pout, double* __restrict__ V,
                                                  const double* __restrict__ tabC,
                                                  unsigned long long* fails, unsigned char* __restrict__ mark,
                                                  double* __restrict__ rate_partial) {
#pragma clang fp contract(off)
  if (MODE == U_FINAL && fails[C_MARKS] == 0) return;
  int i, j, k;
  const bool in = sched_index(box, blockIdx.x, gridDim.x, i, j, k);
  double r = 0.0;
  if (in) {
    const long c = zid(g, i, j, k), nz = g.nz;
    double out[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; v++) out[v] = Pout[v * nz + c];
    PointMetric<double> m;
    load_metric<double>(tabC, g.plane, pid(g, i, j), m);
    const int fl = apply_floors(g, m, g.x1min + (i + 0.5) * g.dx1, out);
    if (fl) {
#pragma unroll
      for (int v = 0; v < NVAR; v++) Pout[v * nz + c] = out[v];
      if (STAGE == 1) {
        double p[NVAR], U0[NVAR], U1[NVAR];
#pragma unroll
        for (int v = 0; v < NVAR; v++) p[v] = Pin[v * nz + c];
        Fluid<double> f0, f1;
        fluid_state(p, m, f0);
        prim_to_flux(p, f0, m, g.gam, 0, U0);
        fluid_state(out, m, f1);
        prim_to_flux(out, f1, m, g.gam, 0, U1);
#pragma unroll
        for (int v = 0; v < NVAR; v++) V[v * nz + c] = 0.5 * (U0[v] + U1[v]);
      }
      if (MODE == U_PROVISIONAL) {
        if (mark[c] == 0) {
          mark[c] = 1;
          atomicAdd(&fails[C_MARKS], 1ull);
        }
      } else {
        atomicAdd(&fails[C_FLOORS], 1ull);
        if (fl & FL_FLUID_FRAME) atomicAdd(&fails[C_FLUID], 1ull);
      }
    }
    if (RATE) r = zone_rate(g, out, m);
  }
  if (RATE) {
    double sm = 0.0;
    block_reduce(r, sm);
    if (threadIdx.x == 0) rate_partial[blockIdx.x] = r;
  }
}

// The implicit solver's pass: per zone, the prims whose conserved variables
// are the U* the update stored, from the stage input as the guess (the
// update's inversion, for the implicit recovery).  Failures counted and
// flagged as the update counts them; with RATE the CFL-rate partials of the
// new prims, over the update's schedule.  The 5 x 5 Newton system of each
// thread lives in LDS (25 doubles per thread, 51 KB per workgroup).
template <bool RATE>
__global__ void __launch_bounds__(BLOCK)
k_implicit(Dev g, Sched box, const double* __restrict__ Pin, const double* __restrict__ ustar,
           double* __restrict__ Pout, const double* __restrict__ tabC, unsigned long long* fails,
           unsigned char* __restrict__ flags, double* __restrict__ rate_partial) {
  __shared__ double jac[25 * BLOCK];
  int i, j, k;
  const bool in = sched_index(box, blockIdx.x, gridDim.x, i, j, k);
  double r = 0.0;
  if (in) {
    const long c = zid(g, i, j, k), nz = g.nz;
    double U[NVAR], p[NVAR], out[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; v++) {
      U[v] = ustar[v * nz + c];
      p[v] = Pin[v * nz + c];
    }
    PointMetric<double> m;
    load_metric<double>(tabC, g.plane, pid(g, i, j), m);
    const int bad = invert_implicit(g, m, U, p, out, jac + threadIdx.x);
#pragma unroll
    for (int v = 0; v < NVAR; v++) Pout[v * nz + c] = out[v];
    if (flags) flags[c] = (unsigned char)bad;
    if (bad) atomicAdd(&fails[C_FAILS], 1ull);
    if (RATE) r = zone_rate(g, out, m);
  }
  if (RATE) {
    double sm = 0.0;
    block_reduce(r, sm);
    if (threadIdx.x == 0) rate_partial[blockIdx.x] = r;
  }
}

// ------------------------------------------------------- reductions etc. --

// Per zone sum_d max(|c+|, |c-|)/dx_d over axes with more than one zone;
// workgroup maxima to partial[].  Grid-stride over the box, so any grid size
// reduces through at most MAX_PARTIALS partials.
__global__ void __launch_bounds__(BLOCK) k_dt_partial(Dev g, Box box, const double* __restrict__ P,
                                                      const double* __restrict__ tabC,
                                                      double* partial) {
  double s = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < box.count(); t += stride) {
    int i, j, k;
    box_index(box, t, i, j, k);
    long c = zid(g, i, j, k);
    double p[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; v++) p[v] = P[v * g.nz + c];
    PointMetric<double> m;
    load_metric<double>(tabC, g.plane, pid(g, i, j), m);
    s = fmax(s, zone_rate(g, p, m));
  }
  double sm = 0.0;
  block_reduce(s, sm);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Face divergence sum_d (phi_d(+) - phi_d(-))/dx_d over interior zones;
// workgroup max and sum of its magnitude (grid-stride).
__global__ void __launch_bounds__(BLOCK) k_face_divb_partial(Dev g, Box box, const double* __restrict__ ph1,
                                                             const double* __restrict__ ph2,
                                                             const double* __restrict__ ph3, double* pmax,
                                                             double* psum) {
  double mx = 0.0, sm = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < box.count(); t += stride) {
    int i, j, k;
    box_index(box, t, i, j, k);
    const long c = zid(g, i, j, k);
    const double dv = ((ph1[c + 1] - ph1[c]) / g.dx1 + (ph2[c + g.s1] - ph2[c]) / g.dx2) +
                      (ph3[c + g.plane] - ph3[c]) / g.dx3;
    mx = fmax(mx, fabs(dv));
    sm += fabs(dv);
  }
  block_reduce(mx, sm);
  if (threadIdx.x == 0) {
    pmax[blockIdx.x] = mx;
    psum[blockIdx.x] = sm;
  }
}

// Corner-centred div B (conserved field sqrt(-g) B^d, four zones per side)
// over the corner box; block max and sum of |div|/sqrt(-g)_corner.
__global__ void __launch_bounds__(BLOCK) k_divb_partial(Dev g, Box box, const double* __restrict__ P,
                                                        const double* __restrict__ tabC,
                                                        const double* __restrict__ corner,
                                                        double* field, double* pmax, double* psum) {
  double mx = 0.0, sm = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < box.count(); t += stride) {
    int i, j, k;
    box_index(box, t, i, j, k);
    const long nz = g.nz;
    auto ub = [&](int d, int a, int b, int cc) {
      return tabC[G_DET * g.plane + pid(g, a, b)] * P[(B1 + d) * nz + zid(g, a, b, cc)];
    };
    double d1 = (ub(0, i, j, k) + ub(0, i, j - 1, k) + ub(0, i, j, k - 1) + ub(0, i, j - 1, k - 1)) -
                (ub(0, i - 1, j, k) + ub(0, i - 1, j - 1, k) + ub(0, i - 1, j, k - 1) +
                 ub(0, i - 1, j - 1, k - 1));
    double d2 = (ub(1, i, j, k) + ub(1, i - 1, j, k) + ub(1, i, j, k - 1) + ub(1, i - 1, j, k - 1)) -
                (ub(1, i, j - 1, k) + ub(1, i - 1, j - 1, k) + ub(1, i, j - 1, k - 1) +
                 ub(1, i - 1, j - 1, k - 1));
    double d3 = (ub(2, i, j, k) + ub(2, i - 1, j, k) + ub(2, i, j - 1, k) + ub(2, i - 1, j - 1, k)) -
                (ub(2, i, j, k - 1) + ub(2, i - 1, j, k - 1) + ub(2, i, j - 1, k - 1) +
                 ub(2, i - 1, j - 1, k - 1));
    double dv = d1 / (4.0 * g.dx1) + d2 / (4.0 * g.dx2) + d3 / (4.0 * g.dx3);
    const double val = fabs(dv) / corner[pid(g, i, j)];
    if (field) field[zid(g, i, j, k)] = val;
    mx = fmax(mx, val);
    sm += val;
  }
  block_reduce(mx, sm);
  if (threadIdx.x == 0) {
    pmax[blockIdx.x] = mx;
    psum[blockIdx.x] = sm;
  }
}

// Single-block final pass over n partials: out[0] = max, out[1] = sum.  With
// cfl > 0 (the dt reduction) also out[2] = cfl / max, the step the update
// kernels can read on the device, and out[3] = 0 when that dt is usable, 1
// when the maximum rate is not positive and finite (out[2] is then 0, so a
// step taken with it leaves the state unchanged).
__global__ void __launch_bounds__(BLOCK) k_reduce_final(const double* pmax, const double* psum,
                                                        int n, double* out, double cfl) {
  // eight independent accumulators per thread, so that its loads are in
  // flight together instead of each waiting for the previous one
  constexpr int U = 8;
  double m[U], a[U];
#pragma unroll
  for (int u = 0; u < U; u++) m[u] = a[u] = 0.0;
  int q = threadIdx.x;
  for (; q + (U - 1) * BLOCK < n; q += U * BLOCK) {
#pragma unroll
    for (int u = 0; u < U; u++) m[u] = fmax(m[u], pmax[q + u * BLOCK]);
    if (psum) {
#pragma unroll
      for (int u = 0; u < U; u++) a[u] += psum[q + u * BLOCK];
    }
  }
  for (; q < n; q += BLOCK) {
    m[0] = fmax(m[0], pmax[q]);
    if (psum) a[0] += psum[q];
  }
  double mx = m[0], sm = a[0];
#pragma unroll
  for (int u = 1; u < U; u++) {
    mx = fmax(mx, m[u]);
    sm += a[u];
  }
  block_reduce(mx, sm);
  if (threadIdx.x == 0) {
    out[0] = mx;
    out[1] = sm;
    if (cfl > 0.0) {
      const bool ok = mx > 0.0 && isfinite(mx);
      out[2] = ok ? cfl / mx : 0.0;
      out[3] = ok ? 0.0 : 1.0;
    }
  }
}

__global__ void __launch_bounds__(BLOCK) k_prims_to_cons(Dev g, Box box, const double* __restrict__ P,
                                                         double* __restrict__ U,
                                                         const double* __restrict__ tabC) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (!box_index(box, t, i, j, k)) return;
  long c = zid(g, i, j, k);
  double p[NVAR], u[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) p[v] = P[v * g.nz + c];
  PointMetric<double> m;
  load_metric<double>(tabC, g.plane, pid(g, i, j), m);
  Fluid<double> f;
  fluid_state(p, m, f);
  prim_to_flux(p, f, m, g.gam, 0, u);
#pragma unroll
  for (int v = 0; v < NVAR; v++) U[v * g.nz + c] = u[v];
}

__global__ void __launch_bounds__(BLOCK) k_cons_to_prims(Dev g, Box box, const double* __restrict__ U,
                                                         const double* __restrict__ G,
                                                         double* __restrict__ P, int* flags,
                                                         const double* __restrict__ tabC,
                                                         unsigned long long* fails) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int i, j, k;
  if (!box_index(box, t, i, j, k)) return;
  long c = zid(g, i, j, k);
  double u[NVAR], gs[NVAR], p[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; v++) {
    u[v] = U[v * g.nz + c];
    gs[v] = G[v * g.nz + c];
  }
  PointMetric<double> m;
  load_metric<double>(tabC, g.plane, pid(g, i, j), m);
  __shared__ double jac[25 * BLOCK];
  int bad = g.inverter == GRMHD_INV_IMPLICIT ? invert_implicit(g, m, u, gs, p, jac + threadIdx.x)
                                             : invert(g, m, u, gs, p);
#pragma unroll
  for (int v = 0; v < NVAR; v++) P[v * g.nz + c] = p[v];
  if (flags) flags[c] = bad;
  if (bad) atomicAdd(fails, 1ull);
}

#include "adjoint.hpp"
#include "pack.hpp"
#include "emhd.hpp"

}  // namespace

// ------------------------------------------------------------- host side --

struct grmhd_ctx {
  grmhd_grid grid;
  grmhd_metric metric;
  grmhd_params params;
  hipStream_t stream;
  Dev dev;
  // workspace carve (device)
  double *P, *P1, *V;
  void *F[3], *E[3];
  double *tabC, *tabF1, *tabF2, *corner, *conn, *dgs;
  double *pmax, *psum, *result;
  unsigned long long* fails;  // counters, slots C_* (failures, floors, flux-correction marks, ...)
  unsigned char* mark;        // per zone: marked by the flux correction's provisional pass
  // face-centred CT: face fields of the state, of stage 1 and the stage
  // register; zone-centre EMFs (stored type) of the upwinded scheme
  double *phi[3] = {nullptr, nullptr, nullptr}, *phi1[3] = {nullptr, nullptr, nullptr},
         *phiV[3] = {nullptr, nullptr, nullptr};
  void* Ec[4] = {nullptr, nullptr, nullptr, nullptr};  // EMFs, then the mass-current scale
  bool faces_loaded = false;
  double* ustar = nullptr;    // implicit recovery: the stage's target conserved variables
  // Extended GRMHD: extra variables of the state and of stage 1, their fluxes,
  // U^n of them, their stage targets, u^t of the step's state and the
  // spatial part of div u
  double *X = nullptr, *X1 = nullptr, *FX[3] = {nullptr, nullptr, nullptr}, *VX = nullptr,
         *xrhs = nullptr, *utn = nullptr, *divu = nullptr;
  double* pdt;              // CFL-rate partials left by the last stage-2 update
  bool rate_ready = false;  // pdt describes the current state (rate_n partials)
  bool ghosts_valid = false;  // the ghost zones of P hold the boundary conditions of its interior
  int rate_n = 0;
  // x3 planes per chunk run of the flux/EMF and update schedules
  int kg_flux = 8, kg_update = 8;
  // optional per-kernel-class timing with HIP events on the context's stream
  unsigned timing = 0;  // bit c set: launches of class c carry timing events
  struct Mark { hipEvent_t a, b; int cls; };
  Mark* marks = nullptr;
  int nmarks = 0, capmarks = 0;
};

namespace {

struct Carve {
  size_t off = 0;
  template <typename T>
  T* take(char* base, size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

bool grid_ok(const grmhd_grid* g, const grmhd_params* p) {
  if (!g || !p) return false;
  if (g->ng != NG || g->n1 < 1 || g->n2 < 1 || g->n3 < 1) return false;
  // padded zone indices (and the flux kernels' zone counters) fit in 31 bits
  if ((long)(g->n1 + 2 * NG) * (g->n2 + 2 * NG) * (g->n3 + 2 * NG) > (1L << 31) - 4096) return false;
  for (int a = 0; a < 6; a++)
    if (g->bc[a] < GRMHD_BC_PERIODIC || g->bc[a] > GRMHD_BC_FROZEN) return false;
  int n[3] = {g->n1, g->n2, g->n3};
  for (int a = 0; a < 3; a++) {
    bool per = g->bc[2 * a] == GRMHD_BC_PERIODIC || g->bc[2 * a + 1] == GRMHD_BC_PERIODIC;
    if (per && g->bc[2 * a] != g->bc[2 * a + 1]) return false;
    if ((g->bc[2 * a] == GRMHD_BC_POLAR || g->bc[2 * a + 1] == GRMHD_BC_POLAR) && (a != 1 || n[a] < NG))
      return false;
    if ((g->bc[2 * a] == GRMHD_BC_OUTFLOW || g->bc[2 * a + 1] == GRMHD_BC_OUTFLOW) && n[a] < 1)
      return false;
  }
  if (!(g->x1max > g->x1min && g->x2max > g->x2min && g->x3max > g->x3min)) return false;
  if (p->recon < GRMHD_RECON_MC || p->recon > GRMHD_RECON_PPMX) return false;
  // the WENO weights' products stay normal in FP64 and the FP32 indicators
  // stay positive for eps >= 1e-36
  if ((p->recon == GRMHD_RECON_WENO5 || p->recon == GRMHD_RECON_WENOZ) &&
      !(p->weno_eps >= 1e-36 && p->weno_eps <= 1.0))
    return false;
  if (p->precision != GRMHD_PREC_FP64 && p->precision != GRMHD_PREC_MIXED) return false;
  if (!(p->gamma_ad > 1.0) || p->newton_maxit < 1 || !(p->newton_tol > 0.0)) return false;
  if ((p->floors != 0 && p->floors != 1) || (p->fofc != 0 && p->fofc != 1)) return false;
  if (p->ct != GRMHD_CT_FLUX && p->ct != GRMHD_CT_FACE_AVG && p->ct != GRMHD_CT_FACE_GS) return false;
  if (p->floors && !(p->rho_min_geom > 0.0 && p->u_min_geom > 0.0 && p->bsq_over_rho_max > 0.0 &&
                     p->bsq_over_u_max > 0.0 && p->u_over_rho_max > 0.0 && p->gamma_max > 1.0))
    return false;
  if (p->inverter != GRMHD_INV_1DW && p->inverter != GRMHD_INV_KASTAUN && p->inverter != GRMHD_INV_IMPLICIT)
    return false;
  // the implicit recovery runs in a pass of its own, without the correction's marks
  if (p->inverter == GRMHD_INV_IMPLICIT && p->fofc) return false;
  if (p->inverter == GRMHD_INV_KASTAUN && !(p->kastaun_wmax > 1.0)) return false;
  // the other integrators take the plain Flux-CT step
  if (p->integrator < GRMHD_INTEG_SSPRK2 || p->integrator > GRMHD_INTEG_SSPRK54) return false;
  if (p->integrator != GRMHD_INTEG_SSPRK2 &&
      (p->floors || p->fofc || p->ct != GRMHD_CT_FLUX || p->inverter == GRMHD_INV_IMPLICIT))
    return false;
  // Extended GRMHD: the semi-implicit predictor-corrector of the plain FP64
  // Flux-CT step with MC or WENO5
  if (p->egrmhd != 0 && p->egrmhd != 1) return false;
  if (p->egrmhd &&
      (p->integrator != GRMHD_INTEG_PC || p->precision != GRMHD_PREC_FP64 ||
       (p->recon != GRMHD_RECON_MC && p->recon != GRMHD_RECON_WENO5) || !(p->tau_r > 0.0) ||
       !(p->chi_emhd >= 0.0) || !(p->nu_emhd >= 0.0) || !isfinite(p->tau_r) || !isfinite(p->chi_emhd) ||
       !isfinite(p->nu_emhd)))
    return false;
  return true;
}

size_t carve(grmhd_ctx* c, char* base, const grmhd_grid* g, const grmhd_params* prm) {
  const int ct = prm->ct, inverter = prm->inverter;
  const bool emhd = prm->egrmhd != 0;
  long nz = (long)(g->n1 + 2 * NG) * (g->n2 + 2 * NG) * (g->n3 + 2 * NG);
  long plane = (long)(g->n1 + 2 * NG) * (g->n2 + 2 * NG);
  Carve cv;
  double *P = cv.take<double>(base, NVAR * nz), *P1 = cv.take<double>(base, NVAR * nz);
  // the stage registers: one (SSPRK2, predictor-corrector), three (SSPRK(5,4))
  double* V = cv.take<double>(base, (prm->integrator == GRMHD_INTEG_SSPRK54 ? 3 : 1) * NVAR * nz);
  double* F[3];
  double* E[3];
  for (int d = 0; d < 3; d++) F[d] = cv.take<double>(base, NVAR * nz);
  for (int d = 0; d < 3; d++) E[d] = cv.take<double>(base, nz);
  double* tabC = cv.take<double>(base, G_NF * plane);
  double* tabF1 = cv.take<double>(base, G_NF * plane);
  double* tabF2 = cv.take<double>(base, G_NF * plane);
  double* corner = cv.take<double>(base, plane);
  double* conn = cv.take<double>(base, NCONN * plane);
  double* dgs = cv.take<double>(base, NDG * plane);
  double* pmax = cv.take<double>(base, MAX_PARTIALS);
  double* psum = cv.take<double>(base, MAX_PARTIALS);
  double* result = cv.take<double>(base, 8);
  double* pdt = cv.take<double>(base, MAX_PARTIALS);
  unsigned long long* fails = cv.take<unsigned long long>(base, 8);
  unsigned char* mark = cv.take<unsigned char>(base, nz);
  double *phi[3] = {}, *phi1[3] = {}, *phiV[3] = {}, *Ec[4] = {};
  if (ct != GRMHD_CT_FLUX) {
    for (int d = 0; d < 3; d++) {
      phi[d] = cv.take<double>(base, nz);
      phi1[d] = cv.take<double>(base, nz);
      phiV[d] = cv.take<double>(base, nz);
      Ec[d] = cv.take<double>(base, nz);
    }
    Ec[3] = cv.take<double>(base, nz);
  }
  double* ustar = inverter == GRMHD_INV_IMPLICIT || emhd ? cv.take<double>(base, NVAR * nz) : nullptr;
  double *X = nullptr, *X1 = nullptr, *FX[3] = {}, *VX = nullptr, *xrhs = nullptr, *utn = nullptr,
         *divu = nullptr;
  if (emhd) {
    X = cv.take<double>(base, 2 * nz);
    X1 = cv.take<double>(base, 2 * nz);
    for (int d = 0; d < 3; d++) FX[d] = cv.take<double>(base, 2 * nz);
    VX = cv.take<double>(base, 2 * nz);
    xrhs = cv.take<double>(base, 2 * nz);
    utn = cv.take<double>(base, nz);
    divu = cv.take<double>(base, nz);
  }
  if (c) {
    c->mark = mark;
    c->ustar = ustar;
    c->X = X;
    c->X1 = X1;
    for (int d = 0; d < 3; d++) c->FX[d] = FX[d];
    c->VX = VX;
    c->xrhs = xrhs;
    c->utn = utn;
    c->divu = divu;
    for (int d = 0; d < 3; d++) {
      c->phi[d] = phi[d];
      c->phi1[d] = phi1[d];
      c->phiV[d] = phiV[d];
      c->Ec[d] = Ec[d];
    }
    c->Ec[3] = Ec[3];
    c->P = P; c->P1 = P1; c->V = V;
    for (int d = 0; d < 3; d++) { c->F[d] = F[d]; c->E[d] = E[d]; }
    c->tabC = tabC; c->tabF1 = tabF1; c->tabF2 = tabF2; c->corner = corner; c->conn = conn;
    c->dgs = dgs;
    c->pmax = pmax; c->psum = psum; c->result = result; c->fails = fails; c->pdt = pdt;
  }
  return cv.off;
}

int hip_check() { return hipGetLastError() == hipSuccess ? GRMHD_OK : GRMHD_E_HIP; }

enum { T_BC = 0, T_FLUX, T_EMF, T_UPDATE1, T_UPDATE2, T_DT, T_FOFC, T_FLOORS, T_FACES, T_NCLASS };

// Start/stop events of one launch of class cls while timing is enabled (null
// events otherwise, or when no more events can be created).
struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
};
EvPair timing_events(grmhd_ctx* c, int cls) {
  EvPair e;
  if (!((c->timing >> cls) & 1u)) return e;
  if (c->nmarks == c->capmarks) {
    int cap = c->capmarks ? 2 * c->capmarks : 256;
    auto* m = (grmhd_ctx::Mark*)realloc(c->marks, sizeof(grmhd_ctx::Mark) * cap);
    if (!m) return e;
    c->marks = m;
    for (int q = c->capmarks; q < cap; q++) {
      if (hipEventCreate(&m[q].a) != hipSuccess || hipEventCreate(&m[q].b) != hipSuccess) {
        c->timing = 0;  // no events: stop timing rather than fail the step
        return e;
      }
      c->capmarks = q + 1;
    }
  }
  const int slot = c->nmarks++;
  c->marks[slot].cls = cls;
  e.a = c->marks[slot].a;
  e.b = c->marks[slot].b;
  return e;
}

// Launch a kernel of class cls on the context's stream.  While timing, the
// start and stop events travel with the dispatch itself (hipExtLaunchKernel),
// so timing adds no marker packets between kernels.
template <typename F, typename... Args>
int launch(grmhd_ctx* c, int cls, F kernel, unsigned nblocks, Args... args) {
  EvPair e = timing_events(c, cls);
  hipExtLaunchKernelGGL(kernel, dim3(nblocks), dim3(BLOCK), 0, c->stream, e.a, e.b, 0, args...);
  return hip_check();
}

// Ghost zones of prims P and, with face-centred CT, ghost faces of the face
// fields ph (the state's or stage 1's).
int fill_ghosts(grmhd_ctx* c, double* P, double* const* ph = nullptr) {
  if (ph && ph[0]) {
    int rc = launch(c, T_BC, k_bc_faces, blocks_for(3 * c->dev.nz), c->dev, ph[0], ph[1], ph[2]);
    if (rc) return rc;
  }
  return launch(c, T_BC, k_bc, blocks_for(ghost_count(c->dev)), c->dev, P);
}

// Ghost zones (and faces) of the state, filled unless they already hold its
// boundary conditions (filled since the state last changed).
int ensure_ghosts(grmhd_ctx* c) {
  if (c->ghosts_valid) return GRMHD_OK;
  int rc = fill_ghosts(c, c->P, c->phi);
  if (rc == GRMHD_OK) c->ghosts_valid = true;
  return rc;
}

// Interior zones' B prims of the state from its face fields.
int cell_b_from_faces(grmhd_ctx* c) {
  const Dev& g = c->dev;
  Box bz = make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1);
  k_cell_b<<<blocks_for(bz.count()), BLOCK, 0, c->stream>>>(g, bz, c->phi[0], c->phi[1], c->phi[2], c->tabC,
                                                             c->P);
  return hip_check();
}

inline unsigned round8(unsigned n) { return (n + 7u) & ~7u; }

// Flux and EMF kernels of one stage, reading the (ghost-filled) prims P.
// Edge EMFs of the stage from the fluxes: the Flux-CT average (also the
// averaged face-centred scheme), or the upwinded scheme from the zone-centre
// EMFs (computed once per stage, from P).  gate/zero as in k_emf.
template <typename FT>
int stage_emfs(grmhd_ctx* c, const unsigned long long* gate, unsigned long long* zero) {
  const Dev& g = c->dev;
  Sched be = make_sched(make_box(0, g.n1, 0, g.n2, 0, g.n3), c->kg_flux);
  if (c->params.ct == GRMHD_CT_FACE_GS)
    return launch(c, T_EMF, k_emf_gs<FT>, blocks_for(be), g, be, (const FT*)c->F[0], (const FT*)c->F[1],
                  (const FT*)c->F[2], (const FT*)c->Ec[0], (const FT*)c->Ec[1], (const FT*)c->Ec[2],
                  (const FT*)c->Ec[3], (FT*)c->E[0], (FT*)c->E[1], (FT*)c->E[2], gate, zero);
  return launch(c, T_EMF, k_emf<FT>, blocks_for(be), g, be, (const FT*)c->F[0], (const FT*)c->F[1],
                (const FT*)c->F[2], (FT*)c->E[0], (FT*)c->E[1], (FT*)c->E[2], gate, zero);
}

template <typename R, typename FT>
int stage_fluxes(grmhd_ctx* c, const double* P, unsigned long long* zero = nullptr,
                 double* const* ph = nullptr) {
  const Dev& g = c->dev;
  FT* F1 = (FT*)c->F[0];
  FT* F2 = (FT*)c->F[1];
  FT* F3 = (FT*)c->F[2];
  Sched b1 = make_sched(make_box(0, g.n1, -1, g.n2, -1, g.n3), c->kg_flux);
  Sched b2 = make_sched(make_box(-1, g.n1, 0, g.n2, -1, g.n3), c->kg_flux);
  Sched b3 = make_sched(make_box(-1, g.n1, -1, g.n2, 0, g.n3), c->kg_flux);
  const bool shared = c->params.recon == GRMHD_RECON_MC || c->params.recon == GRMHD_RECON_WENO5;
  const unsigned n1 = shared ? x1_sweep_blocks((long)(g.n1 + 2) * (g.n2 + 2) * (g.n3 + 2))
                             : round8(blocks_for(b1));
  const bool tiled = c->params.recon == GRMHD_RECON_WENO5 && FLUX_TILE;
  const unsigned n2 = tiled ? tile_blocks(g, 2) : round8(blocks_for(b2));
  const unsigned n3 = tiled ? tile_blocks(g, 3) : blocks_for(b3);
  const double* Pc = P;
  const double* p1 = ph ? ph[0] : nullptr;
  const double* p2 = ph ? ph[1] : nullptr;
  const double* p3 = ph ? ph[2] : nullptr;
  auto go = [&](auto kernel) {
    return launch(c, T_FLUX, kernel, n1 + n2 + n3, g, b1, b2, b3, n1, n2, n3, Pc, (const double*)c->tabF1,
                  (const double*)c->tabF2, (const double*)c->tabC, F1, F2, F3, p1, p2, p3);
  };
  int rc;
  const bool face = ph != nullptr;
  if (c->params.recon == GRMHD_RECON_MC)
    rc = face ? go(k_flux_all<GRMHD_RECON_MC, R, FT, true>) : go(k_flux_all<GRMHD_RECON_MC, R, FT, false>);
  else if (c->params.recon == GRMHD_RECON_DONOR)
    rc = face ? go(k_flux_all<GRMHD_RECON_DONOR, R, FT, true>) : go(k_flux_all<GRMHD_RECON_DONOR, R, FT, false>);
  else if (c->params.recon == GRMHD_RECON_VL)
    rc = face ? go(k_flux_all<GRMHD_RECON_VL, R, FT, true>) : go(k_flux_all<GRMHD_RECON_VL, R, FT, false>);
  else if (c->params.recon == GRMHD_RECON_WENOZ)
    rc = face ? go(k_flux_all<GRMHD_RECON_WENOZ, R, FT, true>) : go(k_flux_all<GRMHD_RECON_WENOZ, R, FT, false>);
  else if (c->params.recon == GRMHD_RECON_MP5)
    rc = face ? go(k_flux_all<GRMHD_RECON_MP5, R, FT, true>) : go(k_flux_all<GRMHD_RECON_MP5, R, FT, false>);
  else if (c->params.recon == GRMHD_RECON_PPM)
    rc = face ? go(k_flux_all<GRMHD_RECON_PPM, R, FT, true>) : go(k_flux_all<GRMHD_RECON_PPM, R, FT, false>);
  else if (c->params.recon == GRMHD_RECON_PPMX)
    rc = face ? go(k_flux_all<GRMHD_RECON_PPMX, R, FT, true>) : go(k_flux_all<GRMHD_RECON_PPMX, R, FT, false>);
  else
    rc = face ? go(k_flux_all<GRMHD_RECON_WENO5, R, FT, true>) : go(k_flux_all<GRMHD_RECON_WENO5, R, FT, false>);
  if (rc) return rc;
  if (c->params.ct == GRMHD_CT_FACE_GS) {
    Box bc = make_box(-1, g.n1, -1, g.n2, -1, g.n3);
    if ((rc = launch(c, T_EMF, k_cell_emf<R, FT>, blocks_for(bc.count()), g, bc, Pc, (const double*)c->tabC,
                     (FT*)c->Ec[0], (FT*)c->Ec[1], (FT*)c->Ec[2], (FT*)c->Ec[3])))
      return rc;
  }
  return stage_emfs<FT>(c, (const unsigned long long*)nullptr, zero);
}

// Face fields of one stage from the edge EMFs: stage 1 phi1 = phi + dt R (and
// the register phiV = (phi + phi1)/2), stage 2 phi = phiV + (dt/2) R.
template <int STAGE, typename FT>
int stage_faces(grmhd_ctx* c, double dt, const double* dt_dev, const unsigned long long* gate) {
  const Dev& g = c->dev;
  Box bf = make_box(0, g.n1, 0, g.n2, 0, g.n3);
  double* const* base = STAGE == 1 ? c->phi : c->phiV;
  double* const* out = STAGE == 1 ? c->phi1 : c->phi;
  double* const* reg = STAGE == 1 ? c->phiV : c->phi1;  // unused in stage 2
  return launch(c, T_FACES, k_face_update<STAGE, FT>, blocks_for(bf.count()), g, bf, (const FT*)c->E[0],
                (const FT*)c->E[1], (const FT*)c->E[2], (const double*)base[0], (const double*)base[1],
                (const double*)base[2], out[0], out[1], out[2], reg[0], reg[1], reg[2], dt, dt_dev, gate);
}

// One stage's update.  With rate (stage 2 of a step) the workgroups also
// leave the CFL-rate partials of the prims they write in c->pdt.
template <int STAGE, typename FT, int MODE = U_PLAIN, int INTEG = GRMHD_INTEG_SSPRK2>
int stage_update(grmhd_ctx* c, const double* Pin, double* Pout, double dt,
                 unsigned long long* fails = nullptr, unsigned char* flags = nullptr,
                 const double* dt_dev = nullptr, bool rate = false) {
  const Dev& g = c->dev;
  // face-centred CT: the zones' field from the stage's new faces
  double* const* ph = c->params.ct == GRMHD_CT_FLUX ? nullptr : (STAGE == 1 ? c->phi1 : c->phi);
  const double* p1 = ph ? ph[0] : nullptr;
  const double* p2 = ph ? ph[1] : nullptr;
  const double* p3 = ph ? ph[2] : nullptr;
  Sched bz = make_sched(make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1), c->kg_update);
  const int cls = STAGE == 1 ? T_UPDATE1 : T_UPDATE2;
  const unsigned nb = blocks_for(bz);
  auto go = [&](auto kernel, double* partial) {
    return launch(c, cls, kernel, nb, g, bz, Pin, Pout, c->V, (const FT*)c->F[0], (const FT*)c->F[1],
                  (const FT*)c->F[2], (const FT*)c->E[0], (const FT*)c->E[1], (const FT*)c->E[2],
                  (const double*)c->tabC, (const double*)c->dgs, dt, dt_dev, fails ? fails : c->fails, flags,
                  partial, c->mark, p1, p2, p3, c->ustar);
  };
  if constexpr (INTEG != GRMHD_INTEG_SSPRK2) {  // the plain Flux-CT path only
    if constexpr (INTEG != GRMHD_INTEG_SSPRK54 || STAGE == 5) {  // the stage that ends a step
      if (rate && nb <= (unsigned)MAX_PARTIALS) return go(k_update<STAGE, FT, true, MODE, false, INTEG>, c->pdt);
    }
    return go(k_update<STAGE, FT, false, MODE, false, INTEG>, (double*)nullptr);
  } else {
    if constexpr (STAGE == 2) {
      if (rate && nb <= (unsigned)MAX_PARTIALS)
        return ph ? go(k_update<STAGE, FT, true, MODE, true>, c->pdt)
                  : go(k_update<STAGE, FT, true, MODE, false>, c->pdt);
    }
    return ph ? go(k_update<STAGE, FT, false, MODE, true>, (double*)nullptr)
              : go(k_update<STAGE, FT, false, MODE, false>, (double*)nullptr);
  }
}

// The floors pass after an update pass (same schedule as the update, so the
// CFL-rate partials it writes with rate are the ones the dt reduction reads).
template <int STAGE, int MODE>
int stage_floors(grmhd_ctx* c, const double* Pin, double* Pout, bool rate) {
  const Dev& g = c->dev;
  Sched bz = make_sched(make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1), c->kg_update);
  const unsigned nb = blocks_for(bz);
  if (STAGE == 2 && rate && nb <= (unsigned)MAX_PARTIALS)
    return launch(c, T_FLOORS, k_floors<STAGE, true, MODE>, nb, g, bz, Pin, Pout, c->V,
                  (const double*)c->tabC, c->fails, c->mark, c->pdt);
  return launch(c, T_FLOORS, k_floors<STAGE, false, MODE>, nb, g, bz, Pin, Pout, c->V,
                (const double*)c->tabC, c->fails, c->mark, (double*)nullptr);
}

// One SSPRK(5,4) stage from the ghost-filled prims Pin: fluxes, EMFs and
// the update of the plain Flux-CT path.
template <int STAGE, typename R, typename FT>
int stage_ssp54(grmhd_ctx* c, const double* Pin, double* Pout, double dt, const double* dt_dev, bool rate) {
  int rc;
  if ((rc = stage_fluxes<R, FT>(c, Pin, nullptr, nullptr))) return rc;
  return stage_update<STAGE, FT, U_PLAIN, GRMHD_INTEG_SSPRK54>(c, Pin, Pout, dt, nullptr, nullptr, dt_dev,
                                                              rate);
}

// One RK2 stage from the ghost-filled prims Pin: fluxes, EMFs, update, then
// floors when enabled (which then write the CFL-rate partials instead of the
// update).  Under the first-order flux correction: the provisional update
// and floors passes mark zones, the marked zones' faces get donor-cell
// fluxes, and the EMF, update and floors passes run again; these launches
// exit at once when nothing was marked.
template <int STAGE, typename R, typename FT>
int stage(grmhd_ctx* c, const double* Pin, double* Pout, double dt, const double* dt_dev, bool rate) {
  int rc;
  if (c->params.integrator != GRMHD_INTEG_SSPRK2) {  // plain Flux-CT stages (validated at create)
    if ((rc = stage_fluxes<R, FT>(c, Pin, nullptr, nullptr))) return rc;
    if (c->params.integrator == GRMHD_INTEG_PC)
      return stage_update<STAGE, FT, U_PLAIN, GRMHD_INTEG_PC>(c, Pin, Pout, dt, nullptr, nullptr, dt_dev, rate);
    return stage_update<STAGE, FT, U_PLAIN, GRMHD_INTEG_RK1>(c, Pin, Pout, dt, nullptr, nullptr, dt_dev, rate);
  }
  const bool floors = c->params.floors != 0;
  const bool urate = rate && !floors;
  const bool faces = c->params.ct != GRMHD_CT_FLUX;
  double* const* phin = faces ? (STAGE == 1 ? c->phi : c->phi1) : nullptr;
  if (!c->params.fofc) {
    if ((rc = stage_fluxes<R, FT>(c, Pin, nullptr, phin))) return rc;
    if (faces && (rc = stage_faces<STAGE, FT>(c, dt, dt_dev, nullptr))) return rc;
    if (c->params.inverter == GRMHD_INV_IMPLICIT) {
      // the update stores U*, the implicit solver's pass recovers the prims
      if ((rc = stage_update<STAGE, FT, U_STORE>(c, Pin, Pout, dt, nullptr, nullptr, dt_dev, false))) return rc;
      const Dev& g = c->dev;
      Sched bz = make_sched(make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1), c->kg_update);
      const unsigned nb = blocks_for(bz);
      const int cls = STAGE == 1 ? T_UPDATE1 : T_UPDATE2;
      if (STAGE == 2 && urate && nb <= (unsigned)MAX_PARTIALS)
        rc = launch(c, cls, k_implicit<true>, nb, g, bz, Pin, (const double*)c->ustar, Pout,
                    (const double*)c->tabC, c->fails, (unsigned char*)nullptr, c->pdt);
      else
        rc = launch(c, cls, k_implicit<false>, nb, g, bz, Pin, (const double*)c->ustar, Pout,
                    (const double*)c->tabC, c->fails, (unsigned char*)nullptr, (double*)nullptr);
      if (rc) return rc;
      return floors ? stage_floors<STAGE, U_PLAIN>(c, Pin, Pout, rate) : GRMHD_OK;
    }
    if ((rc = stage_update<STAGE, FT, U_PLAIN>(c, Pin, Pout, dt, nullptr, nullptr, dt_dev, urate))) return rc;
    return floors ? stage_floors<STAGE, U_PLAIN>(c, Pin, Pout, rate) : GRMHD_OK;
  }
  unsigned long long* nmark = c->fails + C_MARKS;
  if ((rc = stage_fluxes<R, FT>(c, Pin, nmark, phin))) return rc;
  if (faces && (rc = stage_faces<STAGE, FT>(c, dt, dt_dev, nullptr))) return rc;
  if ((rc = stage_update<STAGE, FT, U_PROVISIONAL>(c, Pin, Pout, dt, nullptr, nullptr, dt_dev, urate)))
    return rc;
  if (floors && (rc = stage_floors<STAGE, U_PROVISIONAL>(c, Pin, Pout, rate))) return rc;
  const Dev& g = c->dev;
  Box b1 = make_box(0, g.n1, -1, g.n2, -1, g.n3), b2 = make_box(-1, g.n1, 0, g.n2, -1, g.n3),
      b3 = make_box(-1, g.n1, -1, g.n2, 0, g.n3);
  FT* F1 = (FT*)c->F[0];
  FT* F2 = (FT*)c->F[1];
  FT* F3 = (FT*)c->F[2];
  if ((rc = launch(c, T_FOFC, k_fofc_flux<R, FT>, blocks_for(b1.count() + b2.count() + b3.count()), g, b1, b2,
                   b3, Pin, (const double*)c->tabF1, (const double*)c->tabF2, (const double*)c->tabC, F1, F2,
                   F3, (const unsigned char*)c->mark, (const unsigned long long*)nmark,
                   (const double*)(phin ? phin[0] : nullptr), (const double*)(phin ? phin[1] : nullptr),
                   (const double*)(phin ? phin[2] : nullptr))))
    return rc;
  if ((rc = stage_emfs<FT>(c, (const unsigned long long*)nmark, (unsigned long long*)nullptr))) return rc;
  if (faces && (rc = stage_faces<STAGE, FT>(c, dt, dt_dev, (const unsigned long long*)nmark))) return rc;
  if ((rc = stage_update<STAGE, FT, U_FINAL>(c, Pin, Pout, dt, nullptr, nullptr, dt_dev, urate))) return rc;
  return floors ? stage_floors<STAGE, U_FINAL>(c, Pin, Pout, rate) : GRMHD_OK;
}

// One Extended GRMHD predictor-corrector stage from the ghost-filled prims
// Pin and extra variables Xin (their ghosts filled here): fluxes of the ten
// variables, the EMFs, the update pass, then the implicit pass, which with
// rate leaves the CFL-rate partials of its prims.
template <int STAGE>
int emhd_stage(grmhd_ctx* c, const double* Pin, double* Xin, double* Pout, double* Xout, double dt,
               const double* dt_dev, bool rate) {
  const Dev& g = c->dev;
  int rc;
  if ((rc = launch(c, T_BC, k_bc_extra, blocks_for(ghost_count(g)), g, Xin))) return rc;
  Sched b1 = make_sched(make_box(0, g.n1, -1, g.n2, -1, g.n3), c->kg_flux);
  Sched b2 = make_sched(make_box(-1, g.n1, 0, g.n2, -1, g.n3), c->kg_flux);
  Sched b3 = make_sched(make_box(-1, g.n1, -1, g.n2, 0, g.n3), c->kg_flux);
  const unsigned n1 = round8(blocks_for(b1)), n2 = round8(blocks_for(b2)), n3 = blocks_for(b3);
  double* F1 = (double*)c->F[0];
  double* F2 = (double*)c->F[1];
  double* F3 = (double*)c->F[2];
  auto flux = [&](auto kernel) {
    return launch(c, T_FLUX, kernel, n1 + n2 + n3, g, b1, b2, b3, n1, n2, n3, Pin, (const double*)Xin,
                  (const double*)c->tabF1, (const double*)c->tabF2, (const double*)c->tabC, F1, F2, F3, c->FX[0],
                  c->FX[1], c->FX[2]);
  };
  rc = c->params.recon == GRMHD_RECON_MC ? flux(k_flux_emhd<GRMHD_RECON_MC>) : flux(k_flux_emhd<GRMHD_RECON_WENO5>);
  if (rc) return rc;
  if ((rc = stage_emfs<double>(c, (const unsigned long long*)nullptr, (unsigned long long*)nullptr))) return rc;
  Sched bz = make_sched(make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1), c->kg_update);
  const unsigned nb = blocks_for(bz);
  const int cls = STAGE == 1 ? T_UPDATE1 : T_UPDATE2;
  if ((rc = launch(c, cls, k_targets_emhd, nb, g, bz, Pin, (const double*)c->tabC, (const double*)c->conn,
                   c->xrhs, c->divu)))
    return rc;
  if ((rc = launch(c, cls, k_update_emhd<STAGE>, nb, g, bz, Pin, (const double*)Xin, c->V, c->VX, c->utn,
                   (const double*)F1, (const double*)F2, (const double*)F3, (const double*)c->FX[0],
                   (const double*)c->FX[1], (const double*)c->FX[2], (const double*)c->E[0],
                   (const double*)c->E[1], (const double*)c->E[2], (const double*)c->tabC,
                   (const double*)c->conn, dt, dt_dev, c->ustar, c->xrhs)))
    return rc;
  auto implicit = [&](auto kernel, double* partial) {
    return launch(c, cls, kernel, nb, g, bz, Pin, (const double*)Xin, (const double*)c->ustar,
                  (const double*)c->xrhs, (const double*)c->divu, (const double*)c->utn, Pout, Xout,
                  (const double*)c->tabC, dt, dt_dev, c->fails, partial);
  };
  if (STAGE == 2 && rate && nb <= (unsigned)MAX_PARTIALS) return implicit(k_implicit_emhd<STAGE, true>, c->pdt);
  return implicit(k_implicit_emhd<STAGE, false>, (double*)nullptr);
}

// One step of the configured integrator with dt from the host, or, when
// dt_dev is given, with the dt the device reduction left there.  The update
// that ends the step leaves the CFL-rate partials of the new state, so the
// next dt needs only the final pass.
template <typename R, typename FT>
int do_step(grmhd_ctx* c, double dt, const double* dt_dev = nullptr) {
  int rc;
  if (c->params.ct != GRMHD_CT_FLUX && !c->faces_loaded) return GRMHD_E_STATE;
  c->rate_ready = false;
  if ((rc = ensure_ghosts(c))) return rc;
  c->ghosts_valid = false;
  const Dev& g = c->dev;
  if (c->params.egrmhd) {  // Extended GRMHD: the predictor-corrector with implicit stages
    if ((rc = emhd_stage<1>(c, c->P, c->X, c->P1, c->X1, dt, dt_dev, false))) return rc;
    if ((rc = fill_ghosts(c, c->P1))) return rc;
    if ((rc = emhd_stage<2>(c, c->P1, c->X1, c->P, c->X, dt, dt_dev, true))) return rc;
  } else if (c->params.integrator == GRMHD_INTEG_SSPRK54) {
    // five stages, the prims alternating between P1 and P (U^n lives in a
    // register from the first stage on); the last one's result copied back
    if ((rc = stage_ssp54<1, R, FT>(c, c->P, c->P1, dt, dt_dev, false))) return rc;
    if ((rc = fill_ghosts(c, c->P1))) return rc;
    if ((rc = stage_ssp54<2, R, FT>(c, c->P1, c->P, dt, dt_dev, false))) return rc;
    if ((rc = fill_ghosts(c, c->P))) return rc;
    if ((rc = stage_ssp54<3, R, FT>(c, c->P, c->P1, dt, dt_dev, false))) return rc;
    if ((rc = fill_ghosts(c, c->P1))) return rc;
    if ((rc = stage_ssp54<4, R, FT>(c, c->P1, c->P, dt, dt_dev, false))) return rc;
    if ((rc = fill_ghosts(c, c->P))) return rc;
    if ((rc = stage_ssp54<5, R, FT>(c, c->P, c->P1, dt, dt_dev, true))) return rc;
    if (hipMemcpyAsync(c->P, c->P1, sizeof(double) * NVAR * g.nz, hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
      return GRMHD_E_HIP;
  } else if (c->params.integrator == GRMHD_INTEG_RK1) {  // one stage, its result copied back to the state
    if ((rc = stage<1, R, FT>(c, c->P, c->P1, dt, dt_dev, true))) return rc;
    if (hipMemcpyAsync(c->P, c->P1, sizeof(double) * NVAR * g.nz, hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
      return GRMHD_E_HIP;
  } else {
    if ((rc = stage<1, R, FT>(c, c->P, c->P1, dt, dt_dev, false))) return rc;
    if ((rc = fill_ghosts(c, c->P1, c->phi1))) return rc;
    if ((rc = stage<2, R, FT>(c, c->P1, c->P, dt, dt_dev, true))) return rc;
  }
  const long nb = blocks_for(make_sched(make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1), c->kg_update));
  c->rate_ready = nb <= MAX_PARTIALS;
  c->rate_n = (int)nb;
  return GRMHD_OK;
}

// Enqueue the CFL reduction of the current prims (interior zones only, so no
// ghost fill): result[0] = max signal rate, result[2] = cfl / max,
// result[3] = 0 if that dt is usable.  When the last step's stage-2 update
// left the partials of this state, only the final pass runs.
int launch_dt(grmhd_ctx* c) {
  EvPair e = timing_events(c, T_DT);
  if (c->rate_ready) {
    hipExtLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BLOCK), 0, c->stream, e.a, e.b, 0,
                          (const double*)c->pdt, (const double*)nullptr, c->rate_n, c->result,
                          c->params.cfl);
    return hip_check();
  }
  const Dev& g = c->dev;
  Box bz = make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1);
  long nb = blocks_for(bz.count());
  if (nb > MAX_PARTIALS) nb = MAX_PARTIALS;
  hipExtLaunchKernelGGL(k_dt_partial, dim3((unsigned)nb), dim3(BLOCK), 0, c->stream, e.a, nullptr, 0, g,
                        bz, (const double*)c->P, (const double*)c->tabC, c->pmax);
  hipExtLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BLOCK), 0, c->stream, nullptr, e.b, 0,
                        (const double*)c->pmax, (const double*)nullptr, (int)nb, c->result, c->params.cfl);
  return hip_check();
}

// Kernel-side description of a grid, its metric and parameters.
Dev make_dev(const grmhd_grid* grid, const grmhd_metric* metric, const grmhd_params* params) {
  Dev g;
  g.n1 = grid->n1; g.n2 = grid->n2; g.n3 = grid->n3;
  g.s1 = g.n1 + 2 * NG; g.s2 = g.n2 + 2 * NG; g.s3 = g.n3 + 2 * NG;
  g.nz = (long)g.s1 * g.s2 * g.s3;
  g.plane = (long)g.s1 * g.s2;
  g.dx1 = (grid->x1max - grid->x1min) / g.n1;
  g.dx2 = (grid->x2max - grid->x2min) / g.n2;
  g.dx3 = (grid->x3max - grid->x3min) / g.n3;
  g.idx1 = 1.0 / g.dx1;
  g.idx2 = 1.0 / g.dx2;
  g.idx3 = 1.0 / g.dx3;
  g.x1min = grid->x1min;
  g.x2min = grid->x2min;
  for (int a = 0; a < 6; a++) g.bc[a] = grid->bc[a];
  const bool kerr = metric->metric == GRMHD_METRIC_KERR_MKS;
  g.pole_lo = kerr && fabs(grid->x2min) < 1e-10;
  g.pole_hi = kerr && fabs(grid->x2max - 1.0) < 1e-10;
  g.gam = params->gamma_ad;
  g.weno_eps = params->weno_eps;
  g.tol = params->newton_tol;
  g.maxit = params->newton_maxit;
  g.inverter = params->inverter;
  g.vmax2 = 1.0 - 1.0 / (params->kastaun_wmax * params->kastaun_wmax);
  g.floors = params->floors;
  g.ct = params->ct;
  g.rho_min_geom = params->rho_min_geom;
  g.u_min_geom = params->u_min_geom;
  g.bsq_over_rho_max = params->bsq_over_rho_max;
  g.bsq_over_u_max = params->bsq_over_u_max;
  g.u_over_rho_max = params->u_over_rho_max;
  g.gamma_max = params->gamma_max;
  g.tau = params->tau_r;
  g.chi = params->chi_emhd;
  g.nu = params->nu_emhd;
  g.st = SpaceTime{kerr ? 1 : 0, metric->a, metric->hslope};
  return g;
}

// ------------------------------------------------ CFL step, no allocation --
//
// grmhd_cfl_dt_noalloc: the CFL step of a caller's prims array without a
// context.  The zone-centre metric is evaluated in place (the same
// metric_point the context's tables hold, so the rates are the same bits)
// and the reduction's scratch -- the workgroup maxima and the final pass's
// four results -- is this file-scope device array, one copy per GPU, held
// until the process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns on that GPU (scratch_on_current_device).
constexpr int NOALLOC_PARTIALS = 2048;
__device__ __align__(256) double scratch[NOALLOC_PARTIALS + 8];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

// Device address of this GPU's scratch (looked up once per device, with the
// device current).
int scratch_on_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return GRMHD_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GRMHD_E_HIP;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return GRMHD_OK;
}

// Per zone the CFL signal rate with the metric evaluated at the zone centre;
// workgroup maxima to partial[] (grid-stride, so any box reduces through the
// launch's workgroups).
__global__ void __launch_bounds__(BLOCK) k_dt_partial_point(Dev g, Box box, const double* __restrict__ P,
                                                            double* partial) {
  double s = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < box.count(); t += stride) {
    int i, j, k;
    box_index(box, t, i, j, k);
    const long c = zid(g, i, j, k);
    double p[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; v++) p[v] = P[v * g.nz + c];
    PointMetric<double> m;
    const double xc1 = g.x1min + (i + 0.5) * g.dx1, xc2 = g.x2min + (j + 0.5) * g.dx2;
    metric_point(g.st, xc1, xc2, m.gcov, m.gcon, m.gdet, m.alpha);
    s = fmax(s, zone_rate(g, p, m));
  }
  double sm = 0.0;
  block_reduce(s, sm);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

int sync(grmhd_ctx* c) { return hipStreamSynchronize(c->stream) == hipSuccess ? GRMHD_OK : GRMHD_E_HIP; }

}  // namespace

extern "C" {

size_t grmhd_workspace_bytes(const grmhd_grid* grid, const grmhd_params* params) {
  if (!grid_ok(grid, params)) return 0;
  return carve(nullptr, nullptr, grid, params);
}

int grmhd_cfl_dt_noalloc(const grmhd_grid* grid, const grmhd_metric* metric, const grmhd_params* params,
                         const double* d_prims, double* dt_out, void* hip_stream) {
  if (!grid || !metric || !params || !d_prims || !dt_out || !grid_ok(grid, params)) return GRMHD_E_ARG;
  if (metric->metric != GRMHD_METRIC_MINKOWSKI && metric->metric != GRMHD_METRIC_KERR_MKS)
    return GRMHD_E_ARG;
  double* s = nullptr;
  int rc;
  if ((rc = scratch_on_current_device(&s))) return rc;
  const Dev g = make_dev(grid, metric, params);
  const Box bz = make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1);
  long nb = blocks_for(bz.count());
  if (nb > NOALLOC_PARTIALS) nb = NOALLOC_PARTIALS;  // grid-stride: every box fits the scratch
  hipStream_t st = (hipStream_t)hip_stream;
  k_dt_partial_point<<<(unsigned)nb, BLOCK, 0, st>>>(g, bz, d_prims, s);
  k_reduce_final<<<1, BLOCK, 0, st>>>((const double*)s, (const double*)nullptr, (int)nb,
                                      s + NOALLOC_PARTIALS, params->cfl);
  double smax = 0.0;
  if (hipMemcpyAsync(&smax, s + NOALLOC_PARTIALS, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess || hip_check() != GRMHD_OK)
    return GRMHD_E_HIP;
  if (!(smax > 0.0) || !isfinite(smax)) return GRMHD_E_STATE;
  *dt_out = params->cfl / smax;
  return GRMHD_OK;
}

int grmhd_create(grmhd_ctx** out, const grmhd_grid* grid, const grmhd_metric* metric,
                 const grmhd_params* params, void* d_workspace, size_t ws_bytes, void* hip_stream) {
  if (!out || !metric || !grid_ok(grid, params) || !d_workspace) return GRMHD_E_ARG;
  if (metric->metric != GRMHD_METRIC_MINKOWSKI && metric->metric != GRMHD_METRIC_KERR_MKS)
    return GRMHD_E_ARG;
  if (((uintptr_t)d_workspace & 255) != 0) return GRMHD_E_ARG;
  if (ws_bytes < carve(nullptr, nullptr, grid, params)) return GRMHD_E_NOMEM;
  grmhd_ctx* c = new (std::nothrow) grmhd_ctx();
  if (!c) return GRMHD_E_NOMEM;
  c->grid = *grid;
  c->metric = *metric;
  c->params = *params;
  c->stream = (hipStream_t)hip_stream;
  carve(c, (char*)d_workspace, grid, params);
  c->dev = make_dev(grid, metric, params);
  Dev& g = c->dev;
  k_geometry<<<blocks_for(g.plane), BLOCK, 0, c->stream>>>(g, c->tabC, c->tabF1, c->tabF2, c->corner,
                                                           c->conn, c->dgs);
  // failure count zero; no dt reduced yet (result[3] = 1)
  static const double result0[8] = {0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0};
  if (hipMemsetAsync(c->fails, 0, 8 * sizeof(unsigned long long), c->stream) != hipSuccess ||
      hipMemsetAsync(c->mark, 0, (size_t)g.nz, c->stream) != hipSuccess ||
      (c->X && hipMemsetAsync(c->X, 0, sizeof(double) * NXV * g.nz, c->stream) != hipSuccess) ||
      (c->X1 && hipMemsetAsync(c->X1, 0, sizeof(double) * NXV * g.nz, c->stream) != hipSuccess) ||
      hipMemcpyAsync(c->result, result0, sizeof(result0), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hip_check() != GRMHD_OK) {
    delete c;
    return GRMHD_E_HIP;
  }
  *out = c;
  return GRMHD_OK;
}

int grmhd_load_prims(grmhd_ctx* c, const double* d_prims) {
  if (!c || !d_prims) return GRMHD_E_ARG;
  c->rate_ready = false;
  c->ghosts_valid = false;
  size_t bytes = sizeof(double) * NVAR * c->dev.nz;
  if (hipMemcpyAsync(c->P, d_prims, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  // the stage buffer carries the same (frozen) ghosts
  if (hipMemcpyAsync(c->P1, d_prims, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  // face-centred CT: the zones' field is their faces' mean
  if (c->faces_loaded) return cell_b_from_faces(c);
  return GRMHD_OK;
}

int grmhd_load_extended(grmhd_ctx* c, const double* d_extra) {
  if (!c || !d_extra) return GRMHD_E_ARG;
  if (!c->params.egrmhd) return GRMHD_E_STATE;
  const size_t bytes = sizeof(double) * NXV * c->dev.nz;
  // the stage buffer carries the same (frozen) ghosts
  if (hipMemcpyAsync(c->X, d_extra, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->X1, d_extra, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  return GRMHD_OK;
}

int grmhd_get_extended(grmhd_ctx* c, double* d_extra) {
  if (!c || !d_extra) return GRMHD_E_ARG;
  if (!c->params.egrmhd) return GRMHD_E_STATE;
  int rc;
  if ((rc = launch(c, T_BC, k_bc_extra, blocks_for(ghost_count(c->dev)), c->dev, c->X))) return rc;
  if (hipMemcpyAsync(d_extra, c->X, sizeof(double) * NXV * c->dev.nz, hipMemcpyDeviceToDevice, c->stream) !=
      hipSuccess)
    return GRMHD_E_HIP;
  return GRMHD_OK;
}

int grmhd_load_faces(grmhd_ctx* c, const double* d_faces) {
  if (!c || !d_faces) return GRMHD_E_ARG;
  if (c->params.ct == GRMHD_CT_FLUX) return GRMHD_E_STATE;
  const size_t bytes = sizeof(double) * c->dev.nz;
  for (int d = 0; d < 3; d++) {
    // the stage-1 faces carry the same (frozen) ghosts
    if (hipMemcpyAsync(c->phi[d], d_faces + d * c->dev.nz, bytes, hipMemcpyDeviceToDevice, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(c->phi1[d], d_faces + d * c->dev.nz, bytes, hipMemcpyDeviceToDevice, c->stream) !=
            hipSuccess)
      return GRMHD_E_HIP;
  }
  c->faces_loaded = true;
  c->rate_ready = false;
  c->ghosts_valid = false;
  return cell_b_from_faces(c);
}

int grmhd_get_faces(grmhd_ctx* c, double* d_out) {
  if (!c || !d_out) return GRMHD_E_ARG;
  if (c->params.ct == GRMHD_CT_FLUX || !c->faces_loaded) return GRMHD_E_STATE;
  int rc;
  if ((rc = ensure_ghosts(c))) return rc;
  for (int d = 0; d < 3; d++)
    if (hipMemcpyAsync(d_out + d * c->dev.nz, c->phi[d], sizeof(double) * c->dev.nz, hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      return GRMHD_E_HIP;
  return GRMHD_OK;
}

int grmhd_face_divb(grmhd_ctx* c, double* max_out, double* mean_out) {
  if (!c || !max_out || !mean_out) return GRMHD_E_ARG;
  if (c->params.ct == GRMHD_CT_FLUX || !c->faces_loaded) return GRMHD_E_STATE;
  const Dev& g = c->dev;
  Box b = make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1);
  long nb = blocks_for(b.count());
  if (nb > MAX_PARTIALS) nb = MAX_PARTIALS;
  k_face_divb_partial<<<(unsigned)nb, BLOCK, 0, c->stream>>>(g, b, c->phi[0], c->phi[1], c->phi[2], c->pmax,
                                                              c->psum);
  k_reduce_final<<<1, BLOCK, 0, c->stream>>>(c->pmax, c->psum, (int)nb, c->result, 0.0);
  int rc;
  if ((rc = hip_check())) return rc;
  double res[2];
  if (hipMemcpyAsync(res, c->result, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  if ((rc = sync(c))) return rc;
  *max_out = res[0];
  *mean_out = res[1] / (double)b.count();
  return GRMHD_OK;
}

int grmhd_step(grmhd_ctx* c, double dt) {
  if (!c || !(dt > 0.0) || !isfinite(dt)) return GRMHD_E_ARG;
  if (c->params.precision == GRMHD_PREC_FP64) return do_step<double, double>(c, dt);
  return do_step<float, float>(c, dt);
}

int grmhd_estimate_dt(grmhd_ctx* c, double* dt_out) {
  if (!c || !dt_out) return GRMHD_E_ARG;
  int rc;
  if ((rc = launch_dt(c))) return rc;
  double smax = 0.0;
  if (hipMemcpyAsync(&smax, c->result, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  if ((rc = sync(c))) return rc;
  if (!(smax > 0.0) || !isfinite(smax)) return GRMHD_E_STATE;
  *dt_out = c->params.cfl / smax;
  return GRMHD_OK;
}

int grmhd_step_cfl(grmhd_ctx* c) {
  if (!c) return GRMHD_E_ARG;
  int rc;
  if ((rc = launch_dt(c))) return rc;
  if (c->params.precision == GRMHD_PREC_FP64) return do_step<double, double>(c, 0.0, c->result + 2);
  return do_step<float, float>(c, 0.0, c->result + 2);
}

int grmhd_last_dt(grmhd_ctx* c, double* dt_out) {
  if (!c || !dt_out) return GRMHD_E_ARG;
  double r[2];
  if (hipMemcpyAsync(r, c->result + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  int rc;
  if ((rc = sync(c))) return rc;
  if (r[1] != 0.0) return GRMHD_E_STATE;
  *dt_out = r[0];
  return GRMHD_OK;
}

int grmhd_get_prims(grmhd_ctx* c, double* d_out) {
  if (!c || !d_out) return GRMHD_E_ARG;
  int rc;
  if ((rc = ensure_ghosts(c))) return rc;
  if (hipMemcpyAsync(d_out, c->P, sizeof(double) * NVAR * c->dev.nz, hipMemcpyDeviceToDevice,
                     c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  return GRMHD_OK;
}

int grmhd_divb(grmhd_ctx* c, double* d_divb, double* max_out, double* mean_out) {
  if (!c || !max_out || !mean_out) return GRMHD_E_ARG;
  int rc;
  if ((rc = ensure_ghosts(c))) return rc;
  const Dev& g = c->dev;
  int ilo = g.bc[0] == GRMHD_BC_PERIODIC ? 0 : 1;
  int jlo = g.bc[2] == GRMHD_BC_PERIODIC ? 0 : 1;
  int klo = g.bc[4] == GRMHD_BC_PERIODIC ? 0 : 1;
  Box b = make_box(ilo, g.n1 - 1, jlo, g.n2 - 1, klo, g.n3 - 1);
  long cnt = b.n1 > 0 && b.n2 > 0 && b.n3 > 0 ? b.count() : 0;
  if (cnt == 0) {
    *max_out = *mean_out = 0.0;
    return GRMHD_OK;
  }
  long nb = blocks_for(cnt);
  if (nb > MAX_PARTIALS) nb = MAX_PARTIALS;
  k_divb_partial<<<(unsigned)nb, BLOCK, 0, c->stream>>>(g, b, c->P, c->tabC, c->corner, d_divb, c->pmax, c->psum);
  k_reduce_final<<<1, BLOCK, 0, c->stream>>>(c->pmax, c->psum, (int)nb, c->result, 0.0);
  if ((rc = hip_check())) return rc;
  double res[2];
  if (hipMemcpyAsync(res, c->result, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  if ((rc = sync(c))) return rc;
  *max_out = res[0];
  *mean_out = res[1] / (double)cnt;
  return GRMHD_OK;
}

int grmhd_get_counters(grmhd_ctx* c, long long* out4) {
  if (!c || !out4) return GRMHD_E_ARG;
  unsigned long long f[8];
  if (hipMemcpyAsync(f, c->fails, sizeof(f), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  int rc = sync(c);
  if (rc) return rc;
  out4[0] = (long long)f[C_FAILS];
  out4[1] = (long long)f[C_FLOORS];
  out4[2] = (long long)f[C_FOFC];
  out4[3] = (long long)f[C_FLUID];
  return GRMHD_OK;
}

int grmhd_get_status(grmhd_ctx* c, long long* n_inv_fail, long long* n_floor) {
  if (!c || !n_inv_fail || !n_floor) return GRMHD_E_ARG;
  long long f[4];
  int rc = grmhd_get_counters(c, f);
  if (rc) return rc;
  *n_inv_fail = f[0];
  *n_floor = f[1];
  return GRMHD_OK;
}

int grmhd_reset_status(grmhd_ctx* c) {
  if (!c) return GRMHD_E_ARG;
  return hipMemsetAsync(c->fails, 0, 8 * sizeof(unsigned long long), c->stream) == hipSuccess
             ? GRMHD_OK
             : GRMHD_E_HIP;
}

int grmhd_prims_to_cons(grmhd_ctx* c, const double* d_prims, double* d_cons) {
  if (!c || !d_prims || !d_cons) return GRMHD_E_ARG;
  const Dev& g = c->dev;
  Box bz = make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1);
  k_prims_to_cons<<<blocks_for(bz.count()), BLOCK, 0, c->stream>>>(g, bz, d_prims, d_cons, c->tabC);
  return hip_check();
}

int grmhd_cons_to_prims(grmhd_ctx* c, const double* d_cons, const double* d_guess, double* d_prims,
                        int* d_flags, long long* n_fail) {
  if (!c || !d_cons || !d_guess || !d_prims || !n_fail) return GRMHD_E_ARG;
  const Dev& g = c->dev;
  Box bz = make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1);
  unsigned long long* cnt = c->fails + C_C2P;
  if (hipMemsetAsync(cnt, 0, sizeof(unsigned long long), c->stream) != hipSuccess) return GRMHD_E_HIP;
  k_cons_to_prims<<<blocks_for(bz.count()), BLOCK, 0, c->stream>>>(g, bz, d_cons, d_guess, d_prims, d_flags,
                                                                   c->tabC, cnt);
  int rc = hip_check();
  if (rc) return rc;
  unsigned long long f = 0;
  if (hipMemcpyAsync(&f, cnt, sizeof(f), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  if ((rc = sync(c))) return rc;
  *n_fail = (long long)f;
  return GRMHD_OK;
}

int grmhd_fluxes(grmhd_ctx* c, const double* d_prims, double* d_flux) {
  if (!c || !d_prims || !d_flux) return GRMHD_E_ARG;
  if (c->params.precision != GRMHD_PREC_FP64 || c->params.egrmhd) return GRMHD_E_STATE;
  int rc;
  if ((rc = grmhd_load_prims(c, d_prims))) return rc;
  if ((rc = ensure_ghosts(c))) return rc;
  if ((rc = stage_fluxes<double, double>(c, c->P))) return rc;
  const Dev& g = c->dev;
  Box be = make_box(0, g.n1, 0, g.n2, 0, g.n3);
  k_ct_fluxes<double><<<blocks_for(be.count()), BLOCK, 0, c->stream>>>(
      g, be, (double*)c->F[0], (double*)c->F[1], (double*)c->F[2], (const double*)c->E[0],
      (const double*)c->E[1], (const double*)c->E[2]);
  if ((rc = hip_check())) return rc;
  size_t bytes = sizeof(double) * NVAR * g.nz;
  for (int d = 0; d < 3; d++)
    if (hipMemcpyAsync(d_flux + d * NVAR * g.nz, c->F[d], bytes, hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
      return GRMHD_E_HIP;
  return GRMHD_OK;
}

const char* grmhd_strerror(int code) {
  switch (code) {
    case GRMHD_OK: return "ok";
    case GRMHD_E_ARG: return "invalid argument";
    case GRMHD_E_HIP: return "HIP runtime error";
    case GRMHD_E_STATE: return "invalid state for this call";
    case GRMHD_E_NOMEM: return "workspace too small";
    default: return "unknown error";
  }
}

}  // extern "C"

namespace {

struct VjpCarve {
  double *A, *B, *C, *LV, *LL, *LP, *LPh, *LG, *LE[3], *LS[3], *GZ, *GF[3];
  unsigned char *fl1, *fl2;
  unsigned long long* fails;
};

size_t vjp_carve(const grmhd_grid* g, int recon, char* base, VjpCarve* out) {
  long nz = (long)(g->n1 + 2 * NG) * (g->n2 + 2 * NG) * (g->n3 + 2 * NG);
  int W = recon == GRMHD_RECON_MC ? Stencil<GRMHD_RECON_MC>::W : Stencil<GRMHD_RECON_WENO5>::W;
  Carve cv;
  VjpCarve v;
  v.A = cv.take<double>(base, NVAR * nz);
  v.B = cv.take<double>(base, NVAR * nz);
  v.C = cv.take<double>(base, NVAR * nz);
  v.LV = cv.take<double>(base, NVAR * nz);
  v.LL = cv.take<double>(base, NVAR * nz);
  v.LP = cv.take<double>(base, NVAR * nz);
  v.LPh = cv.take<double>(base, NVAR * nz);
  v.LG = cv.take<double>(base, 5 * nz);
  for (int d = 0; d < 3; d++) v.LE[d] = cv.take<double>(base, nz);
  for (int d = 0; d < 3; d++) v.LS[d] = cv.take<double>(base, (long)NVAR * W * nz);
  v.GZ = cv.take<double>(base, nz);
  for (int d = 0; d < 3; d++) v.GF[d] = cv.take<double>(base, nz);
  v.fl1 = cv.take<unsigned char>(base, nz);
  v.fl2 = cv.take<unsigned char>(base, nz);
  v.fails = cv.take<unsigned long long>(base, 8);
  if (out) *out = v;
  return cv.off;
}

template <int RECON>
int adj_stage(grmhd_ctx* c, const VjpCarve& w, const double* Pin, bool stage1, double* LPout) {
  const Dev& g = c->dev;
  const long nz = g.nz;
  k_adj_emf<<<blocks_for(nz), BLOCK, 0, c->stream>>>(g, w.LL, w.LE[0], w.LE[1], w.LE[2]);
  Box b1 = make_box(0, g.n1, -1, g.n2, -1, g.n3);
  Box b2 = make_box(-1, g.n1, 0, g.n2, -1, g.n3);
  Box b3 = make_box(-1, g.n1, -1, g.n2, 0, g.n3);
  k_adj_face<1, RECON><<<blocks_for(b1.count()), BLOCK, 0, c->stream>>>(g, b1, Pin, c->tabF1, w.LL, w.LE[0],
                                                                      w.LE[1], w.LE[2], w.LS[0], w.GF[0]);
  k_adj_face<2, RECON><<<blocks_for(b2.count()), BLOCK, 0, c->stream>>>(g, b2, Pin, c->tabF2, w.LL, w.LE[0],
                                                                      w.LE[1], w.LE[2], w.LS[1], w.GF[1]);
  k_adj_face<3, RECON><<<blocks_for(b3.count()), BLOCK, 0, c->stream>>>(g, b3, Pin, c->tabC, w.LL, w.LE[0],
                                                                      w.LE[1], w.LE[2], w.LS[2], w.GF[2]);
  k_adj_gather<RECON><<<blocks_for(nz), BLOCK, 0, c->stream>>>(g, b1, b2, b3, w.LS[0], w.LS[1], w.LS[2],
                                                               w.LPh);
  Box bz = make_box(0, g.n1 - 1, 0, g.n2 - 1, 0, g.n3 - 1);
  if (stage1)
    k_adj_zone<true><<<blocks_for(bz.count()), BLOCK, 0, c->stream>>>(g, bz, Pin, c->tabC, c->conn, w.LPh,
                                                                      w.LL, w.LV, w.LG, LPout, w.GZ);
  else
    k_adj_zone<false><<<blocks_for(bz.count()), BLOCK, 0, c->stream>>>(g, bz, Pin, c->tabC, c->conn, w.LPh,
                                                                       w.LL, nullptr, w.LG, LPout, w.GZ);
  return hip_check();
}

template <int RECON>
int step_vjp(grmhd_ctx* c, const VjpCarve& w, const double* d_in, double dt, const double* d_gout,
             double* d_gin, double* g_gamma) {
  const Dev& g = c->dev;
  const long nz = g.nz;
  const size_t bytes = sizeof(double) * NVAR * nz;
  int rc;
  // forward recompute from the checkpoint: A = P^n, B = P^(1), C = P^(n+1).
  // The updates write interior zones (prims and failure flags); B's ghosts
  // are filled before they are read, except frozen ones, which keep the
  // input's (hence the copy only then); C and the flags are read at
  // interior zones only (the inversion's adjoint).
  bool frozen = false;
  for (int f = 0; f < 6; f++) frozen = frozen || c->grid.bc[f] == GRMHD_BC_FROZEN;
  if (hipMemcpyAsync(w.A, d_in, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
      (frozen && hipMemcpyAsync(w.B, d_in, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) ||
      hipMemsetAsync(w.GZ, 0, sizeof(double) * nz, c->stream) != hipSuccess ||
      hipMemsetAsync(d_gin, 0, bytes, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  for (int d = 0; d < 3; d++)
    if (hipMemsetAsync(w.GF[d], 0, sizeof(double) * nz, c->stream) != hipSuccess) return GRMHD_E_HIP;
  if ((rc = fill_ghosts(c, w.A))) return rc;
  if ((rc = stage_fluxes<double, double>(c, w.A))) return rc;
  if ((rc = stage_update<1, double>(c, w.A, w.B, dt, w.fails, w.fl1))) return rc;
  if ((rc = fill_ghosts(c, w.B))) return rc;
  if ((rc = stage_fluxes<double, double>(c, w.B))) return rc;
  if ((rc = stage_update<2, double>(c, w.B, w.C, dt, w.fails, w.fl2))) return rc;
  // reverse sweep
  k_adj_ift<<<blocks_for(nz), BLOCK, 0, c->stream>>>(g, w.C, w.fl2, c->tabC, d_gout, 0, dt, w.LV, w.LL, w.LG,
                                                     w.GZ);
  if ((rc = hip_check())) return rc;
  if ((rc = adj_stage<RECON>(c, w, w.B, false, w.LP))) return rc;
  k_adj_ift<<<blocks_for(nz), BLOCK, 0, c->stream>>>(g, w.B, w.fl1, c->tabC, w.LP, 1, dt, w.LV, w.LL, w.LG,
                                                     w.GZ);
  if ((rc = hip_check())) return rc;
  if ((rc = adj_stage<RECON>(c, w, w.A, true, d_gin))) return rc;
  long nb = blocks_for(nz);
  if (nb > MAX_PARTIALS) nb = MAX_PARTIALS;
  k_adj_gsum<<<(unsigned)nb, BLOCK, 0, c->stream>>>(nz, w.GZ, w.GF[0], w.GF[1], w.GF[2], c->pmax, c->psum);
  k_reduce_final<<<1, BLOCK, 0, c->stream>>>(c->pmax, c->psum, (int)nb, c->result, 0.0);
  if ((rc = hip_check())) return rc;
  double res[2];
  if (hipMemcpyAsync(res, c->result, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return GRMHD_E_HIP;
  if ((rc = sync(c))) return rc;
  *g_gamma = res[1];
  return GRMHD_OK;
}

}  // namespace

extern "C" {

size_t grmhd_vjp_workspace_bytes(const grmhd_grid* grid, const grmhd_params* params) {
  if (!grid_ok(grid, params) || params->floors || params->fofc ||
      (params->recon != GRMHD_RECON_MC && params->recon != GRMHD_RECON_WENO5) ||
      params->ct != GRMHD_CT_FLUX || params->inverter == GRMHD_INV_IMPLICIT ||
      params->integrator != GRMHD_INTEG_SSPRK2)
    return 0;
  return vjp_carve(grid, params->recon, nullptr, nullptr);
}

int grmhd_step_vjp(grmhd_ctx* c, const double* d_prims_in, double dt, const double* d_gprims_out,
                   double* d_gprims_in, double* g_gamma, void* d_vjp_ws, size_t vjp_ws_bytes) {
  if (!c || !d_prims_in || !d_gprims_out || !d_gprims_in || !g_gamma || !d_vjp_ws) return GRMHD_E_ARG;
  if (!(dt > 0.0) || !isfinite(dt)) return GRMHD_E_ARG;
  if (c->params.precision != GRMHD_PREC_FP64) return GRMHD_E_STATE;
  // the adjoint covers the plain step with MC or WENO5 (no floors, no
  // correction)
  if (c->params.floors || c->params.fofc ||
      (c->params.recon != GRMHD_RECON_MC && c->params.recon != GRMHD_RECON_WENO5) ||
      c->params.ct != GRMHD_CT_FLUX || c->params.inverter == GRMHD_INV_IMPLICIT ||
      c->params.integrator != GRMHD_INTEG_SSPRK2)
    return GRMHD_E_STATE;
  if (((uintptr_t)d_vjp_ws & 255) != 0) return GRMHD_E_ARG;
  if (vjp_ws_bytes < vjp_carve(&c->grid, c->params.recon, nullptr, nullptr)) return GRMHD_E_NOMEM;
  VjpCarve w;
  vjp_carve(&c->grid, c->params.recon, (char*)d_vjp_ws, &w);
  if (c->params.recon == GRMHD_RECON_MC) return step_vjp<GRMHD_RECON_MC>(c, w, d_prims_in, dt, d_gprims_out, d_gprims_in, g_gamma);
  return step_vjp<GRMHD_RECON_WENO5>(c, w, d_prims_in, dt, d_gprims_out, d_gprims_in, g_gamma);
}

int grmhd_set_schedule(grmhd_ctx* c, int kg_flux, int kg_update) {
  if (!c || kg_flux < 1 || kg_update < 1) return GRMHD_E_ARG;
  c->kg_flux = kg_flux;
  c->kg_update = kg_update;
  return GRMHD_OK;
}

int grmhd_timing(grmhd_ctx* c, int class_mask) {
  if (!c) return GRMHD_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return GRMHD_E_HIP;
  c->timing = (unsigned)class_mask & ((1u << T_NCLASS) - 1u);
  c->nmarks = 0;
  return GRMHD_OK;
}

int grmhd_timing_report(grmhd_ctx* c, double* total_ms, long long* launches, int nclass) {
  if (!c || !total_ms || !launches || nclass < T_NCLASS) return GRMHD_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return GRMHD_E_HIP;
  for (int q = 0; q < nclass; q++) {
    total_ms[q] = 0.0;
    launches[q] = 0;
  }
  for (int q = 0; q < c->nmarks; q++) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->marks[q].a, c->marks[q].b) != hipSuccess) return GRMHD_E_HIP;
    total_ms[c->marks[q].cls] += ms;
    launches[c->marks[q].cls] += 1;
  }
  return GRMHD_OK;
}

int grmhd_destroy(grmhd_ctx* c) {
  if (!c) return GRMHD_E_ARG;
  for (int q = 0; q < c->capmarks; q++) {
    (void)hipEventDestroy(c->marks[q].a);
    (void)hipEventDestroy(c->marks[q].b);
  }
  free(c->marks);
  delete c;
  return GRMHD_OK;
}


// ---------------------------------------------------------------- packs --

}  // extern "C"

struct grmhd_pack {
  grmhd_params params;
  grmhd_metric metric;
  hipStream_t stream;
  int nb;
  std::vector<BlockView> views;
  std::vector<long> prim_off;  // offset (doubles) of each block in the packed prims
  long prim_total;
  BlockView* d_views;
  int* d_pre;
  unsigned long long* d_fails;
  int items[PH_N];  // work items (workgroups) of each phase launch
  grmhd_grid global;
  int* d_owner;  // ghost exchange: owner block of every global interior zone, or null (frozen ghosts)
  int max_nz;    // padded zones of the largest block
};

namespace {

size_t pack_carve(int nb, const int* n, char* base, grmhd_pack* pk) {
  Carve cv;
  long prim_total = 0;
  for (int b = 0; b < nb; b++) {
    long s = n[b] + 2 * NG;
    long nz = s * s * s, plane = s * s;
    BlockView v;
    memset(&v, 0, sizeof(v));
    v.P = cv.take<double>(base, NVAR * nz);
    v.P1 = cv.take<double>(base, NVAR * nz);
    v.V = cv.take<double>(base, NVAR * nz);
    for (int d = 0; d < 3; d++) v.F[d] = cv.take<double>(base, NVAR * nz);
    for (int d = 0; d < 3; d++) v.E[d] = cv.take<double>(base, nz);
    v.tabC = cv.take<double>(base, G_NF * plane);
    v.tabF1 = cv.take<double>(base, G_NF * plane);
    v.tabF2 = cv.take<double>(base, G_NF * plane);
    v.corner = cv.take<double>(base, plane);
    v.dgs = cv.take<double>(base, NDG * plane);
    if (pk) {
      pk->views.push_back(v);
      pk->prim_off.push_back(prim_total);
    }
    prim_total += NVAR * nz;
  }
  BlockView* dv = cv.take<BlockView>(base, nb);
  int* pre = cv.take<int>(base, PH_N * (nb + 1));
  unsigned long long* fails = cv.take<unsigned long long>(base, 8);
  if (pk) {
    pk->d_views = dv;
    pk->d_pre = pre;
    pk->d_fails = fails;
    pk->prim_total = prim_total;
  }
  return cv.off;
}

// Default tiles: linear runs of BLOCK positions (face boxes of n + 1 by n + 2
// zones fit no power-of-two tile evenly).
int default_tile(int, int& t1, int& t2, int& t3) {
  t1 = t2 = t3 = 0;
  return 0;
}

int pack_upload(grmhd_pack* pk) {
  std::vector<int> pre(PH_N * (pk->nb + 1));
  for (int ph = 0; ph < PH_N; ph++) {
    long acc = 0;
    for (int b = 0; b < pk->nb; b++) {
      pre[ph * (pk->nb + 1) + b] = (int)acc;
      acc += block_items(pk->views[b], ph);
    }
    if (acc > (1L << 30)) return GRMHD_E_ARG;
    pre[ph * (pk->nb + 1) + pk->nb] = (int)acc;
    pk->items[ph] = (int)acc;
  }
  if (hipMemcpy(pk->d_views, pk->views.data(), sizeof(BlockView) * pk->nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pk->d_pre, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice) != hipSuccess)
    return GRMHD_E_HIP;
  return GRMHD_OK;
}

template <int RECON>
int pack_launch(grmhd_pack* pk, int stage, double dt) {
  if (pk->d_owner) {
    PackGlobal G{pk->global.n1, pk->global.n2, pk->global.n3, {0, 0, 0, 0, 0, 0}};
    for (int a = 0; a < 6; a++) G.bc[a] = pk->global.bc[a];
    dim3 grid((unsigned)((pk->max_nz + BLOCK - 1) / BLOCK), (unsigned)pk->nb);
    k_pack_exchange<<<grid, BLOCK, 0, pk->stream>>>(pk->d_views, pk->d_owner, G, stage);
  }
  const BlockView* views = pk->d_views;
  const int nb = pk->nb;
  const int* pre = pk->d_pre;
  bool linear = true;
  for (const BlockView& v : pk->views) linear = linear && v.t1 == 0;
  auto flux = [&](auto kernel) { kernel<<<pk->items[PH_FLUX], BLOCK, 0, pk->stream>>>(views, nb, pre); };
  if (stage == 1) {
    if (linear)
      flux(k_pack_flux<1, RECON, true>);
    else
      flux(k_pack_flux<1, RECON, false>);
    k_pack_emf<<<pk->items[PH_EMF], BLOCK, 0, pk->stream>>>(views, nb, pre);
    k_pack_update<1><<<pk->items[PH_UPDATE], BLOCK, 0, pk->stream>>>(views, nb, pre, dt, pk->d_fails);
  } else {
    if (linear)
      flux(k_pack_flux<2, RECON, true>);
    else
      flux(k_pack_flux<2, RECON, false>);
    k_pack_emf<<<pk->items[PH_EMF], BLOCK, 0, pk->stream>>>(views, nb, pre);
    k_pack_update<2><<<pk->items[PH_UPDATE], BLOCK, 0, pk->stream>>>(views, nb, pre, dt, pk->d_fails);
  }
  return hip_check();
}

}  // namespace

extern "C" {

size_t grmhd_pack_workspace_bytes(int nblocks, const int* n) {
  if (nblocks < 1 || !n) return 0;
  for (int b = 0; b < nblocks; b++)
    if (n[b] < 1) return 0;
  return pack_carve(nblocks, n, nullptr, nullptr);
}

int grmhd_pack_create(grmhd_pack** out, int nblocks, const int* n, const int* offsets_ijk,
                      const grmhd_grid* global, const grmhd_metric* metric, const grmhd_params* params,
                      void* d_ws, size_t ws_bytes, void* stream) {
  if (!out || nblocks < 1 || !n || !offsets_ijk || !global || !metric || !params || !d_ws) return GRMHD_E_ARG;
  if (!grid_ok(global, params) || params->precision != GRMHD_PREC_FP64) return GRMHD_E_ARG;
  // packs advance the plain step with MC or WENO5
  if (params->floors || params->fofc || (params->recon != GRMHD_RECON_MC && params->recon != GRMHD_RECON_WENO5) ||
      params->ct != GRMHD_CT_FLUX || params->inverter == GRMHD_INV_IMPLICIT ||
      params->integrator != GRMHD_INTEG_SSPRK2)
    return GRMHD_E_ARG;
  if (((uintptr_t)d_ws & 255) != 0) return GRMHD_E_ARG;
  for (int b = 0; b < nblocks; b++) {
    const int* o = offsets_ijk + 3 * b;
    if (n[b] < 1 || o[0] < 0 || o[1] < 0 || o[2] < 0 || o[0] + n[b] > global->n1 || o[1] + n[b] > global->n2 ||
        o[2] + n[b] > global->n3)
      return GRMHD_E_ARG;
  }
  if (ws_bytes < pack_carve(nblocks, n, nullptr, nullptr)) return GRMHD_E_NOMEM;
  grmhd_pack* pk = new (std::nothrow) grmhd_pack();
  if (!pk) return GRMHD_E_NOMEM;
  pk->params = *params;
  pk->metric = *metric;
  pk->stream = (hipStream_t)stream;
  pk->nb = nblocks;
  pk->global = *global;
  pk->d_owner = nullptr;
  pk->max_nz = 0;
  pack_carve(nblocks, n, (char*)d_ws, pk);
  const double gd1 = (global->x1max - global->x1min) / global->n1;
  const double gd2 = (global->x2max - global->x2min) / global->n2;
  const double gd3 = (global->x3max - global->x3min) / global->n3;
  bool kerr = metric->metric == GRMHD_METRIC_KERR_MKS;
  for (int b = 0; b < nblocks; b++) {
    const int* o = offsets_ijk + 3 * b;
    Dev& g = pk->views[b].g;
    g.n1 = g.n2 = g.n3 = n[b];
    g.s1 = g.s2 = g.s3 = n[b] + 2 * NG;
    g.nz = (long)g.s1 * g.s2 * g.s3;
    g.plane = (long)g.s1 * g.s2;
    double x1lo = global->x1min + o[0] * gd1, x2lo = global->x2min + o[1] * gd2;
    double x1hi = global->x1min + (o[0] + n[b]) * gd1, x2hi = global->x2min + (o[1] + n[b]) * gd2;
    double x3lo = global->x3min + o[2] * gd3, x3hi = global->x3min + (o[2] + n[b]) * gd3;
    g.dx1 = (x1hi - x1lo) / n[b];
    g.dx2 = (x2hi - x2lo) / n[b];
    g.dx3 = (x3hi - x3lo) / n[b];
    g.idx1 = 1.0 / g.dx1;
    g.idx2 = 1.0 / g.dx2;
    g.idx3 = 1.0 / g.dx3;
    g.x1min = x1lo;
    g.x2min = x2lo;
    for (int a = 0; a < 6; a++) g.bc[a] = GRMHD_BC_FROZEN;
    g.pole_lo = kerr && fabs(x2lo) < 1e-10;
    g.pole_hi = kerr && fabs(x2hi - 1.0) < 1e-10;
    g.gam = params->gamma_ad;
    g.weno_eps = params->weno_eps;
    g.tol = params->newton_tol;
    g.maxit = params->newton_maxit;
    g.inverter = params->inverter;
    g.vmax2 = 1.0 - 1.0 / (params->kastaun_wmax * params->kastaun_wmax);
    g.floors = params->floors;
    g.ct = params->ct;
    g.rho_min_geom = params->rho_min_geom;
    g.u_min_geom = params->u_min_geom;
    g.bsq_over_rho_max = params->bsq_over_rho_max;
    g.bsq_over_u_max = params->bsq_over_u_max;
    g.u_over_rho_max = params->u_over_rho_max;
    g.gamma_max = params->gamma_max;
    g.st = SpaceTime{kerr ? 1 : 0, metric->a, metric->hslope};
    BlockView& v = pk->views[b];
    v.o1 = o[0];
    v.o2 = o[1];
    v.o3 = o[2];
    if (g.nz > pk->max_nz) pk->max_nz = (int)g.nz;
    default_tile(n[b], v.t1, v.t2, v.t3);
    k_geometry<<<blocks_for(g.plane), BLOCK, 0, pk->stream>>>(g, v.tabC, v.tabF1, v.tabF2, v.corner, nullptr,
                                                               v.dgs);
  }
  if (hip_check() || hipMemsetAsync(pk->d_fails, 0, sizeof(unsigned long long), pk->stream) != hipSuccess ||
      pack_upload(pk) != GRMHD_OK) {
    delete pk;
    return GRMHD_E_HIP;
  }
  *out = pk;
  return GRMHD_OK;
}

int grmhd_pack_set_tiles(grmhd_pack* pk, int n, int t1, int t2, int t3) {
  const bool linear = t1 == 0 && t2 == 0 && t3 == 0;
  if (!pk || (!linear && (t1 < 1 || t2 < 1 || t3 < 1 || t1 * t2 * t3 > BLOCK))) return GRMHD_E_ARG;
  if (hipStreamSynchronize(pk->stream) != hipSuccess) return GRMHD_E_HIP;
  for (int b = 0; b < pk->nb; b++)
    if (pk->views[b].g.n1 == n) {
      pk->views[b].t1 = t1;
      pk->views[b].t2 = t2;
      pk->views[b].t3 = t3;
    }
  return pack_upload(pk);
}

int grmhd_pack_load_prims(grmhd_pack* pk, const double* d_prims) {
  if (!pk || !d_prims) return GRMHD_E_ARG;
  for (int b = 0; b < pk->nb; b++) {
    size_t bytes = sizeof(double) * NVAR * pk->views[b].g.nz;
    const double* src = d_prims + pk->prim_off[b];
    if (hipMemcpyAsync(pk->views[b].P, src, bytes, hipMemcpyDeviceToDevice, pk->stream) != hipSuccess ||
        hipMemcpyAsync(pk->views[b].P1, src, bytes, hipMemcpyDeviceToDevice, pk->stream) != hipSuccess)
      return GRMHD_E_HIP;
  }
  return GRMHD_OK;
}

int grmhd_pack_step(grmhd_pack* pk, double dt) {
  if (!pk || !(dt > 0.0) || !isfinite(dt)) return GRMHD_E_ARG;
  int rc;
  for (int stage = 1; stage <= 2; stage++) {
    rc = pk->params.recon == GRMHD_RECON_MC ? pack_launch<GRMHD_RECON_MC>(pk, stage, dt)
                                            : pack_launch<GRMHD_RECON_WENO5>(pk, stage, dt);
    if (rc) return rc;
  }
  return GRMHD_OK;
}

int grmhd_pack_get_prims(grmhd_pack* pk, double* d_out) {
  if (!pk || !d_out) return GRMHD_E_ARG;
  for (int b = 0; b < pk->nb; b++) {
    size_t bytes = sizeof(double) * NVAR * pk->views[b].g.nz;
    if (hipMemcpyAsync(d_out + pk->prim_off[b], pk->views[b].P, bytes, hipMemcpyDeviceToDevice, pk->stream) !=
        hipSuccess)
      return GRMHD_E_HIP;
  }
  return GRMHD_OK;
}

int grmhd_pack_get_status(grmhd_pack* pk, long long* n_inv_fail) {
  if (!pk || !n_inv_fail) return GRMHD_E_ARG;
  unsigned long long f = 0;
  if (hipMemcpyAsync(&f, pk->d_fails, sizeof(f), hipMemcpyDeviceToHost, pk->stream) != hipSuccess ||
      hipStreamSynchronize(pk->stream) != hipSuccess)
    return GRMHD_E_HIP;
  *n_inv_fail = (long long)f;
  return GRMHD_OK;
}

int grmhd_pack_info(grmhd_pack* pk, int* grid_blocks, long long* prim_doubles) {
  if (!pk || !grid_blocks || !prim_doubles) return GRMHD_E_ARG;
  *grid_blocks = pk->items[PH_FLUX] + pk->items[PH_EMF] + pk->items[PH_UPDATE];
  *prim_doubles = pk->prim_total;
  return GRMHD_OK;
}

size_t grmhd_pack_exchange_bytes(const grmhd_grid* global) {
  if (!global || global->n1 < 1 || global->n2 < 1 || global->n3 < 1) return 0;
  return sizeof(int) * (size_t)global->n1 * global->n2 * global->n3;
}

int grmhd_pack_set_exchange(grmhd_pack* pk, void* d_map, size_t map_bytes) {
  if (!pk) return GRMHD_E_ARG;
  if (!d_map) {
    pk->d_owner = nullptr;
    return GRMHD_OK;
  }
  const grmhd_grid& G = pk->global;
  if (((uintptr_t)d_map & 3) != 0 || pk->nb > 65535) return GRMHD_E_ARG;
  if (map_bytes < grmhd_pack_exchange_bytes(&G)) return GRMHD_E_NOMEM;
  std::vector<int> own((size_t)G.n1 * G.n2 * G.n3, -1);
  for (int b = 0; b < pk->nb; b++) {
    const BlockView& v = pk->views[b];
    const int n = v.g.n1;
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
          int& o = own[((size_t)(k + v.o3) * G.n2 + (j + v.o2)) * G.n1 + (i + v.o1)];
          if (o >= 0) return GRMHD_E_ARG;  // blocks overlap
          o = b;
        }
  }
  if (hipStreamSynchronize(pk->stream) != hipSuccess ||
      hipMemcpy(d_map, own.data(), sizeof(int) * own.size(), hipMemcpyHostToDevice) != hipSuccess)
    return GRMHD_E_HIP;
  pk->d_owner = (int*)d_map;
  return GRMHD_OK;
}

int grmhd_pack_destroy(grmhd_pack* pk) {
  if (!pk) return GRMHD_E_ARG;
  delete pk;
  return GRMHD_OK;
}

}  // extern "C"
