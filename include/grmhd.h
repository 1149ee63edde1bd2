/* grmhd.h -- C ABI of the MI355X (gfx950) HARM ideal-GRMHD step.
 *
 * One call advances every zone of a logically Cartesian grid by one
 * two-stage SSP Runge-Kutta step of the HARM scheme (Algorithm section of the
 * KHARMA paper): linear-MC or WENO5 reconstruction, local Lax-Friedrichs
 * fluxes of the ideal stress-energy tensor (EGRMHD section, ideal part),
 * Flux-CT magnetic-field transport, geometric source terms from cached
 * metric derivatives (Core section, GRCoordinates), and the 1D_W
 * conserved->primitive inversion named in the Algorithm and Performance
 * sections (or, selected per context, the bracketed Kastaun et al. 2021
 * recovery the Algorithm section lists among the robust ones).  Metrics: flat Minkowski (Cartesian) or Kerr (M = 1) in modified
 * Kerr-Schild coordinates r = exp(x1), theta = pi x2 + (1-h)/2 sin(2 pi x2),
 * phi = x3.
 *
 * Conventions
 *   - State ("prims"): float64 array [8][n3+6][n2+6][n1+6], x1 fastest,
 *     variables (rho, u, u~1, u~2, u~3, B1, B2, B3); u~ is the velocity
 *     relative to the normal observer, B^i = *F^{it}.  Three ghost layers
 *     per side.  The flux array of debug calls is [3][8][same].
 *   - Every pointer marked "device" is device memory the caller owns (in
 *     practice torch tensors).  The library never allocates device memory:
 *     all scratch lives in the caller's workspace of grmhd_workspace_bytes()
 *     bytes, borrowed for the context's lifetime.
 *   - All work is enqueued on the hipStream_t given at creation, in order.
 *     Calls that return host values (estimate_dt, last_dt, divb, get_status,
 *     cons_to_prims' count) synchronise that stream; the rest are
 *     asynchronous.
 *   - Every function returns 0 (GRMHD_OK) or a negative GRMHD_E_* code and
 *     never throws; grmhd_strerror() names the code.  A context is not
 *     thread-safe.
 *   - A zone whose inversion fails is not an error: it keeps its stage-input
 *     hydro prims (B always follows the conserved field) and is counted.
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GRMHD_OK = 0, GRMHD_E_ARG = -1, GRMHD_E_HIP = -2, GRMHD_E_STATE = -3,
       GRMHD_E_NOMEM = -4 };
enum { GRMHD_METRIC_MINKOWSKI = 0, GRMHD_METRIC_KERR_MKS = 1 };
enum { GRMHD_RECON_MC = 0, GRMHD_RECON_WENO5 = 1, GRMHD_RECON_DONOR = 2, GRMHD_RECON_WENOZ = 3,
       GRMHD_RECON_VL = 4, GRMHD_RECON_MP5 = 5, GRMHD_RECON_PPM = 6, GRMHD_RECON_PPMX = 7 };
enum { GRMHD_PREC_FP64 = 0, GRMHD_PREC_MIXED = 1 };
enum { GRMHD_INV_1DW = 0, GRMHD_INV_KASTAUN = 1, GRMHD_INV_IMPLICIT = 2 };
enum { GRMHD_CT_FLUX = 0, GRMHD_CT_FACE_AVG = 1, GRMHD_CT_FACE_GS = 2 };
enum { GRMHD_INTEG_SSPRK2 = 0, GRMHD_INTEG_PC = 1, GRMHD_INTEG_RK1 = 2, GRMHD_INTEG_SSPRK54 = 3 };
enum { GRMHD_BC_PERIODIC = 0, GRMHD_BC_OUTFLOW = 1, GRMHD_BC_POLAR = 2,
       GRMHD_BC_FROZEN = 3 };

typedef struct grmhd_ctx grmhd_ctx;

/* Interior zone counts and coordinate extents; bc order x1-,x1+,x2-,x2+,x3-,x3+.
 * ng must be 3.  Periodic axes need n >= 1, polar axes n >= 3.  In modified
 * KS an x2 boundary at exactly 0 or 1 is the polar axis: its faces carry no
 * flux and its edges no EMF, whatever the ghost treatment. */
typedef struct {
  int n1, n2, n3, ng;
  double x1min, x1max, x2min, x2max, x3min, x3max;
  int bc[6];
} grmhd_grid;

typedef struct {
  int metric;     /* GRMHD_METRIC_* */
  double a;       /* black-hole spin (Kerr only) */
  double hslope;  /* theta squeeze h of modified KS */
} grmhd_metric;

typedef struct {
  double gamma_ad;    /* adiabatic index, p = (gamma_ad - 1) u */
  double cfl;         /* Courant number of grmhd_estimate_dt */
  double weno_eps;    /* WENO5 / WENO-Z smoothness regulariser, in [1e-36, 1]
                         when either is selected */
  double newton_tol;  /* relative |dW/W| stopping tolerance of 1D_W */
  int newton_maxit;   /* Newton iteration cap (one more step follows convergence) */
  int recon;          /* GRMHD_RECON_*: MC, WENO5, or DONOR (first order: each
                         face's states are its two zones' own values); or two
                         more of the schemes the Solvers section lists: WENOZ
                         (WENO-Z weights d_k (1 + (tau5/(eps + beta_k))^2),
                         Borges et al. 2008 with the power of Castro, Costa &
                         Don 2011), VL (linear, van Leer's harmonic-mean
                         limiter), MP5 (Suresh & Huynh 1997, alpha = 4) and
                         PPM (Colella & Woodward 1984, monotonised-central
                         slopes and their parabola limiter), PPMX (PPM with
                         the extremum-preserving limiter of Colella & Sekora
                         2008, C = 1.25).  Packs and the adjoint take MC or
                         WENO5. */
  int precision;      /* GRMHD_PREC_*: MIXED = FP32 reconstruction, fluxes, EMFs */
  int floors;         /* 1: floors and ceilings after every inversion (fields
                         below); 0: none */
  int inverter;       /* GRMHD_INV_*: 1D_W Newton from the stage-input prims,
                         or the Kastaun et al. root bracket in mu = 1/(h W),
                         which needs no guess (Illinois iteration stopped at
                         |d mu| <= newton_tol mu, at most 4 newton_maxit
                         iterations), or IMPLICIT: the implicit solver's
                         per-zone Newton on U(P) = U* over (rho, u, u~)
                         (Implicit Solver section: secant Jacobian, QR with
                         column pivoting, backtracking line search; step
                         tolerance max(newton_tol, 1e-12)), run as a pass of
                         its own after the update (not with fofc); all leave
                         a failed zone at its guess */
  double kastaun_wmax; /* Lorentz-factor cap of the Kastaun recovery (> 1);
                          ignored by 1D_W */
  /* Floors (Physics section: material and energy injected where density or
   * internal energy fall below set values or too far below the magnetic
   * pressure, in the drift frame).  After each stage's inversion:
   *   rho_fl = max(rho_min_geom r^-3/2, b^2/bsq_over_rho_max),
   *   u_fl   = max(u_min_geom r^-5/2,   b^2/bsq_over_u_max)
   * (r = exp(x1) in modified KS, 1 in flat space); the missing material
   * moves with the E x B drift velocity, is added as conserved variables
   * and the sum re-inverted (fluid-frame fallback if that fails); then the
   * Lorentz factor is capped at gamma_max and u/rho at u_over_rho_max.  All
   * must be > 0 (gamma_max > 1) when floors = 1. */
  double rho_min_geom, u_min_geom, bsq_over_rho_max, bsq_over_u_max;
  double u_over_rho_max, gamma_max;
  int fofc;           /* 1: first-order flux correction (Algorithm section,
                         after Beckwith & Stone 2011): each stage is first
                         taken with the high-order fluxes; zones whose
                         inversion fails or that floors act on are marked,
                         every face of a marked zone gets the LLF flux of
                         donor-cell states, Flux-CT and the update are
                         redone (only when some zone was marked).  Single
                         grids only (packs and the VJP reject it). */
  int ct;             /* GRMHD_CT_*: magnetic-field transport.  FLUX: Flux-CT
                         (Toth 2000; B lives in the zone prims).  FACE_AVG /
                         FACE_GS: face-centred constrained transport (the
                         Stone & Gardiner scheme the Algorithm section names),
                         the state's field being phi_d = sqrt(-g) B^d on the
                         lower d-face of every zone (grmhd_load_faces), the
                         zone B its faces' mean; edge EMFs are the average
                         of the four face EMFs (AVG) or that average with
                         Gardiner & Stone (2005) upwinded gradient terms
                         from zone-centre EMFs, chosen by the sign of the
                         mass flux (GS).  The face divergence is kept to
                         roundoff.  Single grids only. */
  int integrator;     /* GRMHD_INTEG_*: the time integrator (Solvers section's
                         list).  SSPRK2 (the default and the only one packs,
                         the VJP and the options above take); PC: predictor-
                         corrector, U* = U^n + (dt/2) L(P^n), then
                         U^{n+1} = U^n + dt L(P*); RK1: forward Euler, one
                         stage per step; SSPRK54: the five-stage fourth-order
                         SSP Runge-Kutta method of Spiteri & Ruuth (2002) in
                         Shu-Osher form (three conserved-variable registers
                         in the workspace instead of one; every stage
                         inverts its U).  PC, RK1 and SSPRK54 need Flux-CT
                         without floors, the correction or the implicit
                         recovery. */
  int egrmhd;         /* 1: Extended GRMHD (Implicit Solver and Extended Theory
                         section): two more zone-centred variables, the
                         rescaled heat flux qt = q (tau_R/(chi rho Theta^2))^1/2
                         and pressure anisotropy dPt = dP (tau_R/(nu rho
                         Theta))^1/2, Theta = p/rho, with their stress-energy
                         terms q^mu u_nu + q_nu u^mu - dP (bh^mu bh_nu - h^mu_nu/3)
                         (bh = b/|b|, h = delta + u u; none where b^2 = 0) and
                         the damped evolution d_mu(X u^mu) = -(X - X0)/tau_R +
                         (X/2) div u toward the Chandra et al. (2015) targets
                         X0 (from centred spatial gradients of the stage's
                         explicit state, time derivatives left out); div u's
                         time part, the relaxation and X are implicit.  Each
                         stage of the predictor-corrector (integrator must be
                         PC) solves every zone for the hydro prims and X with
                         the implicit solver's Newton (the X equations are
                         linear given the hydro state and are solved within
                         each residual); the inverter field is not used.
                         FP64, Flux-CT, MC or WENO5, no floors or correction,
                         single grids; extra state via grmhd_load_extended. */
  double tau_r, chi_emhd, nu_emhd;  /* Extended GRMHD closure constants: tau_R > 0,
                                       chi >= 0, nu >= 0 */
} grmhd_params;

/* Bytes of device workspace a context with this grid and parameters needs. */
size_t grmhd_workspace_bytes(const grmhd_grid* grid, const grmhd_params* params);

/* Create a context over caller-owned device workspace (>= grmhd_workspace_bytes,
 * 256-byte aligned) and a hipStream_t (NULL = default stream).  Computes the
 * geometry tables on the device (metric at zone centres, faces and corners of
 * every (x1, x2) column; at zone centres also the x1 and x2 derivatives of the
 * metric, which the geometric source contracts with the stress-energy
 * tensor, and the connection, which Extended GRMHD and the adjoint read).
 * E_ARG on bad sizes or enums. */
int grmhd_create(grmhd_ctx** out, const grmhd_grid* grid, const grmhd_metric* metric,
                 const grmhd_params* params, void* d_workspace, size_t ws_bytes,
                 void* hip_stream);

/* Copy padded prims (device, layout above) into the context's state: the
 * primitive state a step treats as fundamental (Glue section: the step
 * type that exchanges primitive variables; Physics section: the GRMHD
 * package's rho, u, velocity, with the field of the transport); with
 * get_prims it is also the checkpoint a restart reloads.  With face-centred
 * CT and faces loaded, the interior zones' B is then set to their faces'
 * mean. */
int grmhd_load_prims(grmhd_ctx* ctx, const double* d_prims);

/* Extended GRMHD only (E_STATE otherwise).  The two extra variables as
 * float64 [2][n3+6][n2+6][n1+6] (device): the rescaled heat flux, then the
 * rescaled pressure anisotropy.  load copies them into the state (zero after
 * creation); get copies the state's out, ghosts filled (periodic, outflow
 * and polar maps as for rho, no sign flips). */
int grmhd_load_extended(grmhd_ctx* ctx, const double* d_extra);
int grmhd_get_extended(grmhd_ctx* ctx, double* d_extra);

/* Face-centred CT only (E_STATE otherwise).  Face fields: float64
 * [3][n3+6][n2+6][n1+6] (device), component d holding sqrt(-g) B^d on the
 * lower d-face of every padded zone; ghost faces are refilled from the
 * boundary conditions before use (frozen ghosts are kept).  load copies
 * them into the state and sets the interior zones' B prims to the faces'
 * mean (steps return E_STATE until faces are loaded); get copies the
 * state's faces out (ghosts filled); face_divb reduces the face divergence
 * sum_d (phi_d(+) - phi_d(-))/dx_d over interior zones (max and mean of its
 * magnitude; synchronises). */
int grmhd_load_faces(grmhd_ctx* ctx, const double* d_faces);
int grmhd_get_faces(grmhd_ctx* ctx, double* d_faces);
int grmhd_face_divb(grmhd_ctx* ctx, double* max_out, double* mean_out);

/* One SSPRK2 step of size dt: U1 = Un + dt L(Pn), P1 = U_to_P(U1; Pn);
 * Un+1 = (Un + U1)/2 + dt L(P1)/2, Pn+1 = U_to_P(Un+1; P1).  Ghosts are
 * refilled before each stage.  Asynchronous. */
int grmhd_step(grmhd_ctx* ctx, double dt);

/* CFL step: cfl / max over interior zones of sum_d max|c+-_d| / dx_d (axes
 * with more than one zone), from the current prims (the global reduction of
 * the Core section's Reductions package, over the fast-magnetosonic speeds
 * the Solvers section's flux kernels evaluate).  Synchronises. */
int grmhd_estimate_dt(grmhd_ctx* ctx, double* dt_out);

/* The CFL step of grmhd_estimate_dt for a prims array d_prims (device,
 * padded layout; only interior zones are read), without a context and
 * without allocating anything: for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid it).  The zone-centre metric is evaluated in place, so the result
 * equals grmhd_estimate_dt's on a context of the same grid, metric and
 * parameters holding the same prims.  The reduction's scratch is a fixed
 * device array of the library (2048 workgroup maxima plus four results,
 * 16.4 KB per GPU, held until the process ends); the reduction strides over
 * the grid, so every grid grmhd_create accepts fits it.  hip_stream: a
 * stream of the current device (NULL = default); the call synchronises it.
 * All calls on one GPU share that scratch: calls that overlap on one GPU
 * (several host threads or streams) race and must be serialised by the
 * caller.  E_ARG for bad sizes or enums, E_STATE when the maximum signal
 * rate is not positive and finite, E_HIP on a runtime error. */
int grmhd_cfl_dt_noalloc(const grmhd_grid* grid, const grmhd_metric* metric, const grmhd_params* params,
                         const double* d_prims, double* dt_out, void* hip_stream);

/* One step of the CFL size without a host round trip: the dt reduction of
 * grmhd_estimate_dt runs on the device and both stages read its result there
 * (the per-step global dt of the Core section's reductions).  Asynchronous.
 * If the maximum signal rate is not positive and finite the step is taken
 * with dt = 0 (state unchanged) and grmhd_last_dt reports E_STATE. */
int grmhd_step_cfl(grmhd_ctx* ctx);

/* The dt of the last reduction (grmhd_step_cfl or grmhd_estimate_dt) to
 * *dt_out (host); E_STATE if it was not usable.  Synchronises. */
int grmhd_last_dt(grmhd_ctx* ctx, double* dt_out);

/* Copy the current padded prims (ghosts filled) to device memory d_out (the
 * primitive state of the Glue section's step; with load_prims, the
 * checkpoint). */
int grmhd_get_prims(grmhd_ctx* ctx, double* d_out);

/* Corner-centred div B of the current state, |div| / sqrt(-g) at interior
 * corners (corners on non-periodic boundaries excluded): max and mean to the
 * host (the divergence diagnostic of the Extras section's field transports,
 * in the corner form Flux-CT keeps at roundoff, Algorithm section); the
 * per-corner field to d_divb (device, padded scalar layout) unless it is
 * NULL.  Synchronises. */
int grmhd_divb(grmhd_ctx* ctx, double* d_divb_or_null, double* max_out, double* mean_out);

/* Inversion failures accumulated since creation (or the last reset), and
 * zones the floors acted on (per stage): the failure and floor-hit counts
 * of the Physics section's Inverter and Floors packages, which the
 * Algorithm section's flux correction exists to reduce.  Synchronises. */
int grmhd_get_status(grmhd_ctx* ctx, long long* n_inv_fail, long long* n_floor);
/* All counters since creation (or the last reset), out[0..3]: inversion
 * failures, zones floors acted on, zones the first-order flux correction
 * marked, floor injections that fell back to the fluid frame (all counted
 * per stage).  Synchronises. */
int grmhd_get_counters(grmhd_ctx* ctx, long long* out4);
int grmhd_reset_status(grmhd_ctx* ctx);

/* Conserved variables at interior zone centres of d_prims into d_cons (both
 * device, padded layout; ghosts of d_cons untouched). */
int grmhd_prims_to_cons(grmhd_ctx* ctx, const double* d_prims, double* d_cons);

/* 1D_W inversion at interior zones: d_cons, d_guess -> d_prims, per-zone
 * failure flags (device int32, padded scalar layout, may be NULL); the
 * failure count to *n_fail.  Synchronises. */
int grmhd_cons_to_prims(grmhd_ctx* ctx, const double* d_cons, const double* d_guess,
                        double* d_prims, int* d_flags, long long* n_fail);

/* Face fluxes of one stage evaluated from d_prims (ghosts filled from it),
 * with Flux-CT applied to the B components of interior faces.  d_flux is
 * [3][8][padded] float64 (device); entries at positions other than interior
 * faces (x1 faces i in [0, n1], j < n2, k < n3, and likewise) are
 * unspecified.  The context's reconstruction is used; the first-order flux
 * correction is not applied (it depends on a provisional update), and with
 * face-centred CT the face fields are not read (these are the Flux-CT
 * fluxes of d_prims).  E_STATE for Extended GRMHD contexts.  For testing
 * and inspection. */
int grmhd_fluxes(grmhd_ctx* ctx, const double* d_prims, double* d_flux);

/* Adjoint of one step (vector-Jacobian product), FP64 only.
 * Given the step's input prims d_prims_in (device, padded) and step size dt,
 * and the adjoint of its output prims d_gprims_out (device, padded; only
 * interior entries are read), writes the adjoint of the input prims to
 * d_gprims_in (device, padded; ghost entries zero: ghosts are functions of the
 * interior through the boundary conditions, frozen ghosts are constants) and
 * the derivative with respect to the adiabatic index to *g_gamma (host).
 * The step is recomputed from d_prims_in (per-step checkpointing); the
 * inversion is differentiated by the implicit-function theorem, limiter and
 * max() branches by the branch taken.  Scratch comes from d_vjp_ws (device,
 * 256-byte aligned, >= grmhd_vjp_workspace_bytes()).  Neither the context's
 * state nor its failure count changes.  Synchronises.  E_STATE for the mixed
 * precision path, floors, the first-order flux correction, a reconstruction
 * other than MC or WENO5, face-centred CT or the implicit recovery (the
 * adjoint covers the plain MC / WENO5 Flux-CT step; the workspace size is
 * then 0). */
size_t grmhd_vjp_workspace_bytes(const grmhd_grid* grid, const grmhd_params* params);
int grmhd_step_vjp(grmhd_ctx* ctx, const double* d_prims_in, double dt, const double* d_gprims_out,
                   double* d_gprims_in, double* g_gamma, void* d_vjp_ws, size_t vjp_ws_bytes);

/* ---- Batched uneven meshblock packs (FP64) ----
 * A pack holds nblocks cubic blocks of n[b]^3 zones, block b being the
 * sub-box starting at interior zone offsets_ijk[3b..3b+2] of the global grid
 * (same metric and parameters); every block has frozen (Dirichlet) ghost
 * zones unless the ghost exchange below is on, and x2 block faces on the
 * polar axis carry no flux.  Each RK2 stage of a pack step is three
 * launches (face fluxes, edge EMFs, zone update), each over the work items
 * of every block.
 * Packed prims: the blocks' padded arrays [8][n+6][n+6][n+6], concatenated in
 * block order (device).  Tile shapes per block size (t1*t2*t3 <= 256, or
 * (0, 0, 0): runs of 256 consecutive positions of each box in x1-fastest
 * order, the default) only change speed.  Errors as for single contexts; E_ARG for blocks outside the
 * global grid, a non-FP64 precision, floors, the first-order flux
 * correction, a reconstruction other than MC or WENO5, face-centred CT or
 * the implicit recovery (packs advance the plain MC / WENO5 Flux-CT
 * step). */
typedef struct grmhd_pack grmhd_pack;
size_t grmhd_pack_workspace_bytes(int nblocks, const int* n);
int grmhd_pack_create(grmhd_pack** out, int nblocks, const int* n, const int* offsets_ijk,
                      const grmhd_grid* global, const grmhd_metric* metric,
                      const grmhd_params* params, void* d_workspace, size_t ws_bytes,
                      void* hip_stream);
int grmhd_pack_set_tiles(grmhd_pack* pack, int n, int t1, int t2, int t3);
int grmhd_pack_load_prims(grmhd_pack* pack, const double* d_prims);
int grmhd_pack_step(grmhd_pack* pack, double dt);
int grmhd_pack_get_prims(grmhd_pack* pack, double* d_out);
int grmhd_pack_get_status(grmhd_pack* pack, long long* n_inv_fail);
/* Ghost exchange between the blocks of a pack (the paper's meshblocks with
 * boundary synchronisation each sub-step; Package structure and Glue
 * sections), on one GPU.  With it on, before each RK2 stage every ghost zone
 * of every block takes the value the single global grid would hold there:
 * the zone of the global grid at that position, mapped by the global
 * boundary conditions (periodic, outflow, polar mirror with u~2 and B2
 * flipped), read from the block that owns it; positions on frozen global
 * axes and zones no block owns keep their values.  Blocks that tile the
 * global grid then advance as the global grid does.  d_map (device, 4-byte
 * aligned, >= grmhd_pack_exchange_bytes(global) bytes, one int per global
 * interior zone) is filled here with the owner map (synchronises) and
 * borrowed while the exchange is on; d_map = NULL switches it off (frozen
 * ghosts, the default).  E_ARG for overlapping blocks or more than 65535
 * blocks, E_NOMEM for a short map. */
size_t grmhd_pack_exchange_bytes(const grmhd_grid* global);
int grmhd_pack_set_exchange(grmhd_pack* pack, void* d_map, size_t map_bytes);
/* Workgroups of one RK2 stage's three launches, and length (doubles) of
 * the packed prims. */
int grmhd_pack_info(grmhd_pack* pack, int* grid_blocks, long long* prim_doubles);
int grmhd_pack_destroy(grmhd_pack* pack);

/* Work order of the heavy kernels: each XCD takes a contiguous run of
 * workgroups in which kg consecutive x3 planes of one (x1, x2) chunk follow
 * each other (flux/EMF and update kernels separately; default 8).  Any
 * kg >= 1 gives the same results; only speed changes.  E_ARG if kg < 1. */
int grmhd_set_schedule(grmhd_ctx* ctx, int kg_flux, int kg_update);

/* Per-kernel-class timing of the classes whose bits are set in class_mask
 * (0 turns timing off, -1 times every class; setting a mask clears earlier
 * records): every launch of a timed class carries a start and a stop HIP
 * event in its own dispatch (hipExtLaunchKernel), so no marker packets are
 * added between kernels.  Classes: 0 ghost fill, 1 face fluxes (x1, x2 and
 * x3 faces in one launch), 2 EMFs, 3 stage-1 update, 4 stage-2 update, 5 dt
 * reduction, 6 the flux correction's donor-cell face fix, 7 floors, 8 the
 * face update of face-centred CT (its ghost faces count as 0, its zone-centre
 * and edge EMFs as 2).  The report sums elapsed milliseconds and counts
 * launches per class into arrays of nclass >= 9 entries.  Both synchronise
 * the stream.
 * For measurement; the step itself is unchanged. */
int grmhd_timing(grmhd_ctx* ctx, int class_mask);
int grmhd_timing_report(grmhd_ctx* ctx, double* total_ms, long long* launches, int nclass);

const char* grmhd_strerror(int code);

/* Release the host side of the context; the workspace stays the caller's. */
int grmhd_destroy(grmhd_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GRMHD_H */
