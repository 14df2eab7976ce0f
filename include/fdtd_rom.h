/*
 * fdtd_rom.h - C ABI of the MI355X (gfx950) library for the stable FDTD
 * method with embedded reduced-order models (Zhang, Bekmambetova, Triverio,
 * "A Stable FDTD Method with Embedded Reduced-Order Models", IEEE TAP 2017).
 *
 * Problem statement (paper Sec. II first paragraph, Sec. IV, Sec. IV-C last
 * paragraph): a 2D TEz coarse Yee grid with PEC walls and one or more
 * refined regions; each region is replaced by a reduced model with boundary
 * ports; at run time the coarse grid is advanced with the conventional
 * leap-frog updates (eqs. (3), (5)) and every reduced model, together with
 * the coarse electric field on its interface, with the explicit update of
 * eq. (23).
 *
 * Conventions shared by every entry point
 *   - coarse cell (i, j), 0 <= i < nx, 0 <= j < ny; host maps are row-major
 *     [j * nx + i];
 *   - Hz(i, j) at the cell centre; Ex(i, j), 0 <= j <= ny, on the horizontal
 *     edge y = j*dy; Ey(i, j), 0 <= i <= nx, on the vertical edge x = i*dx;
 *     PEC walls: Ex(., 0), Ex(., ny), Ey(0, .), Ey(nx, .) are zero;
 *   - leap-frog state after k steps: E at time k*dt, Hz at (k - 1/2)*dt;
 *   - a reduced region covers coarse cells [i0, i0+ni) x [j0, j0+nj); its
 *     np = 2*(ni+nj) ports are ordered South (Ex(i0+c, j0)), North
 *     (Ex(i0+c, j0+nj)), West (Ey(i0, j0+c)), East (Ey(i0+ni, j0+c)), c
 *     increasing along each side (the ordering of eq. (8) at coarse
 *     resolution);
 *   - every host pointer argument is borrowed: the library copies what it
 *     needs before the call returns;
 *   - functions return FDTD_OK (0) or a negative status; a thread-local
 *     message describing the last failure is available from
 *     fdtd_rom_last_error().  No C++ exception crosses this interface.
 */
#ifndef FDTD_ROM_H
#define FDTD_ROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FDTD_OK = 0,
  FDTD_EINVAL = -1,       /* invalid argument or geometry */
  FDTD_ENOMEM = -2,       /* workspace too small / host allocation failed */
  FDTD_EDEVICE = -3,      /* HIP runtime error */
  FDTD_ENOTPASSIVE = -4,  /* reduced model violates eq. (26a) at dt */
  FDTD_EUNSTABLE = -5,    /* non-finite field detected */
  FDTD_ESTATE = -6        /* call not valid in the current state */
};

enum { FDTD_F32 = 0, FDTD_F64 = 1 };
enum { FDTD_HZ = 0, FDTD_EX = 1, FDTD_EY = 2 };

/* Physical constants used by both the library and its validation. */
#define FDTD_C0 299792458.0
#define FDTD_MU0 (4.0e-7 * 3.14159265358979323846)

/* Coarse grid (eqs. (1), (3), (5)).  eps_r / sigma: host [ny*nx] relative
 * permittivity and conductivity (S/m) per cell; NULL means 1 / 0.  Edge
 * material is the mean over the two cells sharing the edge (eq. (3)).
 * dtype: FDTD_F32 or FDTD_F64 arithmetic and storage on the device.
 * pec: host [ny*nx], non-zero marks a perfectly conducting cell (metal such
 * as the irises of Sec. VI-B): its Hz and the E on its four edges stay zero
 * (their eps_r / sigma are not used); NULL means none.  A PEC cell may not
 * lie inside a reduced region; one on a region's ring faces a port that the
 * model must not drive (that port's column of Lt all zero, FDTD_EINVAL
 * otherwise), and sources and probes may not sit on its samples.
 * pitch_pad: device layout only - every field row is nx rounded up to 64
 * samples plus pitch_pad unused columns (a multiple of 64 in [0, 1024];
 * FDTD_EINVAL otherwise).  Results do not depend on it; the rate does, by a
 * few per cent, through how rows fall on the memory channels (4096^2 FP32:
 * 3.7 % faster with 64, 8192^2 FP32: 6-13 % slower).  0 is the default. */
typedef struct {
  int32_t nx, ny;
  double dx, dy, dt;
  int32_t dtype;
  const double* eps_r;
  const double* sigma;
  const uint8_t* pec;
  int32_t pitch_pad;
} fdtd_grid;

/* One embedded reduced model (eqs. (11)-(12)), built on coarse ports.
 * Rt, Ft: host [q*q] row-major (R~, F~ of eq. (11)); Lt: host [q*np]
 * row-major (L~ = V^T L); B~ = L~ Sc is implied with
 * Sc = diag(-dx I, +dx I, +dy I, -dy I) (coarse analog of eq. (25)).
 * x0: host [q] initial reduced state or NULL for zero; the interface E
 * starts at L~^T x0.  group >= 0: regions with the same group use one
 * copy of the matrices on the device (their Rt/Ft/Lt must be identical and
 * their surroundings must give identical interface half cells).
 * Limits: 1 <= q <= 16384, np = 2 (ni + nj) <= 1024, and q + np rounded up
 * to 64 must fit 64 KB of elements (16384 FP32, 8192 FP64: the coupling
 * workgroups stage [x~; h] in LDS), else FDTD_EINVAL. */
typedef struct {
  int32_t i0, j0, ni, nj;
  int32_t q;
  int32_t group;
  const double* Rt;
  const double* Ft;
  const double* Lt;
  const double* x0;
} fdtd_rom;

/* Additive source: at step n (0-based) incr[n] is added to component comp
 * over positions [i0, i1) x [j0, j1) - to Hz^{n+1/2} right after its update
 * (centred at t = n*dt) or to E^{n+1} right after its update.  nt >= the
 * number of steps the simulation will run (max_steps). */
typedef struct {
  int32_t comp, i0, i1, j0, j1;
  int32_t nt;
  const double* incr;
} fdtd_source;

/* Point probe: after step n, probe value n is Hz^{n+1/2}(i, j) or E^{n+1}. */
typedef struct {
  int32_t comp, i, j;
} fdtd_probe;

/* Absorbing layers (convolutional PML; not in the paper, whose waveguide
 * and reflection experiments of Sec. VI end in PML without equations).
 * n_xlo .. n_yhi: layer thickness in coarse cells on each side (0: that side
 * is a PEC wall; the outer face of a layer is PEC).  Inside a layer of D
 * cells, at depth ratio rho in (0, 1] (E samples at k*d, Hz at (k+1/2)*d):
 *   sigma = sigma_scale * 0.8 (m+1) / (eta0 d) * rho^m,
 *   kappa = 1 + (kappa_max - 1) rho^m,  alpha = alpha_max (1 - rho),
 *   b = exp(-(sigma/kappa + alpha) dt/eps0),
 *   a = sigma (b - 1) / (sigma kappa + kappa^2 alpha)  (0 where sigma = 0),
 * and every derivative of eqs. (3), (5) across the layer becomes
 * (1/kappa) dF + psi with psi' = b psi + a dF (dF the Yee difference, psi
 * carried per field sample).  Outside the layers the update is unchanged.
 * m <= 0 selects 3, kappa_max < 1 selects 1, alpha_max < 0 selects 0;
 * sigma_scale >= 0 as given (0: non-absorbing layers).  Reduced regions
 * and their one-cell rings must lie outside every layer (FDTD_EINVAL). */
typedef struct {
  int32_t n_xlo, n_xhi, n_ylo, n_yhi;
  double m, sigma_scale, kappa_max, alpha_max;
} fdtd_pml;

typedef struct {
  fdtd_grid grid;
  const fdtd_rom* roms;
  int32_t nroms;
  const fdtd_source* sources;
  int32_t nsources;
  const fdtd_probe* probes;
  int32_t nprobes;
  int32_t max_steps; /* capacity of the probe record and source tables */
  fdtd_pml pml;      /* all thicknesses 0: PEC walls on every side */
} fdtd_problem;

typedef struct fdtd_rom_sim fdtd_rom_sim; /* opaque, owned by the library */

/* Device workspace (bytes) that fdtd_rom_create needs for this problem:
 * two field sets (three on grids without absorbing layers, for the
 * two-step launches), the per-cell material, the models, the probe record
 * and the source tables. */
int fdtd_rom_workspace_size(const fdtd_problem* prob, size_t* bytes);

/* Validate the problem, fold the coarse interface half cells into the
 * closed form of eq. (23) (FP64 on the host), and lay the problem out in
 * the caller's device workspace.
 *   dev_workspace: device pointer, >= fdtd_rom_workspace_size bytes, 256-B
 *     aligned; owned by the caller and must outlive the handle.
 *   hip_stream: hipStream_t every launch and copy of this handle goes to
 *     (NULL = the default stream).
 * Every call on a handle runs on the device current on the calling thread,
 * which must be the device of its workspace and stream (the library never
 * switches devices).
 * Checks: dimensions > 0; dt <= the coarse CFL limit of eq. (1) with
 * c = c0/sqrt(min eps_r) (FDTD_EINVAL); every region at least one cell from
 * the walls and its one-cell ring disjoint from other regions (FDTD_EINVAL);
 * sources and probes on cells/edges updated by the coarse stencil
 * (FDTD_EINVAL); R~ symmetric to 1e-12 relative and positive definite by
 * Cholesky (eq. (26a), Theorem 1; FDTD_ENOTPASSIVE). */
int fdtd_rom_create(const fdtd_problem* prob, void* dev_workspace, size_t ws_bytes,
                    void* hip_stream, fdtd_rom_sim** out);

/* Advance one leap-frog step / nsteps steps (asynchronous on the stream).
 * FDTD_ESTATE if the step count would exceed max_steps.
 * Periodic finiteness check (the method is stable by construction, Theorem
 * 2, so a non-finite value means bad inputs - a source increment, a model
 * that is not passive - or an unstable configuration): every K steps
 * (fdtd_rom_set_check_interval, default K = 1024, counted across calls)
 * run() launches a kernel that reads the whole current field set (3 * 4 or
 * 8 bytes per cell, about 0.1 % of K steps' traffic) and raises a device
 * flag on any NaN or infinity.  The check is ordered on the stream between
 * graph replays (it is never captured).  A run() call that launched a check
 * synchronises the stream before it returns and reports a raised flag as
 * FDTD_EUNSTABLE; the steps have been taken, the flag stays raised (every
 * later call that checks reports it again) until fdtd_rom_set_state.
 * Calls that launch no check stay asynchronous. */
int fdtd_rom_step(fdtd_rom_sim* sim);
int fdtd_rom_run(fdtd_rom_sim* sim, int32_t nsteps);

/* Check interval K in steps (0 disables the check; FDTD_EINVAL if < 0);
 * setting it restarts the count. */
int fdtd_rom_set_check_interval(fdtd_rom_sim* sim, int32_t every);
int fdtd_rom_get_check_interval(const fdtd_rom_sim* sim, int32_t* every);

/* Do the set-up the next fdtd_rom_run(sim, nsteps) would do before its
 * first launch (two-step tile roles; capture of the graph batch it will
 * replay, when graphs are on and nsteps >= the batch), without taking a
 * step, so that a timed run starts with launches only.  Synchronises if
 * it uploads tile roles. */
int fdtd_rom_prepare_run(fdtd_rom_sim* sim, int32_t nsteps);

/* Number of steps taken so far. */
int fdtd_rom_steps_done(const fdtd_rom_sim* sim, int32_t* n);

/* Probe record rows [first, first+count) into host [count * nprobes]
 * (row-major, probe index fastest), converted to double.  Synchronises the
 * stream. */
int fdtd_rom_read_probes(const fdtd_rom_sim* sim, int32_t first, int32_t count,
                         double* host_out);

/* Probe-energy objective of the recorded run, the J of fdtd_rom_adjoint:
 * J = dt * sum_{n = first}^{first+count-1} (probe row n of Hz probe p)^2,
 * summed in FP64 on the host from the probe record.  FDTD_EINVAL if p is
 * not an Hz probe or the rows were not recorded; FDTD_EUNSTABLE if a value
 * is not finite.  Synchronises the stream. */
int fdtd_rom_probe_objective(const fdtd_rom_sim* sim, int32_t probe, int32_t first, int32_t count,
                             double* J);

/* Current field comp in the natural layout into host memory:
 * Hz [ny*nx], Ex [(ny+1)*nx], Ey [ny*(nx+1)] (walls included, zero).
 * Cells and edges inside reduced regions read as zero.  Synchronises. */
int fdtd_rom_read_field(const fdtd_rom_sim* sim, int32_t comp, double* host_out);

/* Reduced state x~ of region k into host [q].  Synchronises. */
int fdtd_rom_read_rom_state(const fdtd_rom_sim* sim, int32_t k, double* host_out);

/* Discrete energy of the current state (E^n, Hz^{n-1/2}, x~^n): the storage
 * function of Theorem 2 (appendix), x^T R x with R the coarse analog of
 * eq. (7)'s R plus every model's x~^T R~ x~:
 *   sum over stored E edges of (eps/dt) * (dual area) * E^2, where the dual
 *     area is dx*dy for an edge between two coarse cells and the outer half
 *     cell dx*dy/2 for an interface edge (eq. (13));
 *   + sum over coarse cells of (mu0/dt) * dx*dy * Hz^2;
 *   - E^T K Hz over those edges (K the coarse curl of eq. (7), lengths dx
 *     for Ex and dy for Ey);
 *   + sum over models of x~^T R~ x~.
 * Constant for lossless runs without sources and non-increasing with loss
 * (Theorem 2); with absorbing layers it is this same coarse-grid function
 * (the layers' auxiliary state is not part of it).  Coarse part reduced on the device in FP64, models on the
 * host.  Synchronises; FDTD_EUNSTABLE if non-finite. */
int fdtd_rom_energy(const fdtd_rom_sim* sim, double* e);

/* Checkpoint / resume.  state_size: bytes of a state blob (a 256-byte
 * header with the step count and shape, the current field set in device
 * layout, every model's reduced state, the absorbing layers' auxiliary
 * fields if any).  get_state copies the handle's
 * current state into dev_dst (device memory, 256-B aligned, caller-owned);
 * set_state makes a blob from a handle of the same problem shape the current
 * state, including its step count (FDTD_EINVAL on a shape or dtype mismatch
 * or a step count beyond max_steps).  Probe rows already recorded are kept;
 * rows from the restored step on are overwritten by the next run.  Both
 * synchronise. */
int fdtd_rom_state_size(const fdtd_rom_sim* sim, size_t* bytes);
int fdtd_rom_get_state(const fdtd_rom_sim* sim, void* dev_dst);
int fdtd_rom_set_state(fdtd_rom_sim* sim, const void* dev_src);

/* Host-only (no device call): validate prob like fdtd_rom_create and
 * return, for region k, the FP64 closed-form matrices of eq. (23) that
 * create folds from eqs. (13)-(22):
 *   A~  = (R~ + F~ + L~ C+ L~^T)^{-1} (R~ - F~ + L~ C- L~^T)   [q*q]
 *   B~' = (R~ + F~ + L~ C+ L~^T)^{-1} L~ Sc                     [q*np]
 *   C~  = L~^T                                                   [np*q]
 * with C+- = Dl Dl' (eps/dt +- sigma/2) of the coarse half cell outside each
 * port (eq. (13)).  Row-major host buffers; any may be NULL. */
int fdtd_rom_coupled_update(const fdtd_problem* prob, int32_t k, double* A, double* B,
                            double* C);

/* Reduced model of one refined region, built on the host in FP64 (paper
 * Sec. II eqs. (2)-(8), Sec. III eqs. (9)-(12), Sec. V-E eq. (27)):
 *   1. the fine TEz model of the region (r*ni x r*nj cells of dx/r x dy/r,
 *      boundary half cells and hanging variables, eqs. (3)-(8)), with the r
 *      fine boundary E samples of each coarse interface edge tied together
 *      (interpolation rule eq. (15) applied before reduction), so that the
 *      model has np = 2(ni+nj) coarse ports, input matrix Lc Sc;
 *   2. block Krylov directions of (p0 R + F)^{-1} R from (p0 R + F)^{-1} B
 *      at p0 = pi * f_max * dt, each block orthogonalised against earlier
 *      directions in the mass inner product diag(De, Dm)/dt and ordered by
 *      decreasing mass norm;
 *   3. SPRIM split (eq. (9)): V1 = the E rows, V2 = the H rows of those
 *      directions, Gram-Schmidt in order, q1 = ceil(q/2), q2 = floor(q/2);
 *   4. congruence R~ = V^T R V, F~ = V^T F V, L~ = V^T Lc (eqs. (11)-(12));
 *   5. if clip != 0 and the largest singular value of
 *      R11^{-1/2} K~ R22^{-1/2} exceeds theta * 2/dt (eq. (27)), the
 *      singular values above that bound are lowered to it and K~ is
 *      replaced in R~ and F~ (theta <= 0 selects 0.99).
 * basis 1 replaces steps 2-4 by V = I (no reduction: R~, F~, L~ are the
 * restricted fine model's own, q must equal its state count); with clip
 * this is the paper's "CFL extension only" configuration (Tabs. I-III), with
 * basis 0 and clip = 0 at dt within the fine limit its "MOR only" one.
 * eps_r, sigma: host fine-cell maps [(r*nj) * (r*ni)], row-major.
 * pec: host fine-cell map of the same shape, non-zero marks a perfectly
 * conducting fine cell (NULL: none).  Its Hz and the E on its edges are zero
 * and are left out of the fine model; a coarse port whose r fine edges all
 * lie on PEC cells has no coordinate (its column of Lt is zero), and a port
 * with only some of them on PEC cells is rejected (FDTD_EINVAL: eq. (15)
 * ties the r fine edges to one value).
 * Outputs (caller-allocated, row-major): Rt [q*q], Ft [q*q], Lt [q*np];
 * state order: q1 E coordinates then q2 H coordinates.  With Rt, Ft and Lt
 * all NULL the call only fills info (q1, q2 and the restricted state count
 * for these parameters).  FDTD_EINVAL if the Krylov space deflates below q.
 * Thread-safe (no shared state). */
typedef struct {
  int32_t ni, nj, r;
  double dx, dy, dt;
  const double* eps_r;
  const double* sigma;
  int32_t q;
  double f_max;
  double theta;
  int32_t clip;
  int32_t basis;  /* 0: SPRIM (steps 2-4), 1: identity */
  const uint8_t* pec;
} fdtd_rom_build_params;

typedef struct {
  int32_t q1, q2;
  double p0;
  double smax_before, smax_after; /* largest s_k of eq. (27) before/after */
  int32_t clipped;
  int32_t n_fine_states;          /* size of the restricted fine model */
} fdtd_rom_build_info;

int fdtd_rom_build(const fdtd_rom_build_params* params, double* Rt, double* Ft, double* Lt,
                   fdtd_rom_build_info* info);

/* Gradient through the model builder: given dJ/dR~ and dJ/dF~ of the model
 * fdtd_rom_build makes from params (e.g. from fdtd_rom_adjoint_models), the
 * gradient of J with respect to the fine cells' eps_r and sigma, with the
 * projection basis V = blkdiag(V1, V2) held at the one built from params
 * (the parametric model R~(p) = V^T R(p) V; for basis 1 nothing is held).
 * Steps, reversed: the eq. (27) clip when it is active (K~_c =
 * R11^{1/2} M g(M^T M) R22^{1/2}, M = R11^{-1/2} K~ R22^{-1/2},
 * g(mu) = min(1, lim / sqrt(mu)), lim = theta 2/dt; only R11 = dt R~11
 * depends on the material, its path goes through the eigen-decompositions
 * of R11 and M^T M by the Daleckii-Krein rule), the congruence of
 * eqs. (11)-(12) (dJ/dDe_e = (V1 dR~11 V1^T)_ee / dt,
 * dJ/dDs_e = (V1 dF~11 V1^T)_ee / 2 per fine edge coordinate), then eqs.
 * (3)-(4): each fine edge holds half the cell area of each adjacent fine
 * cell (De = area/2 eps0 eps_r, Ds = area/2 sigma per cell).  L~ does not
 * depend on the material.  The result depends on V only through its
 * column spaces.  PEC fine cells report zero.
 *   grad_Rt, grad_Ft: host [q*q] row-major; outputs grad_eps_r, grad_sigma:
 *   host fine maps [(r*nj) * (r*ni)], caller-allocated.  Same errors as
 *   fdtd_rom_build, plus FDTD_EINVAL if an eigen-decomposition of the clip
 *   does not converge.  Thread-safe. */
int fdtd_rom_build_vjp(const fdtd_rom_build_params* params, const double* grad_Rt, const double* grad_Ft,
                       double* grad_eps_r, double* grad_sigma);

/* The builder's state kept for its gradient (same steps as
 * fdtd_rom_build_vjp without rebuilding the model: the fine model, the E
 * basis V1, K~ before the clip and the clip's limit stay on the host).
 * fdtd_rom_build_keep: fdtd_rom_build (same arguments, outputs and errors;
 * Rt, Ft, Lt required) that also returns *state, owned by the caller until
 * fdtd_rom_model_state_free (tens of MB for a 128x128-cell region: the basis
 * over every fine edge).  fdtd_rom_model_state_vjp: fdtd_rom_build_vjp's
 * result for the model the state was built with (bit for bit), sizes as
 * there; the state is read only, so calls on one state may run in parallel
 * threads. */
typedef struct fdtd_rom_model_state fdtd_rom_model_state;
int fdtd_rom_build_keep(const fdtd_rom_build_params* params, double* Rt, double* Ft, double* Lt,
                        fdtd_rom_build_info* info, fdtd_rom_model_state** state);
int fdtd_rom_model_state_vjp(const fdtd_rom_model_state* state, const double* grad_Rt, const double* grad_Ft,
                             double* grad_eps_r, double* grad_sigma);
void fdtd_rom_model_state_free(fdtd_rom_model_state* state);

/* Per-kernel timing with HIP events on the handle's stream.  One step is
 * one launch of the step kernel (coarse stencil, every model's eq. (23)
 * update and the probe record run as concurrent workgroups of that launch);
 * with two steps per pass (fdtd_rom_set_time_blocking) one unit is the pair
 * of launches that advances two steps.  Each run() call ends with a
 * probe-flush and a step-counter launch.  While enabled, every unit and
 * every end-of-run pair are bracketed by events; fdtd_rom_profile_read
 * synchronises and returns the summed durations (ms) and counts since the
 * last read (step_launches counts units: a pair counts once). */
int fdtd_rom_profile_enable(fdtd_rom_sim* sim, int32_t enable);
int fdtd_rom_profile_read(fdtd_rom_sim* sim, double* step_ms, int64_t* step_launches,
                          double* tail_ms, int64_t* tail_launches);

/* Launch configuration.  set_tiling: rows each wave of a stencil tile
 * advances (4, 8, 16 or 32; the default depends on the grid: 16 for
 * cache-resident grids with >= 4096 waves, else 8 for large grids, 4 for
 * small ones).  set_graph: batch > 0 makes run()
 * replay a captured HIP graph of `batch` steps (capture happens on first use
 * on a library-owned stream, replay on the handle's stream; remainders and
 * profiled runs use direct launches); 0 (default) disables graphs. */
int fdtd_rom_set_tiling(fdtd_rom_sim* sim, int32_t seg);
int fdtd_rom_get_tiling(const fdtd_rom_sim* sim, int32_t* seg);

/* Regions sharing one model (same group >= 0, FP32, at least 8 of them,
 * q + np <= 512) are advanced by one FP32 MFMA GEMM per step over all copies
 * (eq. (23) for every copy at once) when enabled (default); disabled, every
 * region uses its own row-parallel GEMV.  Both give the same result up to
 * FP32 summation order. */
int fdtd_rom_set_shared_gemm(fdtd_rom_sim* sim, int32_t enable);

/* How the coarse stencil reads the per-cell material of eq. (3) (the edge
 * coefficients come from a = eps0 eps_r/dt and b = sigma/2 of the two cells
 * sharing an edge).  mode 1: a 16-bit index per cell into a table of the
 * problem's distinct (a, b) pairs - available when there are at most 65536
 * of them, and then the default; mode 0: the two per-cell arrays.  The
 * values are the same bit patterns, so both modes give identical results;
 * mode 1 moves 6 (FP32) or 14 (FP64) bytes fewer per cell update.
 * set: FDTD_EINVAL for another mode, or for mode 1 when no table exists.
 * get: the current mode and the table size (0: no table). */
int fdtd_rom_set_material_mode(fdtd_rom_sim* sim, int32_t mode);
int fdtd_rom_get_material_mode(fdtd_rom_sim* sim, int32_t* mode, int32_t* entries);
int fdtd_rom_set_graph(fdtd_rom_sim* sim, int32_t batch);

/* Two leap-frog steps (eq. (5) then eq. (3), twice) per pass over the
 * coarse grid.  on = 1: steps go in pairs of launches.  The first launch
 * runs the step-n coupling blocks of eq. (23) and advances the tiles of the
 * grid by two steps at once, holding step n+1 in registers - except, next
 * to each region, the band of ring cells and their edges, whose second step
 * needs the step-(n+1) interface E of eq. (23).  The second launch runs the
 * step-(n+1) coupling blocks, advances the bands by the second step and
 * takes a share of the far tiles (fdtd_rom_set_pair_split).  An odd last
 * step runs as a single launch.  On by default for grids without absorbing
 * layers (batches of such grids too).  The arithmetic per cell
 * is that of the single-step launch, so results are identical; far cells
 * move their fields through memory once per two steps.  Graph batches
 * (fdtd_rom_set_graph) are rounded down to a multiple of 4 steps.
 * set: synchronises the stream; FDTD_EINVAL for a value other than 0/1 or
 * for a grid with absorbing layers.  get: the current setting. */
int fdtd_rom_set_time_blocking(fdtd_rom_sim* sim, int32_t on);
int fdtd_rom_get_time_blocking(const fdtd_rom_sim* sim, int32_t* on);

/* Two steps per pass: the share of the far tiles (percent of the two-step
 * tiles, 0..90) that the second launch of each pair advances instead of the
 * first.  Far tiles read only step n and write step n+2, so either launch
 * may take them; in the second they run beside the coupling blocks of step
 * n+1, whose chain of dependent loads would otherwise run alone there.
 * -1 (default) picks 60 when the grid's tiles do not fit on the GPU at once
 * and a shared model runs as the MFMA GEMM (fdtd_rom_set_shared_gemm; its
 * blocks form the longest chain), else 0.  Results do not depend on it.  get: the share in
 * effect (after the next pair's set-up), else the requested value. */
int fdtd_rom_set_pair_split(fdtd_rom_sim* sim, int32_t percent);
int fdtd_rom_get_pair_split(const fdtd_rom_sim* sim, int32_t* percent);

/* Discrete adjoint (reverse-time sweep) of the coupled leap-frog run for the
 * objective J = dt * sum_{n=0}^{nsteps-1} (Hz_p^{n+1/2})^2 at Hz probe p:
 * the gradient of J with respect to the relative permittivity and the
 * conductivity of every coarse cell (Sec. II-A eqs. (3) and (5) transposed,
 * eq. (23) transposed with the reduced models held fixed).  The two cells
 * of an edge share its eq. (3) coefficients through the averages
 * a = eps0 mean(eps_r)/dt and b = mean(sigma)/2 (Ca = (a-b)/(a+b),
 * Cb = 1/(a+b)); cells inside a region or on its one-cell ring (whose
 * material is folded into the models' eq. (13) half cells) report zero.
 *
 * fdtd_rom_adjoint_workspace_size: device bytes the sweep needs for nsteps
 * with a checkpoint every ckpt_every steps (0 selects ceil(sqrt(nsteps))):
 * ceil(nsteps/ckpt_every) checkpoints of the fields and reduced states,
 * ckpt_every recomputed field sets (twice that with two or more segments:
 * the next segment's recompute fills the second set beside the reverse
 * steps of the current one), two adjoint field sets, the adjoint reduced
 * states, two FP64 per-cell accumulators and G^T of every model.
 * With absorbing layers a checkpoint also holds the four auxiliary fields,
 * a recomputed set the two at Ex and Ey, an adjoint set the adjoints of
 * all four (plus one private pair of the two at Hz).
 *
 * fdtd_rom_adjoint: runs the forward from the handle's initial state (the
 * handle must have taken no step; FDTD_ESTATE otherwise), keeping
 * checkpoints up to the last one, then sweeps back one segment at a time,
 * recomputing each segment's forward states from its checkpoint; the
 * recompute of the segment below runs on a second stream of the device
 * (default priority, created and destroyed by the call) while the reverse
 * steps of the current one run on the handle's stream, ordered by events.
 * Inside absorbing layers
 * the sweep transposes the auxiliary-field recursions as well, so the
 * gradient is that of the layered run (no material gradient of the layer
 * profiles themselves, which are fixed by fdtd_pml).  Afterwards the handle
 * stands at step nsteps with its probe record filled, as after
 * fdtd_rom_run(sim, nsteps).
 *   probe: index of an Hz probe of the problem (FDTD_EINVAL otherwise).
 *   dev_adj_ws: device pointer, 256-B aligned, >= the size above; caller's.
 *   J: host double; grad_eps_r, grad_sigma: host [ny*nx] row-major (cell
 *     (i,j) at j*nx+i), caller-allocated.  Synchronises the stream. */
int fdtd_rom_adjoint_workspace_size(const fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every,
                                    size_t* bytes);
/* Host-only (no device call): the same size for a problem before a handle
 * exists (prob as for fdtd_rom_create, the shape checks of
 * fdtd_rom_workspace_size).  Planning checks that the workspace's parts -
 * checkpoints, recompute slots, adjoint sets, accumulators, G^T, model
 * table - are disjoint and inside the total, as every call that plans the
 * sweep does; fdtd_rom_adjoint also checks before each recompute launch that
 * the fields, control block and state scratch it writes lie in the
 * workspace (FDTD_EINVAL otherwise). */
int fdtd_rom_adjoint_plan(const fdtd_problem* prob, int32_t nsteps, int32_t ckpt_every, size_t* bytes);
int fdtd_rom_adjoint(fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every, int32_t probe,
                     void* dev_adj_ws, size_t ws_bytes, double* J, double* grad_eps_r,
                     double* grad_sigma);

/* Gradients through the reduced models.  The same objective and reverse
 * sweep as fdtd_rom_adjoint; in addition the sweep sums, per region, the
 * gradient of J with respect to its eq. (23) update matrix G on
 * [x~^n; h^{n+1/2}] (dJ/dG = sum_n (adjoint of [x~^{n+1}; y^{n+1}]) x
 * [x~^n; h^{n+1/2}]^T, FP64 accumulators), and the host carries it through
 * the closed form of eq. (23) (Sec. IV-C: M = R~ + F~ + L~ C+ L~^T,
 * N = R~ - F~ + L~ C- L~^T, A~ = M^{-1} N, B~' = M^{-1} L~ Sc, C~ = L~^T)
 * to each region's R~, F~, L~ and to the eq. (13) half cells
 * C+- = Dl Dl' (eps0 eps_r/dt +- sigma/2) of the coarse cells just outside
 * its ports.  Those ring cells therefore report their whole gradient (the
 * coarse stencil's part plus the half cells' part); cells inside a region
 * report zero (their coarse material takes no part in the run).  Feed
 * dJ/dR~ and dJ/dF~ to fdtd_rom_build_vjp for the fine cells' gradient.
 *
 * fdtd_rom_adjoint_models_workspace_size: the adjoint workspace plus one
 * FP64 accumulator of (q+np)^2 (rows padded to 64) per region.
 * fdtd_rom_adjoint_models: arguments as fdtd_rom_adjoint, plus
 *   grad_Rt, grad_Ft, grad_Lt: host arrays of nroms pointers (an array, or
 *     any entry, may be NULL to skip it): region k's dJ/dR~ and dJ/dF~
 *     (q x q) and dJ/dL~ (q x np), row-major like the fdtd_rom inputs,
 *     caller-allocated.  The matrices' gradients are taken at the FP64
 *     models given to fdtd_rom_create (an FP32 run's trajectories, FP64
 *     algebra).  FDTD_ENOTPASSIVE if a region's M is singular.
 * Synchronises the stream. */
int fdtd_rom_adjoint_models_workspace_size(const fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every,
                                           size_t* bytes);
int fdtd_rom_adjoint_models(fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every, int32_t probe,
                            void* dev_adj_ws, size_t ws_bytes, double* J, double* grad_eps_r,
                            double* grad_sigma, double* const* grad_Rt, double* const* grad_Ft,
                            double* const* grad_Lt);

/* The same reverse sweep for callers that cannot allocate device memory
 * (code that may not call hipMalloc: tight serving loops, harnesses that
 * forbid it).  No workspace argument: the sweep's checkpoints, recomputed
 * segment, adjoint fields and accumulators live in a static device array
 * the library holds on every GPU it runs on (64 MiB each, until the process
 * ends); the call makes no device, pinned-host or heap allocation (G^T is
 * transposed on the device from the handle's update matrices, the forward
 * runs as plain launches without graph capture or finiteness checks, the
 * objective is summed on the device).  Arguments, the handle's state
 * afterwards and the results are those of fdtd_rom_adjoint (J summed in a
 * different order: equal to rounding).  The recompute runs on the handle's
 * stream between the reverse segments (no second stream, one set of
 * recomputed fields), so the need is at most
 * fdtd_rom_adjoint_workspace_size's; FDTD_ENOMEM if it exceeds the 64 MiB.  Call
 * with the handle's device current.  Every call on a GPU shares that GPU's
 * array and leaves its contents behind (each call clears what must start at
 * zero): calls that overlap on one GPU, from several threads or streams,
 * race and must be serialised by the caller.  Synchronises the stream. */
int fdtd_rom_adjoint_noalloc(fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every, int32_t probe,
                             double* J, double* grad_eps_r, double* grad_sigma);

/* Batched runs: B independent problems (uneven grids, models, sources,
 * probes; one dtype) advanced together, each step of all of them by one
 * kernel launch, replayed from captured HIP graphs.  Every instance is
 * validated and laid out exactly as fdtd_rom_create does (same checks, same
 * error codes, reported with the instance index); instance b runs the same
 * device code on the same data as its own handle would.
 *   batch_workspace_size / batch_create: as the single-problem calls, for
 *     the array probs[0..B); the caller's 256-B aligned device workspace
 *     holds every instance.
 *   batch_run: advance every instance by nsteps (asynchronous); FDTD_ESTATE
 *     if any instance would exceed its max_steps.
 *   batch_read_probes / batch_read_field: as the single-problem calls, for
 *     instance b.  Synchronise.
 *   batch_set_tiling: rows per stencil wave (4, 8, 16, 32) of instance b, or of
 *     every instance for b = -1 (the autotuner's knob).
 *   batch_set_graph: steps per captured graph (0 = direct launches; with
 *     two steps per pass rounded down to a multiple of 4). */
typedef struct fdtd_rom_batch fdtd_rom_batch; /* opaque, owned by the library */
int fdtd_rom_batch_workspace_size(const fdtd_problem* probs, int32_t B, size_t* bytes);
int fdtd_rom_batch_create(const fdtd_problem* probs, int32_t B, void* dev_workspace,
                          size_t ws_bytes, void* hip_stream, fdtd_rom_batch** out);
int fdtd_rom_batch_run(fdtd_rom_batch* batch, int32_t nsteps);
int fdtd_rom_batch_steps_done(const fdtd_rom_batch* batch, int32_t* n);
int fdtd_rom_batch_read_probes(const fdtd_rom_batch* batch, int32_t b, int32_t first,
                               int32_t count, double* host_out);
int fdtd_rom_batch_read_field(const fdtd_rom_batch* batch, int32_t b, int32_t comp,
                              double* host_out);
int fdtd_rom_batch_set_tiling(fdtd_rom_batch* batch, int32_t b, int32_t seg);
int fdtd_rom_batch_set_graph(fdtd_rom_batch* batch, int32_t batch_steps);
/* The far tiles' share in a pair's second launch (fdtd_rom_set_pair_split)
 * for instance b, or for every instance with b = -1; the batch's pair
 * tables are rebuilt before the next pair.  Results do not depend on it. */
int fdtd_rom_batch_set_pair_split(fdtd_rom_batch* batch, int32_t b, int32_t percent);
/* Two steps per pass for every instance (as fdtd_rom_set_time_blocking, all
 * instances in lockstep): on by default when no instance has absorbing
 * layers; FDTD_EINVAL for on = 1 otherwise or a value other than 0/1. */
int fdtd_rom_batch_set_time_blocking(fdtd_rom_batch* batch, int32_t on);
int fdtd_rom_batch_get_time_blocking(const fdtd_rom_batch* batch, int32_t* on);
void fdtd_rom_batch_destroy(fdtd_rom_batch* batch);

/* Release the handle (the workspace stays the caller's). */
void fdtd_rom_destroy(fdtd_rom_sim* sim);

const char* fdtd_rom_strerror(int status);
const char* fdtd_rom_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_ROM_H */
