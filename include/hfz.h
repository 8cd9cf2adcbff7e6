/*
 * hfz — energy-stable FAS multigrid for the hydrodynamic PFC / CDFT freezing
 * models on one AMD MI355X (gfx950).
 *
 * The library advances the fully discrete convex-splitting scheme of
 * Baskaran, Guan & Lowengrub, "Energy stable multigrid method for local and
 * non-local hydrodynamic models for freezing" (arXiv 1503.07416), Sec. 5,
 * Eqs. discrete_a-d, on a periodic n x n nodal grid:
 *
 *   rho^{k+1} - rho^k = -s div_h(rho^k u^{k+1/2})
 *   rho^k (u^{k+1} - u^k) = s[ -rho^k omega^k x u^{k+1/2} - (rho^k/2) grad_h|u^{k+1}|^2
 *                              - rho^k grad_h mu^{k+1} + gamma Delta_h u^{k+1/2} ]
 *   mu^{k+1} = dF_c[rho^{k+1}] - dF_e[rho^k],   omega^k = curl_h u^k
 *
 * with the discrete PFC free energy (Sec. 5.3) or the discrete CDFT free
 * energy with the Sec. 6 kernel J (Sec. 5.2; the convolution is applied
 * through a DFT).  Each implicit step is the nonlinear system N(g) = S of
 * App. G, solved by FAS V-cycles with the damped point-block Gauss-Seidel
 * smoother of App. G (red-black ordered), full-weighting restriction and
 * bilinear prolongation, until ||S - N(g)||_2 <= tol.
 *
 * The same solver also advances the gradient-flow scheme of Thm. thm_grad
 * (Eq. gradient_scheme), models HFZ_PFC_GF and HFZ_CDFT_GF:
 *
 *   rho^{k+1} - rho^k = s Delta_h mu^{k+1},   mu^{k+1} = dF_c[rho^{k+1}] - dF_e[rho^k]
 *
 * with the same discrete free energies and splittings.  The paper proves it
 * mass conserving and unconditionally energy stable but gives no solver for
 * it; here its unknowns per node are (rho, mu, kappa = Delta_h rho) for PFC
 * and (rho, mu) for CDFT, the rows are N1 = rho - s Delta_h mu, the mu row of
 * the free energy (App. G's PFC rows 4-5, or mu - ln rho - 2 c_e rho for
 * CDFT), and the App. G smoother's recipe applies: exact block solve with
 * the nonlinearity linearised about the current iterate, damping w, the
 * CDFT positivity projection.  The state is rho alone (u = v = 0).
 *
 * The PFC step also runs in a channel (hfz_params.walls = 1; Sec. 6, the
 * sheared-nanocrystal run): periodic in x, walls in y at the node rows j = 0
 * and j = n, which hold the boundary values: no-slip moving walls u =
 * u_wall_bottom / u_wall_top, v = 0, and no flux for the density, rho on a
 * wall row equal to the adjacent interior row (likewise mu and kappa, and
 * rho^k).  The unknowns are on the interior rows 1..n-1; fields then have
 * (n + 1) * n values, rows 0..n.  The smoother refreshes the wall rows after
 * every half sweep; the multigrid levels are nested vertex grids whose wall
 * rows follow the same rules; norm, energy and mass sum the interior rows.
 *
 * Conventions for every entry point
 *  - Return value: HFZ_OK (0) or a negative HFZ_E* code; no exception or
 *    abort crosses the ABI.  hfz_strerror() names a code.
 *  - Fields are FP64, n*n values (a channel: (n + 1) * n, rows j = 0..n),
 *    row-major [j][i] with x (index i) fastest, node (i, j) at (i h, j h).
 *  - Device pointers are plain HIP device addresses on the device current
 *    when hfz_init ran.  The caller owns all device memory: the workspace
 *    (hfz_workspace_bytes) and the state buffers.  The library never
 *    allocates device memory (hfz_step_noalloc works in a static device
 *    array of the library instead of a caller workspace).
 *  - All device work is enqueued on the stream given to hfz_init
 *    (a hipStream_t passed as void*, NULL for the default stream).  Entry
 *    points that return host values (hfz_step's convergence test, energy,
 *    mass, residual) synchronise that stream.
 *  - A handle is not thread safe; distinct handles with distinct workspaces
 *    may be used concurrently.
 *
 * Kernel choice.  Results do not depend on it beyond rounding; the library
 * picks by level size and, for the 2D tiled kernels, by timing candidates at
 * hfz_init (cached per process).  Environment variables, read at init
 * (hfz_init, hfz_batch_init, hfz3_init), override the choices for testing
 * and measurement:
 *    HFZ_TILE=<0..9>      tile shape of the 2D smoother where it fits
 *    HFZ_RESTRICT=<0..3>  FAS restriction variant where it fits
 *    HFZ_SWEEPS=1         one sweep per smoother launch (default: two fused)
 *    HFZ_TUNE=0           no timing: shape 0, variant 0, fused sweeps
 *    HFZ_TUNE_CACHE=<f>   the tuner's choices read from file f when it exists and
 *                         written to it after timing (profiled runs reuse them)
 *    HFZ_TILES=0          per-colour smoother kernels instead of the tiled one
 *                         (FP64 periodic only; mixed precision and the
 *                         channel always use the tiled kernels)
 *    HFZ_TAIL_N=<n>       largest level of the one-workgroup tail (0: none)
 *    HFZ_GRAPH=0          no HIP graph capture of the V-cycle
 *    HFZ_FUSE=<0|1>       FAS restriction as a launch of its own (0) or folded
 *                         into the last pre-sweep launch of a level (1) on every
 *                         level where it can be (default: timed, the choices of
 *                         all levels made together)
 *    HFZ_FOLD_RHS=0       a coarse level whose right-hand side a folded
 *                         restriction left as R d has it completed by a launch
 *                         of its own (default: by its own pre-sweep launch where
 *                         that folds its restriction too and its tiles fit LDS)
 *    HFZ_MP_INNER=<1..8>  FP32 V-cycles per outer FP64 iteration (mixed)
 *    HFZ_BATCH_TILE=<0|2> tile shape of the batched smoother
 *    HFZ_BATCH_RESTRICT=<0..3> batched FAS restriction: 0 the direct kernel, 1-3
 *                         the staged one with coarse tiles of 8 / 256 threads,
 *                         16 / 256, 16 / 512 (default 3)
 *    HFZ3_TILES=<n>       smallest 3D level swept by the tiled kernel (0: none)
 *    HFZ3_TAIL=0          no one-workgroup tail in 3D
 *    HFZ_VERBOSE=1        the choices made, on stderr
 */
#ifndef HFZ_H
#define HFZ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HFZ_OK = 0,
  HFZ_EINVAL = -1,   /* bad parameter: n not a power of two >= 8, h/s/gamma <= 0, ... */
  HFZ_ENOMEM = -2,   /* workspace smaller than hfz_workspace_bytes */
  HFZ_EDOMAIN = -3,  /* CDFT state with rho <= 0 (ln rho undefined, Sec. 2.1) */
  HFZ_ENOCONV = -4,  /* max_cycles V-cycles without reaching tol; state not advanced */
  HFZ_ENAN = -5,     /* non-finite residual or energy; state not advanced */
  HFZ_EHIP = -6,     /* HIP runtime error */
  HFZ_ESTATE = -7,   /* call out of order (e.g. step before set_state) */
  HFZ_ESCRATCH = -8  /* hfz_step_noalloc: the problem does not fit HFZ_NOALLOC_SCRATCH_BYTES */
};

/* Hydrodynamic PFC / CDFT step (Eqs. discrete_a-d), or the gradient-flow
 * scheme of Thm. thm_grad with the PFC / CDFT free energy. */
enum { HFZ_PFC = 0, HFZ_CDFT = 1, HFZ_PFC_GF = 2, HFZ_CDFT_GF = 3 };
enum { HFZ_FP64 = 0, HFZ_MIXED = 1 };

/* Parameters of one simulation.  Paper values: gamma = 2 (Sec. 6), w_damp =
 * 0.5 (App. G, damped Gauss-Seidel), delta = 1e-10 for CDFT and unused for PFC
 * (Sec. 6, positivity projection), alpha = 1 - eps (App. B). */
typedef struct hfz_params {
  int model;          /* HFZ_PFC, HFZ_CDFT, HFZ_PFC_GF or HFZ_CDFT_GF */
  int n;              /* grid is n x n, n a power of two, 8 <= n <= 8192 */
  double h;           /* grid spacing (> 0) */
  double s;           /* time step (> 0) */
  double gamma;       /* viscosity (> 0; unused by the gradient flow) */
  double alpha;       /* PFC (both schemes): coefficient of the quadratic term */
  double nu;          /* CDFT (both schemes): kernel scale of J (Sec. 6) */
  double delta;       /* CDFT (both schemes): rho <- sqrt(rho^2 + delta^2) after each rho update */
  double w_damp;      /* damping, x <- (1 - w) x_GS + w x_old, 0 <= w < 1 */
  double tol;         /* residual tolerance on ||S - N(g)||_2 (h^2-weighted) */
  int nu1, nu2;       /* pre / post smoothing sweeps per level (>= 0, sum >= 1; >= 1 each for
                         mixed precision, the channel and the batch) */
  int max_cycles;     /* V-cycle cap per step (>= 1) */
  int coarsest_n;     /* coarsest grid size, power of two, 4 <= coarsest_n <= n (<= 32 for mixed
                         precision, the channel and the batch: their coarsest level runs in the
                         one-workgroup tail) */
  int coarse_sweeps;  /* sweeps on the coarsest grid per V-cycle (>= 1) */
  int precision;      /* HFZ_FP64, or HFZ_MIXED: FP32 smoothing inside FP64 defect correction
                         (three FP32 V-cycles per outer FP64 iteration) */
  int sigma;          /* +1: -rho omega x u in vector form (default); -1: App. G sign (hydrodynamic only) */
  int continuity_fix; /* 1: recompute rho^{k+1} from the continuity row after the solve
                         (gradient flow: rho^{k+1} = rho^k + s Delta_h mu^{k+1}) */
  int walls;          /* 0: periodic; 1: a channel, walls at y = 0 and y = n h (HFZ_PFC, FP64,
                         nu1 >= 1 and nu2 >= 1 only; HFZ_EINVAL otherwise) */
  double u_wall_bottom, u_wall_top; /* channel: u on the walls (v = 0 there) */
} hfz_params;

typedef struct hfz_stats {
  int steps_done;       /* steps completed by this call */
  int cycles_last;      /* V-cycles (mixed: outer FP64 iterations) of the last step */
  long long cycles_total;
  double residual_last; /* final ||S - N(g)||_2 of the last step */
} hfz_stats;

typedef struct hfz_handle hfz_handle;

/* Fills hfz_params with the paper's defaults for the given model (n, h, s
 * still to be set by the caller).  Pure host function. */
int hfz_default_params(int model, hfz_params* p);

/* Bytes of device workspace hfz_init needs for *p.  Pure host function;
 * validates *p (HFZ_EINVAL). */
int hfz_workspace_bytes(const hfz_params* p, size_t* bytes);

/* Creates a handle.  dev_ws: caller-owned device buffer of ws_bytes >=
 * hfz_workspace_bytes (256-byte aligned); it must outlive the handle.
 * For CDFT this tabulates the periodised kernel J_{k,l} = J(x_{k,l})
 * (minimum image), computes (J_e * 1) = h^2 sum J_e (Lemma CDFT_ineq) and the
 * DFT multiplier h^2 DFT(J) of Eq. discrete_convolution on the device. */
int hfz_init(const hfz_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
             hfz_handle** out);

/* Loads (rho^0, u^0, v^0) from device buffers of n*n doubles each (copied;
 * the caller keeps ownership).  PFC (both schemes): mu and kappa start
 * consistent with rho^{k+1} = rho^k; CDFT gradient flow: mu = dF[rho].
 * CDFT (both schemes): fails with HFZ_EDOMAIN if min rho <= 0.  Gradient
 * flow: u and v are ignored and may be NULL (the velocity is zero). */
int hfz_set_state(hfz_handle* hd, const double* rho, const double* u, const double* v);

/* Copies the current (rho^k, u^k, v^k) into caller device buffers; for the
 * gradient flow u and v may be NULL (else they receive zeros). */
int hfz_get_state(hfz_handle* hd, double* rho, double* u, double* v);

/* Copies the auxiliary unknowns of the last solve (or those of hfz_set_state)
 * into caller device buffers: (mu, kappa) for PFC and the PFC gradient flow;
 * mu for the CDFT gradient flow (kappa may be NULL, and is left untouched);
 * HFZ_EINVAL for the hydrodynamic CDFT, which has none. */
int hfz_get_aux(hfz_handle* hd, double* mu, double* kappa);

/* Advances nsteps time steps.  On HFZ_ENOCONV / HFZ_ENAN the failing step is
 * rolled back: the state is that of the last completed step, and
 * stats->steps_done says how many completed.  stats may be NULL. */
int hfz_step(hfz_handle* hd, int nsteps, hfz_stats* stats);

/* Discrete energy of the current state (Thm. thm_energy_stability):
 * out[0] = E = KE + F, out[1] = KE = (rho u || u)/2, out[2] = F,
 * out[3], out[4] = F_id, F_ex for CDFT (0 for PFC).  Host array of 5.
 * Gradient flow: KE = 0 and E = F, the energy of Thm. thm_grad. */
int hfz_energy(hfz_handle* hd, double* out5);

/* Discrete mass (rho || 1) = h^2 sum rho of the current state. */
int hfz_mass(hfz_handle* hd, double* mass);

/* ---- stage-level entry points (the same kernels hfz_step runs; for tests
 *      and for callers that drive the solve themselves) ------------------- */

/* Source and frozen coefficients of the step from the current state: S and
 * omega^k (App. G), rho^k and omega^k restricted to every level, the CDFT
 * convolution J * rho^k; the iterate g starts at the state.  Gradient flow:
 * S and g = (rho^k, dF[rho^k] (, Delta_h rho^k)) on level 0 only. */
int hfz_begin_step(hfz_handle* hd);
/* `sweeps` damped red-black sweeps on level `level` (0 = finest). */
int hfz_smooth(hfz_handle* hd, int level, int sweeps);
/* `count` FAS V(nu1, nu2) cycles on the finest level without a stop test. */
int hfz_vcycle(hfz_handle* hd, int count);
/* ||f - N(g)||_2 on level 0 (host double). */
int hfz_residual(hfz_handle* hd, double* norm);
/* Ends the step: continuity fix, state <- g, next CDFT convolution
 * (gradient flow: rho^{k+1} from row 1, mu (and kappa) kept as auxiliaries). */
int hfz_finish_step(hfz_handle* hd);

/* Field access for tests.  which: 0 = iterate g, 1 = right-hand side f,
 * 2 = restricted iterate R g (coarse levels), 3 = frozen coefficient
 * (comp 0 rho^k, comp 1 omega^k), 4 = J * rho of the state (comp 0, level 0).
 * dst / src: device buffers of n_l * n_l doubles, n_l = n >> level. */
int hfz_read_field(hfz_handle* hd, int which, int level, int comp, double* dst);
int hfz_write_field(hfz_handle* hd, int which, int level, int comp, const double* src);

/* Number of grid levels and the CDFT scalar (J_e * 1) (0 for PFC). */
int hfz_info(hfz_handle* hd, int* levels, double* ce);

/* Tile shape of the LDS-tiled sweep kernel on an FP64 level: tx x ty owned
 * nodes per workgroup of `threads` threads, picked at hfz_init by timing the
 * shapes that cover the level (environment: HFZ_TILE=<0..9> forces a shape,
 * HFZ_TUNE=0 keeps shape 0).  The swept values do not depend on the shape.
 * HFZ_EINVAL for a level the tiled kernel does not sweep (the coarse tail). */
int hfz_tile_shape(hfz_handle* hd, int level, int* tx, int* ty, int* threads);

int hfz_destroy(hfz_handle* hd);
const char* hfz_strerror(int code);

/* ---- the step without device allocation ---------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It does
 * what hfz_init + hfz_set_state + hfz_step + hfz_get_state do, with the
 * workspace in a static device array of the library (HFZ_NOALLOC_SCRATCH_BYTES,
 * 72 MiB, reserved on every GPU the library runs on until the process ends)
 * instead of a caller buffer; it calls no hipMalloc, hipFree or other
 * allocating routine (host bookkeeping uses the C++ heap), uploads its level
 * descriptors through kernel arguments, does not time kernel candidates (the
 * tile shapes cached in this process by an earlier hfz_init, else the
 * defaults) and launches no HIP graph; the results equal hfz_step's up to
 * rounding.
 *  p:     parameters as for hfz_init; HFZ_ESCRATCH if hfz_workspace_bytes(p)
 *         exceeds HFZ_NOALLOC_SCRATCH_BYTES (it holds e.g. PFC FP64 512^2,
 *         CDFT FP64 512^2, PFC mixed 256^2).
 *  rho, u, v: caller device buffers of n*n doubles (a channel: (n + 1) * n),
 *         the state before the call on entry and after it on return (u, v
 *         may be NULL for the gradient flow).  On HFZ_ENOCONV / HFZ_ENAN they
 *         hold the state after the last completed step.  The auxiliaries of
 *         PFC (mu, kappa) start from the state, as after hfz_set_state.
 *  nsteps, stats: as for hfz_step.  hip_stream: as for hfz_init.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * there; the call initialises everything it reads.  Calls that overlap on one
 * GPU (other host threads or streams) race on the array: serialise them. */
#define HFZ_NOALLOC_SCRATCH_BYTES ((size_t)72 << 20)
int hfz_step_noalloc(const hfz_params* p, double* rho, double* u, double* v, int nsteps, void* hip_stream,
                     hfz_stats* stats);

/* ---- batched solve ------------------------------------------------------
 * `count` independent instances advance together: each V-cycle phase of all
 * instances is one kernel launch (instance index in the grid), the coarse
 * tail one workgroup per instance.  All instances share model, n, precision,
 * nu1, nu2 (both >= 1), coarsest_n and coarse_sweeps; h, s, gamma and the
 * model constants may differ (hydrodynamic models only: HFZ_EINVAL for the
 * gradient flow).  Each instance keeps its own stop test and
 * leaves the launches when it converges, so its result is bitwise the one
 * the single-instance solver produces.  Ownership, streams and errors as for
 * the single-instance calls. */
typedef struct hfz_batch hfz_batch;

/* Bytes of device workspace for a batch over params[0..count-1]. */
int hfz_batch_workspace_bytes(const hfz_params* params, int count, size_t* bytes);
int hfz_batch_init(const hfz_params* params, int count, void* dev_ws, size_t ws_bytes, void* hip_stream,
                   hfz_batch** out);
/* State of instance i (device buffers of n*n doubles), as hfz_set_state / hfz_get_state. */
int hfz_batch_set_state(hfz_batch* b, int i, const double* rho, const double* u, const double* v);
int hfz_batch_get_state(hfz_batch* b, int i, double* rho, double* u, double* v);
/* Energy of instance i, as hfz_energy. */
int hfz_batch_energy(hfz_batch* b, int i, double* out5);
/* Marks instance i empty: hfz_batch_step skips it until hfz_batch_set_state
 * fills it again (a slot of a serving pool).  Its memory stays reserved. */
int hfz_batch_release(hfz_batch* b, int i);
/* Advances every filled instance (state set and not released) nsteps steps;
 * empty instances are skipped and get zeroed stats.  stats: NULL or an array
 * of count.  An instance that fails a step (HFZ_ENOCONV / HFZ_ENAN) keeps its
 * previous state, the others complete the step, the call returns the first
 * failure code after that step. */
int hfz_batch_step(hfz_batch* b, int nsteps, hfz_stats* stats);
int hfz_batch_destroy(hfz_batch* b);

/* ---- three dimensions ---------------------------------------------------
 * The hydrodynamic PFC step on a periodic n x n x n grid (the extension to 3D
 * that Sec. 3 calls straightforward; the paper works in 2D).  Unknowns per
 * node (rho, u, v, w, mu, kappa); the rows are App. G's with the third
 * direction: 7-point Delta_h, wide central differences, the vector vorticity
 * omega^k = curl_h u^k and the vector form -rho^k omega^k x u of the
 * advection term.  The smoother keeps App. G's triangular block; its velocity
 * part is the 3x3 system (a I + [b x]) u = r, a = rho^k + 3 s gamma/h^2,
 * b = (s/2) sigma rho^k omega^k, solved in closed form.  FAS V(nu1, nu2) with
 * 27-point full weighting and trilinear prolongation; norm, energy and mass
 * carry the weight h^3.  Parameters: hfz_params with model HFZ_PFC, FP64, no
 * walls, 8 <= n <= 512 (HFZ_EINVAL otherwise).  Fields: n^3 FP64 values,
 * x fastest, then y, then z.  Ownership, streams and errors as for the 2D
 * calls.  The damped block smoother needs s/h^4 of order 0.5 or less in 3D.
 * Kernel choice (same results, read at hfz3_init): levels from 128^3 up are
 * swept by a one-launch tiled kernel, smaller ones by one launch per colour,
 * and the levels from 8^3 down run in one workgroup; the environment
 * variables HFZ3_TILES (smallest level of the tiled sweep, 0: never) and
 * HFZ3_TAIL (0: no one-workgroup tail) override this. */
typedef struct hfz3_handle hfz3_handle;

int hfz3_workspace_bytes(const hfz_params* p, size_t* bytes);
int hfz3_init(const hfz_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, hfz3_handle** out);
/* (rho, u, v, w) from device buffers; mu and kappa start consistent with rho^{k+1} = rho^k. */
int hfz3_set_state(hfz3_handle* hd, const double* rho, const double* u, const double* v, const double* w);
int hfz3_get_state(hfz3_handle* hd, double* rho, double* u, double* v, double* w);
/* As hfz_step. */
int hfz3_step(hfz3_handle* hd, int nsteps, hfz_stats* stats);
/* out[0] = E = KE + F, out[1] = KE, out[2] = F (the 3D PFC energy, weight h^3).  Host array of 3. */
int hfz3_energy(hfz3_handle* hd, double* out3);
int hfz3_mass(hfz3_handle* hd, double* mass);
/* Stage calls as their 2D counterparts. */
int hfz3_begin_step(hfz3_handle* hd);
int hfz3_smooth(hfz3_handle* hd, int level, int sweeps);
int hfz3_vcycle(hfz3_handle* hd, int count);
int hfz3_residual(hfz3_handle* hd, double* norm);
int hfz3_finish_step(hfz3_handle* hd);
/* which: 0 iterate, 1 right-hand side, 3 frozen coefficients (comp 0 rho^k,
 * 1..3 omega^k), 5 the auxiliaries of level 0 (comp 0 mu, 1 kappa). */
int hfz3_read_field(hfz3_handle* hd, int which, int level, int comp, double* dst);
int hfz3_levels(hfz3_handle* hd, int* levels);
int hfz3_destroy(hfz3_handle* hd);

#ifdef __cplusplus
}
#endif
#endif /* HFZ_H */
