/*
 * cmcg.h - C ABI of the MI355X (gfx950) controllability-method solver for the Helmholtz
 * equation: the periodic solution of the time-harmonically forced wave equation is found by
 * conjugate gradients on its initial state (Grote, Nataf, Tang, Tournier, "Parallel
 * Controllability Methods for the Helmholtz Equation", the CMCG Algorithm of Sec. 2.3).
 *
 * Every call returns a cmcg_status (0 = CMCG_OK); nothing unwinds across the ABI.  A handle
 * must not be used by two threads at once; different handles are independent.  All device
 * work of a handle runs on the HIP stream given in cmcg_options (NULL = a stream the handle
 * creates).  The handle owns all device memory it allocates until cmcg_destroy.
 *
 * Problem (eq. HE):  -lap u - k^2 u = f in the box [0, n_x h] x [0, n_y h] (x [0, n_z h]),
 * h = 1 / n_x, k = omega / c(x);  du/dn - i k u = gS on absorbing faces, du/dn = gN on
 * Neumann faces, u = gD on sound-soft nodes (F2) or cells (F1).  Time domain (eq. WE / eq. mixWE): the forced
 * wave equation with source Re(f e^{-i omega t}) and boundary data Re(gS e^{-i omega t});
 * one period T = 2 pi / omega is N = ceil(T c_max / (courant h)) leapfrog steps, dt = T / N.
 *
 * Formulations:
 *  1 (F1, dim 2): first-order velocity/flux system (Sec. 3.1, eq. mixWE) on a staggered grid:
 *    v and c at the n_x x n_y cell centres, flux on interior faces, absorbing condition
 *    p.n + v/c = gS on boundary faces.  Energy metric of eq. mix_cost_functional_J.
 *  2 (F2, dim 3): second-order system (Sec. 2, eq. WE) on the (n+1)^3 nodes, mass-lumped
 *    7-point stencil, energy metric of eq. cost_functional_J, Riesz map of
 *    eq. CMCG_PRECONDITIONIER solved on the device each iteration.
 *
 * Array layouts (host arrays unless stated):
 *  - F1 cell fields (c, f, u): n_y rows of n_x values, x fastest.
 *  - F2 node fields (c, f, sound_soft, u): (n_z+1) planes of (n_y+1) rows of (n_x+1) values.
 *  - gS: the faces -x, +x, -y, +y[, -z, +z] concatenated.  F1: n_y values for each x face,
 *    n_x for each y face.  F2: each face's nodes in array order of the two remaining axes
 *    (slower axis first): (n_z+1)(n_y+1) for x faces, (n_z+1)(n_x+1) for y faces,
 *    (n_y+1)(n_x+1) for z faces.
 *  - Packed state vectors (cmcg_apply, cmcg_get_state, cmcg_filter), FP64 DEVICE arrays:
 *    F1: [Px (n_y rows of n_x-1), Py (n_y-1 rows of n_x), v (n_y rows of n_x)];
 *    F2: [u (all nodes), v (all nodes)], sound-soft entries zero.
 */
#ifndef CMCG_H
#define CMCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cmcg_handle cmcg_handle;

typedef enum {
  CMCG_OK = 0,
  CMCG_ENOTCONV = 1,      /* warning: max_iter reached; the result is the last iterate   */
  CMCG_EINVAL = -1,       /* invalid argument (sizes, NaN or non-positive c or omega...)  */
  CMCG_ECFL = -2,         /* courant * sqrt(dim) >= 1: leapfrog would be unstable          */
  CMCG_ENOMEM = -3,       /* device allocation failed                                      */
  CMCG_EDEVICE = -4,      /* a HIP call failed; see cmcg_last_error()                      */
  CMCG_EBREAKDOWN = -5,   /* CG breakdown: <qhat, d> <= 0 or a non-finite scalar           */
  CMCG_EUNSUPPORTED = -6  /* a valid combination this library does not implement           */
} cmcg_status;

enum { CMCG_ABSORBING = 0, CMCG_NEUMANN = 1 };
enum { CMCG_FP64 = 0, CMCG_FP32_MIXED = 1 };

#define CMCG_MAX_SHOTS 8

/* One component of a multi-frequency ("super-shot") source (Concluding remarks): a source that
 * superposes time-harmonic components at integer multiples of one base frequency omega has the
 * common period T = 2 pi / omega, so one CMCG solve finds its periodic solution and the filter
 * at each component's frequency extracts that component's Helmholtz solution.  The arrays have
 * the layouts of the cmcg_problem fields of the same names and the same NULL rules. */
typedef struct {
  int32_t harmonic;            /* m >= 1: the component oscillates as e^{-i m omega t}; the
                                  harmonics of a problem are distinct and 2 m < N              */
  const double *f_re, *f_im;
  const double *gS_re, *gS_im;
  const double *gD_re, *gD_im;
} cmcg_shot;

typedef struct {
  int32_t dim;                 /* 2 (F1) or 3 (F2)                                           */
  int32_t formulation;         /* 1 = first-order staggered, 2 = second-order nodal           */
  int64_t n[3];                /* cells per axis; n[2] ignored in 2D; h = 1 / n[0]             */
  double omega;                /* angular frequency > 0                                        */
  const double *c;             /* wave speed > 0 (cell or node field); NULL -> c_const         */
  double c_const;
  const double *f_re, *f_im;   /* source amplitude (same layout as c); either may be NULL      */
  const double *gS_re, *gS_im; /* boundary data, concatenated faces: gS on absorbing faces
                                  (du/dn - i k u = gS), gN on Neumann faces (du/dn = gN);
                                  either may be NULL (zero)                                    */
  const uint8_t *sound_soft;   /* 1 = Dirichlet node (F2) or cell (F1), layout of c; NULL = none.
                                  F1 Dirichlet cells hold v = Re(-i omega gD e^{-i omega t})
                                  (eq. mixWE_DBC) and carry no unknown                         */
  const double *gD_re, *gD_im; /* Dirichlet data u = gD on the sound-soft nodes or cells (layout
                                  of c, read there only); NULL = homogeneous                   */
  int32_t face_bc[6];          /* -x,+x,-y,+y,-z,+z: CMCG_ABSORBING or CMCG_NEUMANN            */
  double courant;              /* sigma in (0, 1/sqrt(dim)); 0 -> 0.5                          */
  int32_t n_shots;             /* 0: one time-harmonic source at omega with the data above.
                                  1..CMCG_MAX_SHOTS: the source is the sum of `shots`, omega is
                                  their base frequency (T = 2 pi / omega, N from T as above),
                                  and f, gS and gD above must be NULL.  The filter outputs
                                  (cmcg_solve, cmcg_finish, cmcg_filter) then hold n_shots
                                  fields, one per shot in shot order, each of field_len values;
                                  the first-order field is u = i V / (m omega).                */
  const cmcg_shot *shots;      /* n_shots components (copied at create), or NULL               */
} cmcg_problem;

typedef struct {
  int32_t precision;           /* CMCG_FP64, or CMCG_FP32_MIXED: FP32 fields and stencil
                                  arithmetic, FP64 iterate, residual, scalars and sums         */
  double tol;                  /* stop when sqrt(<r,r>_E / <r0,r0>_E) <= tol (Step 5.8)        */
  int32_t max_iter;            /* CG iteration cap (> 0)                                       */
  int32_t device;              /* HIP device ordinal                                           */
  void *hip_stream;            /* hipStream_t to run on, or NULL                                */
  int32_t steps_per_launch;    /* leapfrog steps fused per kernel launch (temporal blocking):
                                  F1 1..8 (default 7); F2 1..4 for the
                                  homogeneous steps (default 4 in FP32, 3 in FP64, the FP64
                                  refreshes of FP32-mixed solves included; a value given here
                                  sets both; 1 = one step per launch); 0 = library default.
                                  Results do not depend on it (bitwise)                        */
  int32_t riesz_max_iter;      /* F2: cap on the Riesz (elliptic) PCG iterations; 0 = default  */
  double riesz_tol;            /* F2: relative tolerance of the Riesz solve; 0 = default       */
  double fp64_refresh;         /* FP32-mixed: recompute the true gradient with FP64 periods
                                  whenever <r,r>_E has fallen by fp64_refresh^2 since the last
                                  refresh, and before declaring convergence (reliable updates);
                                  0 = default 0.1, < 0 = never                                  */
  int32_t riesz_mode;          /* F2 Riesz map q_u = P_u qh_u (eq. CMCG_PRECONDITIONIER):
                                  CMCG_RIESZ_SOLVE: S^{-1} by multigrid-preconditioned CG to
                                  riesz_tol (the exact map); CMCG_RIESZ_VCYCLE: one fixed
                                  symmetric multigrid V-cycle B ~ S^{-1} (an SPD stand-in: CG
                                  converges to the same minimiser, the stopping norm is the B
                                  one; FP32-mixed solves apply it in FP32 storage and
                                  arithmetic); 0 = default: SOLVE for FP64, VCYCLE for
                                  FP32-mixed                                                   */
  int32_t runup_periods;       /* initial run-up (Sec. 4.2.3): before the CG iteration, integrate
                                  the forced scheme from rest over this many periods with the
                                  source switched on by Mur's transient theta_tr (t_tr = the
                                  run-up's length) and start CG from the state reached; the
                                  stopping test then compares with the residual at rest, so the
                                  solve stops at the accuracy a start from rest stops at.
                                  0 = start from rest.  Run in FP64.                           */
  int32_t output;              /* how cmcg_solve / cmcg_finish turn the minimiser into u:
                                  CMCG_OUTPUT_FILTER (0, default): the fundamental-frequency
                                  filter over one forced period (eq. fundamental-frequency-
                                  solution / eq. TH_FILTERED_MIXED_SOLUTION); on a pure-Neumann
                                  nodal box its result is shifted by the constant that the
                                  compatibility condition fixes (eq. cc_neumann_eta).
                                  CMCG_OUTPUT_STEP6: read u off the state itself, as cmcg_step6
                                  does (single-frequency sources; not on a pure-Neumann box)   */
} cmcg_options;

enum { CMCG_OUTPUT_FILTER = 0, CMCG_OUTPUT_STEP6 = 1 };

enum { CMCG_RIESZ_DEFAULT = 0, CMCG_RIESZ_SOLVE = 1, CMCG_RIESZ_VCYCLE = 2 };

typedef struct {
  int32_t iterations;          /* CG iterations done                                           */
  int32_t steps_per_period;    /* N                                                            */
  double dt;
  double rel_residual;         /* last sqrt(<r,r>_E / <r0,r0>_E)                               */
  double seconds;              /* device time of the last cmcg_solve (HIP events), create excluded */
  double seconds_fwd, seconds_adj, seconds_riesz, seconds_other;  /* phase split of iterations */
  double grid_updates;         /* grid-point updates (cell- or node-steps) of the last solve   */
  int64_t riesz_iterations;    /* F2: total inner PCG iterations                               */
  int32_t fp64_refreshes;      /* FP32-mixed: number of FP64 true-gradient refreshes           */
  int32_t runup_periods;       /* periods of initial run-up done by the last cmcg_begin         */
  double seconds_runup;        /* device time of that run-up (part of seconds)                 */
  double dram_bytes;           /* compulsory HBM traffic of the last solve's stencil launches:
                                  each launch reads its input arrays (state, coefficients,
                                  sources, subtrahend) once and writes its outputs once; the CG
                                  vector operations, the Riesz map and the per-component
                                  kernels of multi-frequency sources are not counted           */
  int32_t riesz_unconverged;   /* F2, CMCG_RIESZ_SOLVE: Riesz solves of the last solve (or
                                  apply) that stopped at riesz_max_iter above riesz_tol.  CG then
                                  ran with an inexact map, and cmcg_solve returns CMCG_ENOTCONV */
  double seconds_bulk_fwd, seconds_bulk_adj;   /* device time of the bulk launches of the CG
                                  iterations' forward / backward periods (HIP events around each
                                  period's run of them): first order, the launches between a
                                  period's first and last; second order, the blocked launches
                                  of full depth.  Each direction's bulk runs one kernel instance */
  int64_t bulk_launches_fwd, bulk_launches_adj;   /* the number of those launches              */
} cmcg_report;

/* Create a solver for `problem`: validates it, sets T, N and dt, allocates the device state and
 * copies the inputs host -> device.  The caller may free its arrays afterwards.  On error *out
 * is NULL. */
cmcg_status cmcg_create(const cmcg_problem *problem, const cmcg_options *opts, cmcg_handle **out);

/* Full CMCG solve from z = 0 (Steps 1-6) followed by the fundamental-frequency filter
 * (eq. fundamental-frequency-solution for F2, eq. TH_FILTERED_MIXED_SOLUTION for F1).
 * u_re, u_im: caller-allocated, host or device, same layout as c (either may be NULL to skip
 * the copy), n_fields such fields back to back (cmcg_info).  May be called repeatedly.
 * Returns CMCG_ENOTCONV when max_iter is reached. */
cmcg_status cmcg_solve(cmcg_handle *h, double *u_re, double *u_im, cmcg_report *rep);

/* NULL-safe. */
void cmcg_destroy(cmcg_handle *h);

const char *cmcg_status_string(cmcg_status s);
/* Message of the last failure on this thread ("" if none). */
const char *cmcg_last_error(void);

/* ---- stage-level calls (same kernels as cmcg_solve; used by tests and benchmarks) ---- */

typedef struct {
  int32_t steps_per_period;
  double dt, T, h;
  int64_t state_len;           /* length of a packed state vector                             */
  int64_t field_len;           /* length of the output field u                                */
  int64_t device_bytes;        /* device memory held by the handle                            */
  int32_t n_fields;            /* fields written by the filter outputs: n_shots, or 1          */
  int32_t steps_per_launch;    /* leapfrog steps fused per launch in homogeneous periods, after
                                  the library default is applied                              */
  int32_t block_rows;          /* F2 with steps_per_launch > 1: grid rows per wavefront of the
                                  blocked launches' tiles (a tile is 64 nodes by block_rows x
                                  block_waves rows); 0 otherwise                              */
  int32_t block_waves;         /* F2 with steps_per_launch > 1: wavefronts per workgroup of the
                                  blocked launches; 0 otherwise                               */
} cmcg_info;

cmcg_status cmcg_get_info(const cmcg_handle *h, cmcg_info *info);

enum {
  CMCG_OP_FORWARD = 0,         /* E z: homogeneous leapfrog from t = 0                         */
  CMCG_OP_FORCED = 1,          /* Phi(z) = E z + s: forced leapfrog from t = 0                  */
  CMCG_OP_ADJOINT = 2,         /* E* y = M_E^{-1} E^T M_E y: the backward (adjoint) period, the
                                  exact transpose of the discrete forward period in the energy
                                  inner product (eq. AWE / eq. mixJ_deriative_2, discrete)      */
  CMCG_OP_RIESZ = 3            /* F2: P y = blockdiag(S^{-1}, M^{-1}) y (eq. CMCG_PRECONDITIONIER);
                                  F1: M_E^{-1} y                                               */
};

/* out = op(in) over `steps` leapfrog steps (0 = one full period N; F1 only for steps != 0).
 * in, out: packed FP64 device vectors of length state_len; the work runs in the handle's
 * precision (FP32-mixed rounds `in` to FP32).  in and out may alias. */
cmcg_status cmcg_apply(cmcg_handle *h, int32_t op, int32_t steps, const double *in, double *out);

/* Filter output from an explicit initial state z (packed FP64 device vector): one forced period
 * from z with the accumulation of eq. fundamental-frequency-solution / eq.
 * TH_FILTERED_MIXED_SOLUTION (one accumulation per shot, at its frequency).  u_re, u_im: host
 * or device, n_fields fields of the layout of c. */
cmcg_status cmcg_filter(cmcg_handle *h, const double *z, double *u_re, double *u_im);

/* The solution read off a state z (packed FP64 device vector) without time stepping: the paper's
 * Step 6 output in time-discrete form, exact for the time-discrete periodic state.
 *  F2 (Step 6, eq. TH_SOLUTION): u = u_0 + i v_1 / wh with wh = sin(omega dt) / dt on the free
 *    nodes, gD on the sound-soft nodes.  Without sound-soft nodes a minimiser may be shifted by
 *    a constant (Thm 1), which is removed by the compatibility condition (eq. CC):
 *    the constant lam with 1^T [S - wt^2 M - i wh B] (u - lam) = 1^T Fhat, wt = 2 sin(omega dt
 *    / 2) / dt.  A pure-Neumann box returns CMCG_EUNSUPPORTED (its mode eta is invisible here;
 *    the filter handles it).
 *  F1 (eq. mix_solution): u = i V / omega from the cell rows of the time-discrete system,
 *    V = dt c^2 (Fhat + D Q) / (-2 i sin(theta) + 2 gamma cos(theta)), theta = omega dt / 2,
 *    with the flux amplitude Q = P_0 / cos(theta) + i dt G v_0 / (2 sin(theta)); divergence-free
 *    flux fields (the non-uniqueness of Thm 2) do not change it.
 * Single-frequency sources only (CMCG_EINVAL with shots).  u_re, u_im: host or device, layout
 * of c. */
cmcg_status cmcg_step6(cmcg_handle *h, const double *z, double *u_re, double *u_im);

/* The solve split in three: cmcg_begin (z = 0, Steps 1-4), cmcg_iterate (up to `iters` CG
 * iterations of Step 5; stops early at tol), cmcg_finish (filter + copy out).  cmcg_solve is
 * begin + iterate(max_iter) + finish.  *converged is set to 1 once tol is met. */
cmcg_status cmcg_begin(cmcg_handle *h);
cmcg_status cmcg_iterate(cmcg_handle *h, int32_t iters, int32_t *converged, cmcg_report *rep);
cmcg_status cmcg_finish(cmcg_handle *h, double *u_re, double *u_im, cmcg_report *rep);

/* Copy the current CG iterate z (which = 0), residual r (1) or direction d (2) into a packed
 * FP64 device vector. */
cmcg_status cmcg_get_state(cmcg_handle *h, int32_t which, double *out);

/* Long-time integration without controllability (Sec. 4.2.2, the "do-nothing" approach) and
 * the run-up of Sec. 4.2.3: the forced scheme from rest over `periods` >= 1 periods, in FP64,
 * the source multiplied by Mur's transient theta_tr (t_tr = periods T) if ramp != 0.  Writes
 * the state at t = periods T into z_out (packed FP64 device vector of state_len; cmcg_filter
 * extracts U from it).  Does not touch the CG state. */
cmcg_status cmcg_runup(cmcg_handle *h, int32_t periods, int32_t ramp, double *z_out);

/* Periodicity misfit J(z) = 1/2 (Phi(z) - z)^T M_E (Phi(z) - z) of a packed FP64 device state
 * (eq. cost_functional_J / eq. mix_cost_functional_J, discrete), computed with one FP64 forced
 * period.  The paper's relative misfit divides sqrt(J) by ||f|| + ||g_S|| (Sec. 4.2.1). */
cmcg_status cmcg_misfit(cmcg_handle *h, const double *z, double *J);

/* ---- allocation-free stage call ----
 * For callers that cannot allocate device memory where they call: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The operator of cmcg_apply on
 * a first-order problem, without a handle: the library lays out the problem's coefficient and
 * source fields and the period's working states in one fixed device buffer of
 * CMCG_STATIC_SCRATCH_BYTES per GPU (a static device array, held until the process ends), so
 * the call allocates nothing: no device, pinned-host, stream or event allocation.
 * Arguments: problem and options as for cmcg_create (precision, device, steps_per_launch and
 * hip_stream are used; NULL hip_stream runs on the null stream; tol and max_iter must be valid),
 * then op, steps, in and out as for cmcg_apply (packed FP64 device vectors of the problem's
 * state length; they may alias).  The result equals cmcg_apply's bit for bit.
 * Errors: CMCG_ENOMEM, before any device work, when the problem's fields do not fit the buffer
 * (first-order grids up to about 500 x 500 cells in FP64, 450 x 450 in FP32-mixed);
 * CMCG_EUNSUPPORTED for second-order problems; the validation errors of cmcg_create.
 * The buffer is shared by every call on a GPU and keeps the last call's contents; each call
 * clears what it uses.  Calls that overlap on one GPU (other threads, or concurrently running
 * streams) race on it.  Returns after the work on its stream has finished. */
#define CMCG_STATIC_SCRATCH_BYTES (64ull << 20)
cmcg_status cmcg_apply_static(const cmcg_problem *problem, const cmcg_options *opts, int32_t op,
                              int32_t steps, const double *in, double *out);

/* ---- continuous-batching server (first-order 2D solves) ----
 * Solves of different grid sizes and frequencies share the GPU: submitted requests wait in
 * arrival order until their device footprint fits the HBM budget and a slot is free; admitted
 * requests keep their CG state resident.  Each cmcg_server_step (a tick) is ONE launch of a
 * persistent kernel on a co-resident grid: it advances every running solve through rounds of
 * its CG algorithm (Sec. 2.3, with the FP64 refreshes of FP32-mixed solves), one operation per
 * solve per round (a launch of a period's leapfrog steps, a CG vector pass, a reduction or a
 * decision, all taken on the device), with a grid barrier between rounds, until its work budget
 * is spent or the solves have finished; the host then hands out finished results and admits
 * waiting requests.  A solve's result does not depend on what it shares the GPU with: it equals
 * the single-solve path's bit for bit.  Not thread-safe. */
typedef struct cmcg_server cmcg_server;

typedef struct {
  int64_t hbm_budget_bytes;    /* admission budget for the resident solves' device memory     */
  int32_t max_slots;           /* cap on concurrently resident solves (0 = 16)                 */
  int32_t steps_per_launch;    /* leapfrog steps per launch (0 = library default)              */
  int32_t device;
  void *hip_stream;            /* stream for all server work, or NULL                          */
  int64_t barrier_spin_limit;  /* polls a workgroup of the serving kernel makes at a grid barrier
                                  before it gives up (0 = default, about 16 M); a tick whose
                                  barrier gave up fails its running solves (CMCG_EDEVICE)      */
} cmcg_server_options;

enum { CMCG_REQ_QUEUED = 0, CMCG_REQ_RUNNING = 1, CMCG_REQ_DONE = 2, CMCG_REQ_FAILED = -1 };

cmcg_status cmcg_server_create(const cmcg_server_options *opts, cmcg_server **out);
/* Copies the problem's host arrays; the request starts queued.  opts->precision, tol and
 * max_iter apply to this solve; its stream is the server's.  *id identifies it in poll.
 * Served solves start from rest and have a single-frequency source (CMCG_EUNSUPPORTED for a
 * run-up or shots). */
cmcg_status cmcg_server_submit(cmcg_server *s, const cmcg_problem *p, const cmcg_options *opts,
                               int64_t *id);
/* One tick: admit what fits, advance the running solves, finish those that are done.  Optional
 * counts: *active = the solves the tick advanced (resident during it, finished ones included),
 * *queued = the requests still waiting for admission after it. */
cmcg_status cmcg_server_step(cmcg_server *s, int32_t *active, int32_t *queued);
/* *state = CMCG_REQ_*; when DONE, copies the filtered solution (host arrays, layout of c) and
 * the report, and returns the solve's status (CMCG_OK or CMCG_ENOTCONV); when FAILED, returns
 * the failure status.  The poll that reports DONE or FAILED releases the request: its id is
 * unknown afterwards (CMCG_EINVAL). */
cmcg_status cmcg_server_poll(cmcg_server *s, int64_t id, int32_t *state, double *u_re,
                             double *u_im, cmcg_report *rep);
/* Device bytes held by resident solves, and the running / queued counts. */
cmcg_status cmcg_server_stats(const cmcg_server *s, int64_t *used_bytes, int32_t *active,
                              int32_t *queued);
/* Ticks that advanced solves, the kernel launches those ticks made (the persistent serving
 * kernel's; the field setup of admitted requests is not counted) and the rounds those launches
 * ran (one operation of every resident solve each). */
cmcg_status cmcg_server_launches(const cmcg_server *s, int64_t *ticks, int64_t *launches,
                                 int64_t *rounds);
void cmcg_server_destroy(cmcg_server *s);   /* NULL-safe */

#ifdef __cplusplus
}
#endif

#endif /* CMCG_H */
