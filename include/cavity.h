/*
 * cavity.h -- C ABI of the MI355X driven-lid-cavity time stepper.
 *
 * The library advances the two-dimensional incompressible Navier-Stokes
 * equations in vorticity-stream function form on the unit square with a
 * moving lid (N. Cardoso and P. Bicudo, "Time dependent simulation of the
 * Driven Lid Cavity at High Reynolds Number", arXiv:0809.3098):
 *
 *   - Sec. 2, eqs. (vort0), (stream0), (str), (vortfinal): the model;
 *   - Sec. 3, eq. (Lwn): central-difference right-hand side for omega;
 *   - Sec. 3, eqs. (SSPRK54_1)-(SSPRK54_5): SSPRK(5,4) time integration;
 *   - Sec. 3, eqs. (stream_4O), (SequationFinal): fourth-order compact
 *     stream equation, solved by successive over-relaxation;
 *   - Sec. 3, eq. (vel): velocities from psi;
 *   - Sec. 3.1: psi = 0 on the walls, Thom's wall vorticity;
 *   - Sec. 3.2: Re = |U| L / nu with L = 1, monitors RES_psi, RES_omega
 *     (eqs. resS, resV).
 *
 * Every entry point returns an int status (CAVITY_OK = 0 or a negative
 * cavity_status); no C++ exception crosses this boundary.  After a failure
 * cavity_last_error() returns a message for the calling thread.
 *
 * Field layout: every field exchanged through this ABI is an n x n array of
 * IEEE double, row-major, indexed [j][i] with i the x index (fastest) and j
 * the y index; node (i, j) sits at (i h, j h), h = 1/(n-1); the moving lid is
 * row j = n-1.  Field pointers are DEVICE pointers on the device that owns
 * the handle's stream; the library never keeps them after the call returns.
 *
 * Streams: all work is enqueued on the hip_stream given to cavity_create
 * (NULL = the null stream).  Calls that return host results (stats, info)
 * synchronise that stream before returning; the others only enqueue.
 */
#ifndef CAVITY_H
#define CAVITY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum cavity_status {
  CAVITY_OK = 0,
  CAVITY_EINVAL = -1,     /* invalid argument (message says which)            */
  CAVITY_ENOMEM = -2,     /* workspace too small                               */
  CAVITY_EHIP = -3,       /* a HIP runtime call failed                         */
  CAVITY_ENOCONV = -4,    /* a Poisson solve hit poisson_max_sweeps; the step
                             completed with the last iterate and the state stays
                             usable                                            */
  CAVITY_ENONFINITE = -5, /* NaN/Inf met in a residual; the handle is poisoned */
  CAVITY_ESTATE = -6      /* handle poisoned by an earlier ENONFINITE/EHIP     */
};

/* Arithmetic of the Poisson smoother and stencil sweeps. */
enum cavity_precision {
  CAVITY_FP64 = 0,   /* everything in double precision (the paper's setting)   */
  CAVITY_MIXED = 1   /* FP32 smoother sweeps and FP32 transport stencil with
                        FP64 residual, FP64 iterative refinement of psi, FP64
                        stage accumulation of omega and FP64 wall vorticity    */
};

/* Starting value of the Poisson solve of each SSPRK stage (Sec. 3, eqs.
 * SSPRK54_1-5 with eq. SequationFinal per stage).  The paper does not say
 * what a solve starts from; a converged solve ends within poisson_tol of the
 * same discrete solution from any start, so the choice changes the number of
 * sweeps, not the result beyond that tolerance.  Values of
 * cavity_params.warm_start:
 *   0 (CAVITY_WARM_DEFAULT): for converged solves CAVITY_WARM_LEVELS_FP64
 *     levels in FP64 (interpolated) and CAVITY_WARM_LEVELS_MIXED in mixed
 *     precision (the least-squares polynomial of degree
 *     CAVITY_WARM_DEGREE_MIXED through them), the fastest on the 1024^2
 *     workloads (more levels, or a higher degree, pass on more of the
 *     solves' own tolerance-level differences, amplified by the
 *     extrapolation weights); CAVITY_WARM_PREVIOUS in the coupled mode
 *     (fixed_sweeps > 0, whose fixed iteration starts from the previous
 *     stage's psi by definition);
 *   1 (CAVITY_WARM_PREVIOUS): the psi of the stage before;
 *   2 ... 8 (levels): the polynomial through the same stage's solutions of
 *     the last `levels` steps, evaluated at the current step.  Consecutive
 *     steps' solutions of one stage differ by O(dt); the extrapolation error
 *     is O(dt^levels).  Costs 5 * levels FP64 fields of workspace.  Right
 *     after cavity_create (also with resume = 1) no step is on file: the
 *     first steps use the steps on file, and the previous stage's psi while
 *     fewer than two are. */
enum cavity_warm_start {
  CAVITY_WARM_DEFAULT = 0,
  CAVITY_WARM_PREVIOUS = 1,
  CAVITY_WARM_LEVELS_FP64 = 6,
  CAVITY_WARM_LEVELS_MIXED = 8,
  CAVITY_WARM_DEGREE_MIXED = 5,
  CAVITY_WARM_LEVELS_MAX = 8
};

/* Parameters of one cavity (Sec. 3.2: unit square, lid speed U on top). */
typedef struct cavity_params {
  int32_t n;                  /* nodes per side including walls, 5 <= n <= 16385   */
  int32_t precision;          /* enum cavity_precision                            */
  double re;                  /* Reynolds number > 0; nu = |u_lid| / re            */
  double u_lid;               /* lid speed U (sign allowed); 0 needs dt > 0 and nu  */
  double nu;                  /* > 0 overrides the viscosity derived from re        */
  double dt;                  /* > 0: fixed time step; <= 0: dt = cfl * h / |u_lid|  */
  double cfl;                 /* used when dt <= 0; <= 0 means 0.5                  */
  double poisson_tol;         /* stop when max-norm residual of the compact stream
                                 equation, in vorticity units, is <= this; <= 0
                                 means 1e-10                                       */
  int32_t poisson_max_sweeps; /* per solve; <= 0 means 200 * n                      */
  int32_t resume;             /* 1: omega0 and psi0 (both required) are a state
                                 saved by cavity_fields after a step and are
                                 adopted as they are, walls included, without a
                                 Poisson solve, so the run continues exactly
                                 with warm_start = CAVITY_WARM_PREVIOUS and
                                 within the solve tolerance otherwise (the
                                 extrapolation history starts empty)              */
  double sor_omega;           /* relaxation parameter in (0, 2); <= 0 chooses,
                                 for the coupled mode, w5 = 2 / (1 + sin(pi h)),
                                 and for converged solves w5 - 5/8 (w5 - w9),
                                 w9 = 2 / (1 + sqrt(1 - mu^2)), mu = 0.8 cos(pi h)
                                 + 0.2 cos^2(pi h) (faster for the four-colour
                                 order; the converged result does not depend
                                 on it)                                            */
  const double* omega0;       /* nullable device n*n initial vorticity (walls are
                                 replaced by Thom's values); NULL = fluid at rest   */
  const double* psi0;         /* nullable device n*n warm start for the first
                                 Poisson solve (or the saved psi when resume = 1);
                                 its wall values are ignored (psi = 0 on walls);
                                 NULL = zeros                                      */
  int32_t fixed_sweeps;       /* 0: every stage solves the stream equation to
                                 poisson_tol.  > 0: coupled mode of Sec. 3 eq.
                                 (SequationFinal) as a fixed iteration -- every
                                 stage relaxes psi exactly this many four-colour
                                 sweeps with parameter sor_omega (the relaxation
                                 beta; Sec. 4 reports 0.8 down to 0.1 as Re
                                 grows), starting from the previous stage's psi,
                                 with no stopping test.  Needs CAVITY_FP64, the
                                 SOR solver and CAVITY_EXEC_STREAM; the initial
                                 solve of cavity_create and cavity_poisson still
                                 solve to poisson_tol                              */
  int32_t warm_start;         /* enum cavity_warm_start: 0, 1 or 2 ... 8 levels;
                                 0 or 1 when fixed_sweeps > 0                      */
} cavity_params;

/* Per-cavity results of cavity_step. */
typedef struct cavity_stats {
  int64_t step;               /* steps taken since create                          */
  double t;                   /* simulated time                                    */
  double dt;                  /* time step in use                                  */
  double res_psi;             /* RES_psi of the last step (eq. resS), sum / n      */
  double res_omega;           /* RES_omega of the last step (eq. resV), sum / n    */
  double domega_inf_over_dt;  /* max |omega^{n+1} - omega^n| / dt                  */
  double ke;                  /* 0.5 h^2 sum over interior of (u^2 + v^2)          */
  double last_resid_inf;      /* residual max-norm at the end of the last solve    */
  int64_t sweeps_total;       /* relaxation sweeps since create                    */
  int64_t sweeps_last_step;   /* relaxation sweeps in the last step (5 solves)     */
  int32_t floor_limited;      /* 1 if a solve of the last step stopped at the
                                 rounding floor above poisson_tol                   */
  int32_t status;             /* CAVITY_OK / CAVITY_ENOCONV for this cavity        */
} cavity_stats;

/* Result of a stand-alone Poisson solve. */
typedef struct cavity_poisson_info {
  int64_t sweeps;             /* relaxation sweeps performed                       */
  double resid_inf;           /* final residual max-norm (vorticity units)        */
  int32_t floor_limited;      /* see cavity_stats                                  */
  int32_t status;             /* CAVITY_OK or CAVITY_ENOCONV                      */
} cavity_poisson_info;

typedef struct cavity_s* cavity_t;

/*
 * Device workspace needed for `count` cavities with parameters p[0..count-1].
 * Writes the byte count to *bytes.  EINVAL on bad parameters.
 */
int cavity_workspace_bytes(const cavity_params* p, int32_t count, size_t* bytes);

/*
 * Create a handle for `count` independent cavities (count > 1 is the batched
 * Reynolds sweep: every cavity advances in the same calls).
 *   p          host array[count] of parameters; read during the call only.
 *   d_ws       caller-owned device buffer of ws_bytes bytes (>= the size from
 *              cavity_workspace_bytes), 256-byte aligned, kept alive and
 *              untouched by the caller until cavity_destroy.
 *   hip_stream hipStream_t (NULL = null stream) all work is enqueued on.
 *   out        receives the handle.
 * The initial state is omega0 (or rest), psi solved from it with the compact
 * equation (Sec. 3) and the wall vorticity set by Thom's formula (Sec. 3.1).
 * Synchronises the stream.  Errors: EINVAL, ENOMEM, EHIP, ENOCONV, ENONFINITE.
 */
int cavity_create(const cavity_params* p, int32_t count, void* d_ws, size_t ws_bytes,
                  void* hip_stream, cavity_t* out);

/*
 * Advance every cavity by nsteps SSPRK(5,4) steps (eqs. SSPRK54_1-5).  Each
 * stage evaluates eq. (Lwn) with eq. (vel), combines interior nodes, solves
 * the compact stream equation by four-colour SOR (eq. SequationFinal) to
 * poisson_tol, and refreshes the wall vorticity by Thom's formula.
 *   stats  nullable host array[count]; when given, the monitors of the last
 *          step are computed and the call synchronises the stream.
 * Returns ENOCONV if any solve hit its sweep limit (state still valid),
 * ENONFINITE if a residual was not finite (handle poisoned), ESTATE on a
 * poisoned handle.
 */
int cavity_step(cavity_t h, int32_t nsteps, cavity_stats* stats);

/*
 * Advance every cavity until it reaches a steady state in the sense of
 * Sec. 4: the monitors RES_psi and RES_omega of one step (eqs. resS, resV)
 * both at or below their thresholds.  The monitors are evaluated on the last
 * step of every group of check_every steps; the run stops once every cavity
 * has met its thresholds, or after max_steps steps.  Cavities that met them
 * keep advancing with the others (a steady state stays steady).
 *   max_steps      >= 1, steps of this call at most.
 *   check_every    >= 1, steps between monitor evaluations.
 *   res_psi_tol, res_omega_tol
 *                  nullable host arrays[count] of thresholds (> 0); NULL takes
 *                  the values of Sec. 4: 1e-12 and 1e-10 for Re <= 20 000,
 *                  1e-10 and 1e-8 above (Re = |u_lid| / nu).
 *   steady_step    host array[count], out: the step count since create at
 *                  which the cavity first met its thresholds, -1 if it did
 *                  not within this call.
 *   stats          nullable host array[count]: results of the last step.
 * Synchronises the stream after every group.  Errors as cavity_step; not
 * reaching a steady state is not an error (steady_step = -1).
 */
int cavity_run_steady(cavity_t h, int64_t max_steps, int32_t check_every,
                      const double* res_psi_tol, const double* res_omega_tol,
                      int64_t* steady_step, cavity_stats* stats);

/*
 * Solve the compact stream equation for cavity idx.
 *   d_omega  nullable device n*n vorticity (walls included, used as given);
 *            NULL solves for the handle's current vorticity in place.
 *   d_psi    nullable device n*n output for psi.
 *   info     nullable host result; when given the call synchronises.
 * With d_omega != NULL the handle's state is not modified.
 */
int cavity_poisson(cavity_t h, int32_t idx, const double* d_omega, double* d_psi,
                   cavity_poisson_info* info);

/*
 * Allocation-free Poisson solve, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid allocation): the same
 * FP64 four-colour SOR solve of the compact stream equation as cavity_poisson
 * with a vorticity given (from a zero start, with the relaxation, sweep kernel
 * and residual-check spacing a cavity of this n gets by default, so the result
 * is bitwise that of cavity_poisson on such a cavity), without a handle.  Its
 * right-hand side, iterate pair, partial maxima and control block live in a
 * device array of the library, 24 MiB + 64 KiB per device, held from the
 * first call on a device until the process ends; the call allocates no memory
 * (no hipMalloc, hipFree or host pinning).  Every call on one device uses
 * that device's array: calls that overlap on one device (other host threads,
 * other streams) race and must not be made.
 *   n              5 <= n <= 1024 (nodes per side including walls); larger n
 *                  -> CAVITY_EINVAL
 *   poisson_tol    as in cavity_params (<= 0 means 1e-10)
 *   sor_omega      as in cavity_params (<= 0: the default relaxation)
 *   poisson_max_sweeps  as in cavity_params (0 means 200 * n)
 *   d_omega        device n*n vorticity (walls included), read only
 *   d_psi          device n*n output for psi (walls 0)
 *   hip_stream     stream of the current device the work is enqueued on
 *   info           nullable host result
 * Synchronises the stream (the host reads the stopping decision).  Errors:
 * EINVAL, EHIP, ENOCONV (psi holds the last iterate), ENONFINITE.
 */
int cavity_poisson_noalloc(int32_t n, double poisson_tol, double sor_omega,
                           int32_t poisson_max_sweeps, const double* d_omega, double* d_psi,
                           void* hip_stream, cavity_poisson_info* info);

/*
 * Copy out the fields of cavity idx as device n*n double arrays; each pointer
 * is nullable.  u, v follow eq. (vel) inside and the wall values of Sec. 3.1
 * (u = U on the lid row except its corners, 0 elsewhere; v = 0 on walls).
 */
int cavity_fields(cavity_t h, int32_t idx, double* d_psi, double* d_omega, double* d_u,
                  double* d_v);

/*
 * Apply `sweeps` relaxation sweeps of eq. (SequationFinal) in four-colour
 * order (rounded up to a whole number of kernel launches) with no convergence
 * check and no host synchronisation; the handle's state is not modified.
 *   arith 0: FP64 sweeps on a scratch copy of cavity idx's psi for the
 *            right-hand side of its current vorticity; the result is copied to
 *            d_psi_out (nullable device n*n).
 *   arith 1: FP32 sweeps of the correction equation for the FP64 residual of
 *            the current psi (cavity idx must be CAVITY_MIXED); d_psi_out must
 *            be NULL.
 * Writes the number of sweeps performed to *done (nullable).  Used to time
 * the smoothers alone and to apply a fixed number of sweeps.
 */
int cavity_relax(cavity_t h, int32_t idx, int32_t sweeps, int32_t arith, double* d_psi_out,
                 int64_t* done);

/*
 * Launch configuration of a cavity's Poisson smoother.  The sweep kernel loads
 * a tile_x x tile_y tile of psi plus a halo into LDS (and the right-hand side
 * of the nodes each thread updates into registers) and runs
 * sweeps_per_launch four-colour sweeps there; only compiled combinations are
 * accepted (EINVAL otherwise).  Results do not depend on the
 * tile shape or thread count; sweeps_per_launch, check_every and sor_omega
 * change the sweep schedule and so the last bits of the converged result.
 */
typedef struct cavity_tuning {
  int32_t tile_x, tile_y;        /* FP64 sweep kernel tile (nodes)                 */
  int32_t sweeps_per_launch;     /* sweeps per FP64 launch                          */
  int32_t threads;               /* threads per block of the FP64 kernel            */
  int32_t tile_x32, tile_y32;    /* FP32 correction sweeps (CAVITY_MIXED)          */
  int32_t sweeps_per_launch32;
  int32_t threads32;
  int32_t check_every;           /* FP64: sweeps between residual checks (rounded
                                    up to whole launch pairs)                     */
  int32_t inner_sweeps;          /* mixed: FP32 sweeps per refinement round        */
  int32_t xcd_bands;             /* 1: each XCD relaxes a contiguous band of tiles */
  int32_t solver;                /* enum cavity_solver                              */
  double sor_omega;              /* relaxation parameter in (0, 2)                 */
  int32_t warm_degree;           /* extrapolated warm starts (warm_start = L >= 2
                                    levels): degree d of the polynomial through the
                                    L steps on file, 1 <= d <= L - 1; d = L - 1
                                    interpolates them, a lower degree is their
                                    least-squares fit, which passes on less of the
                                    solves' own tolerance-level differences
                                    (default: L - 1 in FP64, at most
                                    CAVITY_WARM_DEGREE_MIXED in mixed precision).
                                    0 in cavity_set_tuning keeps the current degree;
                                    cavity_get_tuning reports 0 when the cavity
                                    has no extrapolated starts                      */
} cavity_tuning;

/*
 * Poisson solver of a cavity.  Both converge the same compact equation
 * (eq. SequationFinal's fixed point) to poisson_tol.
 *   CAVITY_SOLVER_SOR  four-colour SOR, the paper's relaxation (default)
 *   CAVITY_SOLVER_MG   geometric multigrid V(2,2)-cycles: four-colour
 *                      Gauss-Seidel smoothing with the same sweep kernel,
 *                      the compact operator rediscretised on coarser grids
 *                      (m intervals -> ceil(m/2); non-nested levels use
 *                      bilinear transfers in physical coordinates).  In
 *                      CAVITY_MIXED each refinement round is one FP32
 *                      V-cycle on the correction.  CAVITY_EXEC_STREAM only
 */
enum cavity_solver { CAVITY_SOLVER_SOR = 0, CAVITY_SOLVER_MG = 1 };

/*
 * Read / replace the launch configuration of cavity idx (host only).  idx = -1
 * addresses the batched persistent kernel shared by every cavity of the handle
 * (its sor_omega and xcd_bands are unused; each cavity keeps its own
 * relaxation parameter).  Replacing a configuration discards captured graphs.
 */
int cavity_get_tuning(cavity_t h, int32_t idx, cavity_tuning* t);
int cavity_set_tuning(cavity_t h, int32_t idx, const cavity_tuning* t);

/*
 * How cavity_step runs the Poisson solves.
 *   CAVITY_EXEC_STREAM      one launch per S sweeps, every cavity on its own;
 *                           the host reads each solve's decision once per chunk
 *                           of enqueued launches (default for one cavity, and
 *                           for several when one has n > 512).
 *                           With several cavities each runs on a stream of its
 *                           own (created by the handle, default priority),
 *                           forked from the handle's stream at the start of a
 *                           step and joined back at its end, so that small
 *                           cavities use the CUs a large one leaves idle.
 *   CAVITY_EXEC_PERSISTENT  one persistent launch per stage solves every cavity
 *                           of the handle (tile list over all cavities, grid
 *                           barriers between sweep rounds, per-cavity stopping
 *                           decisions on the device); one readback per step.
 *   CAVITY_EXEC_RESIDENT    as STREAM, but an FP64 SOR solve of a cavity whose
 *                           tiles fit the device at once runs as one launch:
 *                           one block per tile for the whole solve keeps its
 *                           tile on chip and swaps halos with its neighbours
 *                           after every few sweeps; the residual is checked as
 *                           often as in STREAM and the solve stops two rounds
 *                           of sweeps after the check that ends it (so its
 *                           sweep counts, and results to within the
 *                           tolerance, differ from STREAM).  Other cavities
 *                           (mixed, multigrid, coupled, too large) run as in
 *                           STREAM.
 *   CAVITY_EXEC_GRAPH       as PERSISTENT, with the whole step (five stages)
 *                           captured once per buffer parity in a hipGraph and
 *                           replayed (default for count > 1 when every cavity
 *                           has n <= 512: cavities too small to fill the GPU
 *                           alone are fused into one launch).  When every
 *                           cavity is in the coupled mode (fixed_sweeps > 0)
 *                           the graph holds the per-launch sweeps instead.
 * Both persistent modes need one precision for all cavities and the SOR
 * solver; a coupled cavity allows STREAM and RESIDENT, and GRAPH only if all
 * cavities of the handle are coupled (EINVAL otherwise).  With the same tile
 * sweeps per launch, check spacing and relaxation, STREAM, PERSISTENT and
 * GRAPH give bitwise identical results.
 */
enum cavity_exec {
  CAVITY_EXEC_STREAM = 0,
  CAVITY_EXEC_PERSISTENT = 1,
  CAVITY_EXEC_GRAPH = 2,
  CAVITY_EXEC_RESIDENT = 3
};
int cavity_set_exec(cavity_t h, int32_t mode);
int cavity_get_exec(cavity_t h, int32_t* mode);

/*
 * Autotuner.  For cavity idx: times every compiled sweep kernel (tile shape,
 * sweeps per launch, threads, XCD-banded tile order) with back-to-back
 * launches and keeps the fastest per FP64 / FP32 smoother; then chooses the
 * sweep schedule (FP64: residual-check spacing; mixed: FP32 sweeps per
 * refinement round) by timing complete Poisson solves of the cavity's current
 * vorticity.  For idx = -1: times the batched persistent kernel per tile shape.
 * Measurements use scratch buffers; the simulation state is not modified
 * (results may differ in the last bits afterwards, since the schedule does).
 * cache_path (nullable): a JSON-lines file; an entry for the same key (device
 * architecture, n, precision, batch members) is applied without measuring,
 * and a new result is appended.  The applied tuning is returned in *chosen
 * (nullable).  Synchronises the stream; takes a few seconds.
 */
int cavity_autotune(cavity_t h, int32_t idx, const char* cache_path, cavity_tuning* chosen);

/* Release the handle (host memory only; the workspace stays the caller's). */
int cavity_destroy(cavity_t h);

/* The weights of the warm start of a stage solve (see enum cavity_warm_start;
 * Sec. 3, eqs. SSPRK54_1-5 with eq. SequationFinal per stage): with `levels`
 * steps on file, the start is sum_q w[q-1] psi(step - q), q = 1 ... levels,
 * the value at the current step of the polynomial of the given degree through
 * the same stage's solutions of those steps (interpolation for degree =
 * levels - 1, least squares below).  The same weights the device applies.
 * Host only (no device, no handle); w (host) receives `levels` doubles.
 * CAVITY_EINVAL for levels outside [2, CAVITY_WARM_LEVELS_MAX], degree
 * outside [1, levels - 1] or w NULL. */
int cavity_warm_weights(int32_t levels, int32_t degree, double* w);

/* Message of the last failure on the calling thread ("" if none). */
const char* cavity_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CAVITY_H */
