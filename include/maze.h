/*
 * maze.h -- C ABI of libmaze.so, the MI355X (gfx950) implementation of the
 * Poisson MaZe per-timestep hot path:
 *
 *   charge assignment onto a periodic grid  ->  PLCG solve of the SHAKE
 *   constraint system, warm-started from the previous step  ->  force
 *   interpolation back onto the ions.
 *
 * Paper: Troni, Grassano, Narayan, Roux, Bonella, "Mass-Zero constrained
 * molecular dynamics for electrostatic interactions", arXiv 2505.20418.
 *
 * Common conventions
 *  - Units are Gaussian inside: charge in e, length in A, potential in e/A.
 *    `coulomb_k` scales every energy and force (1.0 -> e^2/A and e^2/A^2,
 *    14.3996454784 -> eV and eV/A).
 *  - Cubic periodic box of side `box`. N = lround(box / grid_spacing) grid
 *    points per side, effective spacing h = box / N (Section 2, equation
 *    "linearproblem"). Grid point (i, j, k) sits at (i h, j h, k h); grids
 *    are N*N*N contiguous doubles, index (i*N + j)*N + k (z fastest).
 *  - Positions are n*3 contiguous doubles (x, y, z per ion); positions may
 *    lie outside [0, box) and are wrapped periodically. Forces use the same
 *    layout.
 *  - Every pointer argument named *_dev is DEVICE memory on the current HIP
 *    device (e.g. torch.Tensor.data_ptr()); the caller owns it and keeps it
 *    alive until the call returns. Host pointers are named explicitly.
 *  - Work is queued on cfg.stream (NULL = the default stream). Each solve
 *    polls its convergence flag from the host, so the step entry points
 *    return once the solver has converged; the remaining kernels (field
 *    update, force interpolation) may still be running on the stream. A
 *    non-NULL maze_stats* makes the call synchronise the stream before it
 *    returns.
 *  - A session is not thread safe; different sessions are independent.
 *  - Return codes: MAZE_OK; MAZE_NOT_CONVERGED (> 0, a warning: outputs
 *    were written and the state advanced); negative = error, nothing was
 *    written and the state is unchanged.
 */
#ifndef MAZE_H
#define MAZE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MAZE_ABI_VERSION 2

typedef struct maze_session maze_session;

enum {
  MAZE_OK = 0,
  MAZE_NOT_CONVERGED = 1,   /* max_iter reached or CG breakdown */
  MAZE_E_INVALID = -1,      /* bad argument, config or buffer */
  MAZE_E_NOT_NEUTRAL = -2,  /* |sum Q| > 1e-10 sum |Q| */
  MAZE_E_OOM = -3,          /* device allocation failed */
  MAZE_E_DEVICE = -4,       /* HIP runtime error */
  MAZE_E_NONFINITE = -5,    /* NaN or Inf in the positions */
  MAZE_E_CAPACITY = -6      /* request exceeds a fixed capacity
                               (maze_step_batch_noalloc) */
};

enum { MAZE_FP64 = 0, MAZE_MIXED = 1 };
enum { MAZE_GUESS_ZERO = 0, MAZE_GUESS_STATIC = 1, MAZE_GUESS_TIMEPROP = 2 };
enum { MAZE_NORM_REL2 = 0, MAZE_NORM_ABSMAX = 1 };
enum {
  MAZE_FLAG_MULTIGRID = 1,
  /* forces by equation "F_Benoit" (-k Q sum grad W phi, the derivative on
     the assignment weights) instead of equation "F_nostra"; not momentum
     conserving, for the comparison of force estimators */
  MAZE_FLAG_WEIGHT_GRADIENT_FORCE = 2,
  /* accept charges that do not sum to zero: the zero-mode projection then
     acts as a uniform neutralising background (the single-charge
     measurements of the two-particle appendix) */
  MAZE_FLAG_ALLOW_NET_CHARGE = 4,
  /* issue the CG iterations after the first poll as replays of a captured
     HIP graph of kPollBatch sweeps (instantiated on first use per
     precision, parity and solution vector, up to 4 per precision and
     parity, freed by maze_destroy) instead of kernel by kernel; same
     kernels and arguments, so results are bitwise those without it. Needs a non-null cfg.stream (MAZE_E_INVALID otherwise);
     single-session solves only (batched and multigrid solves launch
     directly); ignored while maze_profile_enable is on. */
  MAZE_FLAG_GRAPH_CHUNKS = 8,
  /* run the Jacobi PLCG two iterations per pass pair: the s-step CG (s = 2)
     of Chronopoulos and Gear, whose iterates equal those of the PLCG of
     Appendix B in exact arithmetic. A basis kernel forms
     [p, Bp, B^2 p, r/6, B r/6] (B = A/6 - I) and its Gram sums; an
     update kernel applies two iterations' coefficients. 32 bytes per point
     per two iterations in FP32 (64 in FP64), against 48 (96). The test on
     the residual after the first of the two iterations uses its Gram form;
     with MAZE_NORM_ABSMAX the test runs every two iterations. Not with
     MAZE_FLAG_MULTIGRID (MAZE_E_INVALID). Batches run batched forms of both
     kernels; sessions without the flag in the same batch are solved as a
     batch of their own. */
  MAZE_FLAG_SSTEP = 16
};

typedef struct {
  int32_t n_ions;         /* > 0 */
  int32_t order;          /* assignment order: 2 = linear weights on the 8
                             nearest grid points (default), 4 = centred
                             cubic B-spline on 64 points */
  double  box;            /* L [A], > 0 */
  double  grid_spacing;   /* requested h [A]; 4 <= lround(L/h) <= 1024 */
  double  tol;            /* stopping tolerance, > 0. MAZE_NORM_REL2:
                             ||M y - sigma_p||_2 <= tol ||q||_2 for a step
                             (identical to the Poisson relative residual
                             ||M phi + 4 pi q/h|| / ||4 pi q/h||);
                             MAZE_NORM_ABSMAX: max|residual| <= tol */
  int32_t max_iter;       /* CG iteration cap per solve (>= 0) */
  int32_t precision;      /* MAZE_FP64 or MAZE_MIXED (FP32 stencil and
                             vectors, FP64 dots, norms, projection and an
                             outer refinement on the FP64 residual) */
  int32_t residual_norm;  /* MAZE_NORM_REL2 or MAZE_NORM_ABSMAX */
  int32_t flags;          /* bitwise OR of MAZE_FLAG_*; MAZE_FLAG_MULTIGRID: precondition the
                             PLCG with a geometric multigrid V-cycle (red-
                             black Gauss-Seidel, full-weighting restriction,
                             trilinear prolongation, CG on the coarsest
                             grid; the multigrid of the Results section)
                             instead of the Jacobi diagonal. The outer CG is
                             then FP64 in both precision modes; MAZE_MIXED
                             runs the V-cycle in FP32. Needs a grid that
                             halves down to at most 12^3 points. */
  double  coulomb_k;      /* energy/force scale, > 0 */
  void*   stream;         /* hipStream_t or NULL */
} maze_config;

typedef struct {
  int32_t grid_n;         /* N */
  int32_t iters;          /* CG iterations (sum over refinements) */
  int32_t refinements;    /* outer FP64 refinements (mixed), else 0 */
  int32_t converged;      /* 1 if the stopping test was met */
  int32_t status;         /* status of the call for this session (batch) */
  int32_t pad;
  double  h;              /* effective grid spacing */
  double  rel_residual;   /* true ||residual||_2 / ||rhs scale||_2, FP64 */
  double  max_abs_residual;
  double  net_charge;     /* sum of the assigned grid charge before the
                             zero-mode projection */
  double  energy;         /* (1/2) k phi.q, equation "energy_discr" */
} maze_stats;

/* Library version of this header's ABI. */
int maze_abi_version(void);

/* Human-readable text of a status code (static storage). */
const char* maze_strerror(int status);

/* Device bytes a session with this config allocates (for admission by HBM
 * budget). Returns 0 for an invalid config. */
size_t maze_device_bytes(const maze_config* cfg);

/* Creates a session: validates cfg, copies the charges (fixed for the
 * session's lifetime), allocates every device buffer (the only allocation
 * of the session), assigns the charges of pos0 and performs a cold Poisson
 * solve from zero for phi^0 (the paper's pseudocode figure is not
 * available; this reading also sets phi^{-1} = phi^0 and y = 0).
 * charges_dev: n_ions doubles; pos0_dev: n_ions*3 doubles.
 * On success *out holds the session (free with maze_destroy). Errors:
 * MAZE_E_INVALID, MAZE_E_NOT_NEUTRAL, MAZE_E_NONFINITE, MAZE_E_OOM,
 * MAZE_E_DEVICE; *out is NULL then. */
int maze_init(const maze_config* cfg, const double* charges_dev,
              const double* pos0_dev, maze_session** out, maze_stats* st);

/* One MaZe step k -> k+1 (Section 2, equations "SHAKE", "SHAKEy" and
 * "SHAKEPhiFinal"; Appendix B for the Jacobi PLCG):
 *   q       = charge assigned from pos_dev (positions r^{k+1}), projected
 *             to zero mean
 *   phi_p   = 2 phi^k - phi^{k-1}
 *   sigma_p = (h / 4 pi) M phi_p + q
 *   M y     = sigma_p  by Jacobi PLCG from y* of the previous step
 *   phi^{k+1} = phi_p - (4 pi / h) y*   (mean-zero gauge)
 *   forces  = equation "F_nostra": -k Q_a sum_n W(r_a - r_n) (D phi)_n with
 *             central differences
 *   energy  = (1/2) k phi^{k+1} . q
 * field_dev (N^3 doubles) and energy_dev (1 double) may be NULL;
 * forces_dev (n_ions*3 doubles) may be NULL. */
int maze_step(maze_session* s, const double* pos_dev, double* field_dev,
              double* forces_dev, double* energy_dev, maze_stats* st);

/* Direct Poisson solve of equation "linearproblem" for the charge of
 * pos_dev, from the guess named by `guess` (zero, "static" phi^k, or
 * "time-propagated" 2 phi^k - phi^{k-1}; convergence subsection). The MaZe
 * history (phi^k, phi^{k-1}, y*) is left untouched. Outputs as maze_step. */
int maze_solve(maze_session* s, int guess, const double* pos_dev,
               double* field_dev, double* forces_dev, double* energy_dev,
               maze_stats* st);

/* Advances `count` distinct sessions by one step each, with the CG sweeps
 * of all of them issued together: per CG iteration, one launch per template
 * class (segment length and halo width of the session's grid) covers every
 * unconverged session of a precision, and sessions that have converged drop
 * out. Sessions may differ in grid size and precision; they must share the
 * device and the stream of sessions[0]. Per-session semantics and outputs are
 * those of maze_step. Each session has two launch shapes (maze_launch_shape):
 * a batch whose sessions together need fewer than 256 workgroups in their
 * throughput shapes is swept in the latency shapes, and each session's
 * result is then bitwise the one it gets stepped alone; a larger batch is
 * swept in the throughput shapes, and each result then meets the session's
 * tolerance but sums in another order (MAZE_BATCH_MODE=latency or
 * =throughput in the environment forces one mode). pos_dev[i], forces_dev[i] (forces_dev or an entry may be
 * NULL) belong to session i; energies_dev (count doubles, device) and st
 * (count entries, host) may be NULL; st[i].status holds session i's status.
 * A session whose positions are rejected is left unchanged while the others
 * advance. The return value is the most severe status over the sessions.
 * The first call with more sessions than any call before on a device
 * allocates that device's batch table (device and pinned host memory kept
 * until the process ends); calls on one device must not overlap. */
int maze_step_batch(maze_session* const* sessions, int32_t count,
                    const double* const* pos_dev, double* const* forces_dev,
                    double* energies_dev, maze_stats* st);

/* maze_step_batch for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid allocation after start-up): the same
 * arguments, semantics, kernels and results as maze_step_batch (bitwise,
 * for the same batch), but the batch table lives in a fixed array in the
 * library's device data, one copy per GPU kept until the process ends,
 * instead of a table allocated by the first large call. The call itself
 * makes no device, pinned-host or event allocation (host bookkeeping uses
 * the C++ heap, as every entry point does). Limits: at most 256 sessions
 * per call (more: MAZE_E_CAPACITY, before any other check) and devices
 * 0..63. Every call on a device shares that device's table, so calls that
 * overlap on one device race (as calls of maze_step_batch do); nothing of a
 * previous call is read. The table's host mirror is ordinary (pageable)
 * memory, so each convergence poll waits for the work queued before it
 * instead of overlapping the next group of CG iterations: somewhat slower
 * than maze_step_batch on small grids. Sessions must have been created by
 * maze_init (which looks up the table's device address once per device). */
int maze_step_batch_noalloc(maze_session* const* sessions, int32_t count,
                            const double* const* pos_dev, double* const* forces_dev,
                            double* energies_dev, maze_stats* st);

/* Grid side N of a session (0 for NULL). */
int maze_grid_n(const maze_session* s);

/* Debug/inspection copy of one internal grid (N^3 doubles) into out_dev:
 * which = 0 phi^k, 1 phi^{k-1}, 2 y*, 3 q as assigned (the zero-mode
 * projection is applied where q is read, not stored), 4 sigma_p. */
int maze_get_grid(const maze_session* s, int which, double* out_dev);

/* Checkpoint of the warm-start state (phi^k, phi^{k-1}, y*, step count and
 * config) into a HOST buffer of maze_state_bytes() bytes. maze_load checks
 * the header (MAZE_E_INVALID on mismatch or a short buffer). */
size_t maze_state_bytes(const maze_session* s);
int maze_save(const maze_session* s, void* host_buf, size_t bytes);
int maze_load(maze_session* s, const void* host_buf, size_t bytes);

/* Sweep timing for measurement. When enabled, the runtime brackets every
 * sixteenth CG sweep of each solve (at most 512 per solve) with a pair of
 * HIP events on the session stream, and keeps the durations of the sampled
 * sweeps that did work. maze_profile_read copies 8 doubles into out8 (HOST
 * memory) and resets them:
 *   {FP64 sweeps timed, their total ms, FP32 sweeps timed, their total ms,
 *    FP64 CG iterations, FP32 CG iterations, 0, 0}
 * With MAZE_FLAG_SSTEP the timed unit is one outer step of two iterations
 * (basis and update kernel, with a third event between them), and the last
 * two entries hold the total ms of the update kernels of the timed FP64 and
 * FP32 outer steps. Enabling creates the events (the only allocation
 * outside maze_init). Sampling adds event records to the stream: about 0.5%
 * of a 256^3 step. */
int maze_profile_enable(maze_session* s, int on);
int maze_profile_read(maze_session* s, double* out8);

/* Launch shapes of the session's CG sweep. The latency shape, used alone
 * and in batches below the fill level, is picked at maze_init by timing the
 * candidate shapes on the session's own buffers (cached per device, grid
 * size and precision; MAZE_AUTOTUNE=0 in the environment selects fixed
 * defaults). The throughput shape, used in batches that fill the device, is
 * the one with the longest runs and segments that fits (16 x planes, 1024
 * points). MAZE_SWEEP_SHAPE="ppt:cx" forces both. With MAZE_FLAG_SSTEP the
 * latency shape is that of the update kernel: the sweep shape or a
 * 512-thread shape, whichever runs the outer step faster with the basis
 * kernel's shape (see maze_basis_shape; MAZE_UPDATE_SHAPE="threads:ppt:cx"
 * forces one, and a forced MAZE_SWEEP_SHAPE or MAZE_AUTOTUNE=0 keeps the
 * sweep shape).
 * out8 (HOST, 8 int32): {points per thread, x planes per workgroup,
 * workgroups, segment length} of the latency shape, then of the throughput
 * shape; threads per workgroup = segment length / points per thread. */
int maze_launch_shape(const maze_session* s, int32_t* out8);

/* Launch shape of the basis kernel of the two-iteration CG
 * (MAZE_FLAG_SSTEP): picked at maze_init together with the update kernel's
 * shape (each kernel's best shape depends on the other's) by timing whole
 * outer steps of the session's latency shape and of 512- and 1024-thread
 * shapes (longer segments, less halo work) on the session's own buffers;
 * the pair is cached per device, grid size and precision.
 * MAZE_BASIS_SHAPE="threads:ppt:cx" forces one, MAZE_AUTOTUNE=0 keeps the
 * latency shape. Without the flag it is the latency shape. out4 (HOST,
 * 4 int32): {threads per workgroup, points per thread, x planes per
 * workgroup, workgroups}. */
int maze_basis_shape(const maze_session* s, int32_t* out4);

/* Layout of the two-iteration CG's kernels (MAZE_FLAG_SSTEP). Where N is 64,
 * 128 or 256 the shape tuner also times a wavefront-row layout of the basis
 * kernel: each wavefront holds whole z rows (N / 64 consecutive points per
 * lane), takes its z neighbours from its own lanes and its y neighbours
 * from LDS, and a workgroup of W wavefronts covers W - 2 rows of the
 * plane (the stencil of Appendix B's matrix-vector product, unchanged);
 * W = 8, and at N = 256 in mixed precision also W = 16.
 * out2 (HOST, 2 int32):
 * {wavefronts per workgroup of the basis kernel, of the update kernel}, 0
 * for the segment layout (the update kernel has no wavefront-row form, so
 * its entry is 0). In the wavefront-row layout maze_basis_shape's points
 * per thread is N / 64. MAZE_BASIS_SHAPE="zv:W:cx" (cx planes per x run)
 * forces one. */
int maze_sstep_layout(const maze_session* s, int32_t* out2);

/* Residual trace of the last solve (for convergence studies such as the
 * residual-versus-iteration comparison of Appendix B). When enabled, each
 * solve records, per CG iteration k, the norm of the recursive residual
 * ||r_k||_2 divided by the right-hand-side scale (||q - qbar||_2 for a MaZe
 * step, ||4 pi q / h||_2 for a direct solve), as rows of three doubles
 * {pass, k, ||r_k|| / scale}; pass counts the FP32 inner solves of the
 * mixed-precision refinement (0 in FP64). Mixed precision also records the
 * FP64 true residual before each pass as {pass, -1, residual / scale}.
 * Recording copies the history to the host after every solve (a stream
 * synchronisation), so it is for studies, not for timing. Enabling clears
 * the trace; every solve replaces it.
 * maze_trace_read copies min(max_rows, n) rows into out (HOST memory, 3 *
 * max_rows doubles) and stores the number of rows n in *n_rows. */
int maze_trace_enable(maze_session* s, int on);
int maze_trace_read(const maze_session* s, double* out, int max_rows, int* n_rows);

/* Frees every device buffer of the session (NULL is a no-op). */
void maze_destroy(maze_session* s);

/* ---- molecular-dynamics driver around the step (not part of the
 * electrostatic path; Section 2 uses velocity Verlet for the ions, the
 * Results section a Born-Huggins-Mayer short-range term). ---- */
typedef struct {
  int32_t n_ions;
  int32_t pad;
  double* pos_dev;            /* n*3, updated in place (unwrapped) */
  double* vel_dev;            /* n*3 [A/fs], updated in place */
  const double* mass_dev;     /* n [amu] */
  const int32_t* species_dev; /* n, 0 or 1; pair row = s_i + s_j */
  double* f_es_dev;           /* n*3 electrostatic force [eV/A] */
  double* f_sr_dev;           /* n*3 short-range force [eV/A] */
  double* scratch_dev;        /* 6*n + 8*ceil(n/256) doubles of scratch */
  double* scalars_dev;        /* 8 doubles: [0] work energy of the
                                 electrostatic force (trapezoid rule),
                                 [1] short-range energy, [2] kinetic
                                 energy, [3..5] total momentum,
                                 [6] electrostatic energy, [7] unused */
  double dt;                  /* fs */
  double accel;               /* (eV/(A amu)) -> A/fs^2 */
  double cutoff;              /* short-range cutoff [A], <= box/2 */
  double bmh_table[15];       /* 3 rows (Na-Na, Na-Cl, Cl-Cl) of
                                 A [eV], B [1/A], s [A], C [eV A^6],
                                 D [eV A^8]: V = A e^{B(s-r)} - C/r^6 - D/r^8,
                                 shifted to zero at the cutoff */
  /* Langevin dynamics (Results section: canonical equilibration with the
   * OVRVO integrator). gamma: friction [1/fs], >= 0; 0 selects plain
   * velocity Verlet and kT, seed are not read. kT: thermostat temperature
   * k_B T [eV], >= 0. seed: key of the noise (maze_langevin_noise). */
  double gamma;
  double kT;
  uint64_t seed;
} maze_md_state;

/* Forces at the current positions: runs maze_step on pos (advancing the
 * MaZe history by one step at fixed positions) and the short-range term,
 * zeroes the work accumulator and fills the scalars. */
int maze_md_prime(maze_session* s, const maze_md_state* md, maze_stats* st);

/* One MD step. With gamma = 0, velocity Verlet: half kick, drift, maze_step
 * + short range at the new positions, work update, half kick, kinetic
 * energy and momentum. With gamma > 0, OVRVO: the same step between two
 * Ornstein-Uhlenbeck half steps v <- a v + sqrt((1 - a^2) kT accel / m) xi,
 * a = exp(-gamma dt / 2), one before the first half kick (half 0) and one
 * after the closing half kick (half 1), with xi the deviates
 * maze_langevin_noise gives for (seed, step, half) and step the session's
 * step count at entry (the count maze_step advances and maze_save keeps);
 * kinetic energy and momentum are then taken after the second half step.
 */
int maze_md_step(maze_session* s, const maze_md_state* md, maze_stats* st);

/* One velocity-Verlet step of `count` distinct sessions together: the
 * half kick and drift of each, their MaZe steps batched as in
 * maze_step_batch, then the short range and the closing half kick of each.
 * mds[i] belongs to sessions[i]; all sessions share a device and stream.
 * st (count entries, host, nullable) receives per-session stats and status.
 * Note: a session whose MaZe step is rejected has still been kicked and
 * drifted; its caller owns the recovery of the particle state. Returns the
 * most severe status. */
int maze_md_step_batch(maze_session* const* sessions, const maze_md_state* const* mds,
                       int32_t count, maze_stats* st);

/* Standard normal deviates of the Langevin noise. out_dev (DEVICE, n*3
 * doubles) receives, for ions i = 0..n-1, the deviates that OVRVO half step
 * `half` (0 or 1) of step `step` draws with key `seed`: Philox4x32-10
 * (Salmon, Moraes, Dror and Shaw, SC'11) of counter (i, half, step mod 2^32,
 * step div 2^32) and key (seed mod 2^32, seed div 2^32) gives words x0..x3;
 * the Box-Muller transform with u1 = (x + 1) 2^-32 and u2 = x' 2^-32 turns
 * (x0, x1) into the x and y deviates (r cos 2 pi u2, r sin 2 pi u2,
 * r = sqrt(-2 ln u1)) and (x2, x3) into z (r cos). Asynchronous on
 * `stream` (hipStream_t; NULL: the null stream). MAZE_E_INVALID for n < 0,
 * half not 0 or 1, step < 0 or a NULL out_dev with n > 0. */
int maze_langevin_noise(uint64_t seed, int64_t step, int32_t half, int32_t n, double* out_dev,
                        void* stream);

/* ---- structural and transport observables (Results section: radial pair
 * distribution functions, velocity autocorrelation functions and mean
 * squared displacements of molten NaCl). ---- */

/* Pair-distance histograms for g_IJ(r). For every pair i < j of the n ions
 * (pos_dev, DEVICE n*3 doubles, any periodic image), dx = x_j - x_i is
 * wrapped to dx - box rint(dx / box) per axis and r2 = dx^2 + dy^2 + dz^2
 * is summed in that order without fused multiply-add; the pair adds one to
 * hist_dev[row * nbins + b], row = s_i + s_j (species_dev, DEVICE n int32:
 * 0 Na, any other value Cl; rows Na-Na, Na-Cl, Cl-Cl), where edges2_dev[b] <= r2 <
 * edges2_dev[b + 1] (DEVICE, nbins + 1 ascending squared bin edges). Pairs
 * outside the edges are not counted. hist_dev (DEVICE, 3 * nbins uint64) is
 * accumulated, not cleared. 1 <= nbins <= 4096 and box > 0, else
 * MAZE_E_INVALID. Asynchronous on `stream`. */
int maze_rdf_accumulate(const double* pos_dev, const int32_t* species_dev, int32_t n, double box,
                        const double* edges2_dev, int32_t nbins, uint64_t* hist_dev,
                        void* stream);

/* Time correlations per species over time origins. Samples are numbered
 * k = 0, 1, ... in call order; sample k stores a copy of (positions,
 * velocities) as a time origin when k is a multiple of origin_every, and
 * every stored origin with lag l = k - k_o <= max_lag adds
 * sum_i v_i(k_o).v_i(k) and sum_i |r_i(k) - r_i(k_o)|^2 over the ions of
 * each species (positions unwrapped, as the MD driver keeps them) to the
 * sums of lag l, and one to counts[l]. Each (origin, sample) pair is one
 * workgroup's fixed-order reduction, so the sums are reproducible.
 * maze_tcf_create allocates max_lag / origin_every + 1 origin slots of n
 * ions and the sums on the current device and copies species_dev (DEVICE, n
 * int32, 0 or 1); sample and read run on `stream`. */
typedef struct maze_tcf maze_tcf;
int maze_tcf_create(int32_t n, const int32_t* species_dev, int32_t max_lag, int32_t origin_every,
                    void* stream, maze_tcf** out);
/* pos_dev, vel_dev: DEVICE n*3 doubles. Asynchronous. */
int maze_tcf_sample(maze_tcf* t, const double* pos_dev, const double* vel_dev);
/* sums_host (HOST, 4 * (max_lag + 1) doubles: rows VACF Na, VACF Cl, MSD
 * Na, MSD Cl, not normalised) and counts_host (HOST, max_lag + 1 int64,
 * origins seen at each lag); either may be NULL. Synchronises the stream. */
int maze_tcf_read(const maze_tcf* t, double* sums_host, int64_t* counts_host);
void maze_tcf_destroy(maze_tcf* t);

/* ---- continuous batches ------------------------------------------------
 * Steps of many sessions in flight together, for serving: a step joins the
 * batched CG launches already running as soon as it is added, and leaves
 * them when its solve ends, so a short step does not wait for a long one and
 * a step that arrives while others are on the device overlaps with them.
 * Per session the kernels, launch shapes and stopping decisions are those of
 * maze_step / maze_md_step alone (each session keeps its own latency
 * shapes), so every result is bitwise the one the session gets stepped
 * alone. Not for multigrid sessions. All sessions of a batch share its
 * device and stream. */
typedef struct maze_batch maze_batch;

/* Creates a batch on the current device for at most max_sessions (1..4096)
 * steps in flight, its work queued on `stream` (hipStream_t; the sessions'
 * cfg.stream must be the same). Allocates the batch's launch tables and
 * poll buffers (device and pinned host memory), freed by
 * maze_batch_destroy. */
int maze_batch_create(void* stream, int32_t max_sessions, maze_batch** out);

/* Adds one step of session s (at most one step of a session in flight).
 * With md non-NULL it is a full MD step as maze_md_step (kick and drift
 * are queued now, the short range and the closing kick when the solve
 * ends; *md is copied, and the buffers it names must stay valid until the
 * step is taken); else a MaZe step at positions pos_dev (device, n*3 doubles) whose
 * forces (forces_dev, n*3) and energy (energy_dev, 1 double) are written
 * when it finishes (either may be NULL). The step's assignment, right-hand
 * side and first CG unit are queued at once. tag is returned with the
 * result. MAZE_E_CAPACITY when the batch is full; MAZE_E_INVALID for a
 * session already in flight, on another device or stream, or multigrid. */
int maze_batch_add(maze_batch* b, maze_session* s, const maze_md_state* md,
                   const double* pos_dev, double* forces_dev, double* energy_dev, uint64_t tag);

/* Queues one poll group of CG units (about 100 us of device work) in which
 * one launch per kernel class covers every running solve, then acts on the
 * status of the group before: solves that ended leave the launches and
 * queue their finishing kernels (or, in mixed precision, their FP64
 * refinement, after which another FP32 pass may join); steps whose
 * finishing kernels have completed become ready. *n_ready (nullable)
 * receives the number of ready steps. Call it repeatedly while steps are in
 * flight; it blocks only on the status copy of the group before. */
int maze_batch_advance(maze_batch* b, int32_t* n_ready);

/* Removes up to max ready steps, oldest first: tags[i] (HOST, max entries)
 * and st[i] (HOST, max entries, nullable; st[i].status holds the step's
 * status, MAZE_E_NONFINITE for rejected positions, which leave the MaZe
 * state unchanged). *n (nullable) receives the number removed. */
int maze_batch_take(maze_batch* b, int32_t max, uint64_t* tags, maze_stats* st, int32_t* n);

/* Steps added and not yet taken out of flight (ready steps excluded). */
int maze_batch_in_flight(const maze_batch* b);

/* Finishes the steps in flight, then frees the batch (NULL is a no-op). */
void maze_batch_destroy(maze_batch* b);

/* ---- measurement ---------------------------------------------------------
 * Streaming copy of `bytes` (a multiple of 16) from src_dev to dst_dev
 * (DEVICE buffers that do not overlap), queued on `stream`: 16-byte vector
 * loads and stores, the buffer cut into contiguous chunks, one per
 * workgroup (16384 workgroups). On
 * footprints far beyond the caches its rate (2 * bytes / time) is the
 * practical HBM ceiling for kernels that read and write every byte once,
 * against which the solver kernels are compared. MAZE_E_INVALID for NULL
 * pointers, pointers not 16-byte aligned or a size that is not a multiple of
 * 16. */
int maze_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MAZE_H */
