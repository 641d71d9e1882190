/*
 * Plain FP64 CPU oracle of the Poisson MaZe per-timestep path.
 *
 * TEST INFRASTRUCTURE ONLY: it exists so that the device implementation can
 * be checked against something slow and obviously correct. Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the HIP implementation.
 *
 * Built with -O2 -ffp-contract=off: every floating-point operation below is
 * rounded on its own, in the order written, with no blocking or fusion.
 *
 * Paper: Troni, Grassano, Narayan, Roux, Bonella, "Mass-Zero constrained
 * molecular dynamics for electrostatic interactions" (arXiv 2505.20418).
 * Each function names the passage it follows.
 */
#include "maze_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Timing build only: loops whose iterations are independent (each writes
 * its own element and reads nothing another iteration writes) run across
 * threads when compiled with -fopenmp. Every reduction (dot products, norms,
 * sums, the charge scatter, the pair forces) stays a plain sequential loop,
 * so the threaded build returns bitwise the results of the plain one. */
#ifdef _OPENMP
#define ORACLE_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define ORACLE_PARALLEL_FOR
#endif

static long long flat(int N, int i, int j, int k) {
  return ((long long)i * N + j) * N + k;
}

static int wrap_index(long long i, int N) {
  long long m = i % N;
  if (m < 0) m += N;
  return (int)m;
}

static long long grid_points(int N) { return (long long)N * N * N; }

/* Section 2, discretisation paragraph (equation "linearproblem"): N points
 * per side; the requested spacing is rounded to a whole number of points
 * and the effective spacing is box / N. */
int oracle_grid_n(double box, double grid_spacing) {
  if (!(box > 0.0) || !(grid_spacing > 0.0)) return 0;
  return (int)lround(box / grid_spacing);
}

/* Centred cubic B-spline, the weight function named in the force paragraph
 * after equation "F_nostra" (Section 2.1). */
static double bspline3(double s) {
  double a = fabs(s);
  if (a < 1.0) return 2.0 / 3.0 - a * a + a * a * a / 2.0;
  if (a < 2.0) {
    double t = 2.0 - a;
    return t * t * t / 6.0;
  }
  return 0.0;
}

static double bspline3_deriv(double s) {
  double a = fabs(s);
  double sg = (s < 0.0) ? -1.0 : 1.0;
  if (a < 1.0) return -2.0 * s + 1.5 * s * a;
  if (a < 2.0) {
    double t = 2.0 - a;
    return -sg * t * t / 2.0;
  }
  return 0.0;
}

/* Wrap a coordinate into [0, box) and express it in grid units. */
static double grid_coordinate(double coord, double box, int N) {
  double h = box / N;
  double xw = coord - box * floor(coord / box);
  return xw / h;
}

/* Charge-assignment weights along one axis (Section 2.1, text after equation
 * "F_nostra": q_n = Q W(r - r_n)). order 2 uses the two nearest grid points
 * (the 8-point stencil the force sum runs over); order 4 uses the centred
 * cubic B-spline on four points. */
void oracle_axis_weights(int order, double coord, double box, int N,
                         int32_t* idx, double* w) {
  double u = grid_coordinate(coord, box, N);
  double fl = floor(u);
  double t = u - fl;
  long long i0 = (long long)fl;
  if (order == 2) {
    idx[0] = wrap_index(i0, N);
    idx[1] = wrap_index(i0 + 1, N);
    w[0] = 1.0 - t;
    w[1] = t;
  } else {
    idx[0] = wrap_index(i0 - 1, N);
    idx[1] = wrap_index(i0, N);
    idx[2] = wrap_index(i0 + 1, N);
    idx[3] = wrap_index(i0 + 2, N);
    w[0] = bspline3(1.0 + t);
    w[1] = bspline3(t);
    w[2] = bspline3(1.0 - t);
    w[3] = bspline3(2.0 - t);
  }
}

/* Derivative of the 1-D weights with respect to the coordinate (used only
 * by the alternative force of equation "F_Benoit"). */
static void axis_weight_derivs(int order, double coord, double box, int N,
                               double* dw) {
  double h = box / N;
  double u = grid_coordinate(coord, box, N);
  double t = u - floor(u);
  if (order == 2) {
    dw[0] = -1.0 / h;
    dw[1] = 1.0 / h;
  } else {
    /* weight of point i0 + m is B(u - i0 - m) = B(t - m) */
    dw[0] = bspline3_deriv(t + 1.0) / h;
    dw[1] = bspline3_deriv(t) / h;
    dw[2] = bspline3_deriv(t - 1.0) / h;
    dw[3] = bspline3_deriv(t - 2.0) / h;
  }
}

/* Charge assignment q_n = sum_alpha Q_alpha W(r_alpha - r_n), Section 2.1,
 * accumulated in ion order. */
void oracle_spread_raw(int n, const double* pos, const double* Q, double box,
                       int N, int order, double* q) {
  long long G = grid_points(N);
  memset(q, 0, sizeof(double) * (size_t)G);
  for (int a = 0; a < n; ++a) {
    int32_t ix[4], iy[4], iz[4];
    double wx[4], wy[4], wz[4];
    oracle_axis_weights(order, pos[3 * a + 0], box, N, ix, wx);
    oracle_axis_weights(order, pos[3 * a + 1], box, N, iy, wy);
    oracle_axis_weights(order, pos[3 * a + 2], box, N, iz, wz);
    for (int i = 0; i < order; ++i)
      for (int j = 0; j < order; ++j)
        for (int k = 0; k < order; ++k) {
          double c = Q[a] * wx[i];
          c = c * wy[j];
          c = c * wz[k];
          q[flat(N, ix[i], iy[j], iz[k])] += c;
        }
  }
}

/* Removal of the zero mode: the periodic M is singular on constants, so the
 * charge is made neutral on the grid (a uniform compensating background, as
 * the paper does for the single-charge measurement in Appendix A) and the
 * potential is fixed to mean zero. */
double oracle_project_mean(int N, double* x) {
  long long G = grid_points(N);
  double s = 0.0;
  for (long long n = 0; n < G; ++n) s += x[n];
  double mean = s / (double)G;
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) x[n] -= mean;
  return mean;
}

/* The matrix M of the footnote to equation "linearproblem": -6 on the
 * diagonal and +1 for each of the six axis neighbours, periodic. */
void oracle_apply_M(int N, const double* x, double* out) {
  ORACLE_PARALLEL_FOR
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int k = 0; k < N; ++k) {
        double s = x[flat(N, wrap_index(i + 1, N), j, k)];
        s += x[flat(N, wrap_index(i - 1, N), j, k)];
        s += x[flat(N, i, wrap_index(j + 1, N), k)];
        s += x[flat(N, i, wrap_index(j - 1, N), k)];
        s += x[flat(N, i, j, wrap_index(k + 1, N))];
        s += x[flat(N, i, j, wrap_index(k - 1, N))];
        out[flat(N, i, j, k)] = s - 6.0 * x[flat(N, i, j, k)];
      }
}

static double dot(long long G, const double* a, const double* b) {
  double s = 0.0;
  for (long long n = 0; n < G; ++n) s += a[n] * b[n];
  return s;
}

static double max_abs(long long G, const double* a) {
  double m = 0.0;
  for (long long n = 0; n < G; ++n) {
    double v = fabs(a[n]);
    if (v > m) m = v;
  }
  return m;
}

static int met(double rr, const double* r, long long G, double thr, int norm) {
  if (norm == ORACLE_NORM_ABSMAX) return max_abs(G, r) <= thr;
  return sqrt(rr) <= thr;
}

/* Preconditioned linear conjugate gradient (Appendix B) for A x = b with
 * A = -M, which is symmetric positive definite on mean-zero vectors, and
 * the Jacobi preconditioner built from the diagonal of the matrix (6 I).
 * Hestenes-Stiefel recurrences, written out step by step. */
int oracle_pcg(int N, const double* b, double* x, double thr, int norm,
               int max_iter, int* iters) {
  long long G = grid_points(N);
  double* r = (double*)malloc(sizeof(double) * (size_t)G);
  double* z = (double*)malloc(sizeof(double) * (size_t)G);
  double* p = (double*)malloc(sizeof(double) * (size_t)G);
  double* w = (double*)malloc(sizeof(double) * (size_t)G);
  /* r = b - A x = b + M x */
  oracle_apply_M(N, x, w);
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) r[n] = b[n] + w[n];
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) z[n] = r[n] / 6.0;
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) p[n] = z[n];
  double rho = dot(G, r, z);
  double rr = dot(G, r, r);
  int k = 0;
  int ok = met(rr, r, G, thr, norm);
  while (!ok && k < max_iter) {
    /* w = A p = -M p */
    oracle_apply_M(N, p, w);
    ORACLE_PARALLEL_FOR
    for (long long n = 0; n < G; ++n) w[n] = -w[n];
    double pw = dot(G, p, w);
    if (!(pw > 0.0) || !isfinite(pw)) break;  /* breakdown */
    double alpha = rho / pw;
    ORACLE_PARALLEL_FOR
    for (long long n = 0; n < G; ++n) x[n] += alpha * p[n];
    ORACLE_PARALLEL_FOR
    for (long long n = 0; n < G; ++n) r[n] -= alpha * w[n];
    k += 1;
    rr = dot(G, r, r);
    ok = met(rr, r, G, thr, norm);
    if (ok) break;
    ORACLE_PARALLEL_FOR
    for (long long n = 0; n < G; ++n) z[n] = r[n] / 6.0;
    double rho_new = dot(G, r, z);
    double beta = rho_new / rho;
    ORACLE_PARALLEL_FOR
    for (long long n = 0; n < G; ++n) p[n] = z[n] + beta * p[n];
    rho = rho_new;
  }
  free(r); free(z); free(p); free(w);
  if (iters) *iters = k;
  return ok;
}

/* Equation "F_nostra" with the central differences of the equation before
 * it: F_alpha = -k Q_alpha sum_n W(r_alpha - r_n) (D phi)_n, over the same
 * grid points and weights used to spread the charge. */
void oracle_gather(int n, const double* pos, const double* Q, double box,
                   int N, int order, const double* phi, double coulomb_k,
                   double* F) {
  double h = box / N;
  for (int a = 0; a < n; ++a) {
    int32_t ix[4], iy[4], iz[4];
    double wx[4], wy[4], wz[4];
    oracle_axis_weights(order, pos[3 * a + 0], box, N, ix, wx);
    oracle_axis_weights(order, pos[3 * a + 1], box, N, iy, wy);
    oracle_axis_weights(order, pos[3 * a + 2], box, N, iz, wz);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < order; ++i)
      for (int j = 0; j < order; ++j)
        for (int k = 0; k < order; ++k) {
          int I = ix[i], J = iy[j], K = iz[k];
          double W = wx[i] * wy[j];
          W = W * wz[k];
          double dx = (phi[flat(N, wrap_index(I + 1, N), J, K)] -
                       phi[flat(N, wrap_index(I - 1, N), J, K)]) / (2.0 * h);
          double dy = (phi[flat(N, I, wrap_index(J + 1, N), K)] -
                       phi[flat(N, I, wrap_index(J - 1, N), K)]) / (2.0 * h);
          double dz = (phi[flat(N, I, J, wrap_index(K + 1, N))] -
                       phi[flat(N, I, J, wrap_index(K - 1, N))]) / (2.0 * h);
          acc[0] += W * dx;
          acc[1] += W * dy;
          acc[2] += W * dz;
        }
    for (int d = 0; d < 3; ++d) F[3 * a + d] = -coulomb_k * Q[a] * acc[d];
  }
}

/* Equation "F_Benoit": -k Q_alpha sum_n grad W(r_alpha - r_n) phi_n. */
void oracle_gather_weight_gradient(int n, const double* pos, const double* Q,
                                   double box, int N, int order,
                                   const double* phi, double coulomb_k,
                                   double* F) {
  for (int a = 0; a < n; ++a) {
    int32_t ix[4], iy[4], iz[4];
    double wx[4], wy[4], wz[4], dx[4], dy[4], dz[4];
    oracle_axis_weights(order, pos[3 * a + 0], box, N, ix, wx);
    oracle_axis_weights(order, pos[3 * a + 1], box, N, iy, wy);
    oracle_axis_weights(order, pos[3 * a + 2], box, N, iz, wz);
    axis_weight_derivs(order, pos[3 * a + 0], box, N, dx);
    axis_weight_derivs(order, pos[3 * a + 1], box, N, dy);
    axis_weight_derivs(order, pos[3 * a + 2], box, N, dz);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < order; ++i)
      for (int j = 0; j < order; ++j)
        for (int k = 0; k < order; ++k) {
          double v = phi[flat(N, ix[i], iy[j], iz[k])];
          acc[0] += dx[i] * wy[j] * wz[k] * v;
          acc[1] += wx[i] * dy[j] * wz[k] * v;
          acc[2] += wx[i] * wy[j] * dz[k] * v;
        }
    for (int d = 0; d < 3; ++d) F[3 * a + d] = -coulomb_k * Q[a] * acc[d];
  }
}

/* Equation "energy_discr": V_c = (1/2) phi . q. */
double oracle_energy(int N, const double* phi, const double* q,
                     double coulomb_k) {
  return 0.5 * coulomb_k * dot(grid_points(N), phi, q);
}

/* ------------------------------------------------------------------ */
/* Session: the MaZe time step of Section 2 (equations "SHAKE" to       */
/* "SHAKEPhiFinal").                                                    */
/* ------------------------------------------------------------------ */
struct oracle_session {
  oracle_config cfg;
  int N;
  double h;
  double* Q;
  double* phi_k;
  double* phi_km1;
  double* y;
  double* q;
  double* sigma;
  double* work;
  long long step;
};

static void true_residual(int N, const double* b, const double* x,
                          double* scratch, double* l2, double* amax) {
  /* r = b - A x = b + M x */
  long long G = grid_points(N);
  oracle_apply_M(N, x, scratch);
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) scratch[n] = b[n] + scratch[n];
  *l2 = sqrt(dot(G, scratch, scratch));
  *amax = max_abs(G, scratch);
}

static double l2norm(long long G, const double* a) { return sqrt(dot(G, a, a)); }

static int check_positions(int n, const double* pos) {
  for (int i = 0; i < 3 * n; ++i)
    if (!isfinite(pos[i])) return 0;
  return 1;
}

static void fill_stats(oracle_stats* st, const oracle_session* s, int iters,
                       int converged, double rel, double amax, double net,
                       double energy) {
  if (!st) return;
  st->grid_n = s->N;
  st->iters = iters;
  st->converged = converged;
  st->pad = 0;
  st->h = s->h;
  st->rel_residual = rel;
  st->max_abs_residual = amax;
  st->net_charge = net;
  st->energy = energy;
}

/* Spread, record the net charge, then project (neutral grid charge). */
static double spread_projected(oracle_session* s, const double* pos) {
  oracle_spread_raw(s->cfg.n_ions, pos, s->Q, s->cfg.box, s->N, s->cfg.order,
                    s->q);
  long long G = grid_points(s->N);
  double net = 0.0;
  for (long long n = 0; n < G; ++n) net += s->q[n];
  oracle_project_mean(s->N, s->q);
  return net;
}

/* Direct Poisson solve (-M) phi = 4 pi q / h from a given start; the
 * stopping threshold is tol * ||4 pi q / h||_2 (or tol in max-norm). */
static int poisson_solve(oracle_session* s, double* phi, int* iters,
                         double* rel, double* amax) {
  long long G = grid_points(s->N);
  double* b = s->sigma;  /* reuse as the right-hand side */
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) b[n] = 4.0 * M_PI * s->q[n] / s->h;
  double bn = l2norm(G, b);
  double thr = (s->cfg.residual_norm == ORACLE_NORM_ABSMAX) ? s->cfg.tol
                                                             : s->cfg.tol * bn;
  int ok = oracle_pcg(s->N, b, phi, thr, s->cfg.residual_norm,
                      s->cfg.max_iter, iters);
  oracle_project_mean(s->N, phi);
  double l2;
  true_residual(s->N, b, phi, s->work, &l2, amax);
  *rel = (bn > 0.0) ? l2 / bn : l2;
  return ok;
}

int oracle_init(const oracle_config* cfg, const double* charges,
                const double* pos0, oracle_session** out,
                oracle_stats* st) {
  if (!cfg || !charges || !pos0 || !out) return ORACLE_E_INVALID;
  *out = NULL;
  int N = oracle_grid_n(cfg->box, cfg->grid_spacing);
  if (cfg->n_ions <= 0 || N < 4 || N > 1024 ||
      (cfg->order != 2 && cfg->order != 4) || !(cfg->tol > 0.0) ||
      cfg->max_iter < 0)
    return ORACLE_E_INVALID;
  double qs = 0.0, qa = 0.0;
  for (int i = 0; i < cfg->n_ions; ++i) {
    qs += charges[i];
    qa += fabs(charges[i]);
  }
  if (fabs(qs) > 1e-10 * qa) return ORACLE_E_NOT_NEUTRAL;
  if (!check_positions(cfg->n_ions, pos0)) return ORACLE_E_INVALID;

  oracle_session* s = (oracle_session*)calloc(1, sizeof(oracle_session));
  s->cfg = *cfg;
  s->N = N;
  s->h = cfg->box / N;
  long long G = grid_points(N);
  s->Q = (double*)malloc(sizeof(double) * (size_t)cfg->n_ions);
  memcpy(s->Q, charges, sizeof(double) * (size_t)cfg->n_ions);
  s->phi_k = (double*)calloc((size_t)G, sizeof(double));
  s->phi_km1 = (double*)calloc((size_t)G, sizeof(double));
  s->y = (double*)calloc((size_t)G, sizeof(double));
  s->q = (double*)calloc((size_t)G, sizeof(double));
  s->sigma = (double*)calloc((size_t)G, sizeof(double));
  s->work = (double*)calloc((size_t)G, sizeof(double));

  /* Initial state (the pseudocode figure is not available): a cold Poisson
   * solve for phi^0 from zero, phi^{-1} = phi^0 and y = 0. */
  double net = spread_projected(s, pos0);
  int iters = 0;
  double rel, amax;
  int ok = poisson_solve(s, s->phi_k, &iters, &rel, &amax);
  memcpy(s->phi_km1, s->phi_k, sizeof(double) * (size_t)G);
  double e = oracle_energy(N, s->phi_k, s->q, cfg->coulomb_k);
  fill_stats(st, s, iters, ok, rel, amax, net, e);
  *out = s;
  return ok ? ORACLE_OK : ORACLE_NOT_CONVERGED;
}

/* One MaZe step (Section 2, from the Verlet update of phi to equation
 * "SHAKEPhiFinal"):
 *   q^{k+1}   = charge of the new positions
 *   phi_p     = 2 phi^k - phi^{k-1}
 *   sigma_p   = (h / 4 pi) M phi_p + q^{k+1}
 *   M y       = sigma_p, solved by PLCG from the previous y (the SHAKE
 *               warm start), threshold tol * ||q^{k+1}||_2
 *   phi^{k+1} = phi_p - (4 pi / h) y */
int oracle_step(oracle_session* s, const double* pos, double* field,
                double* forces, double* energy, oracle_stats* st) {
  if (!s || !pos) return ORACLE_E_INVALID;
  if (!check_positions(s->cfg.n_ions, pos)) return ORACLE_E_INVALID;
  int N = s->N;
  long long G = grid_points(N);
  double h = s->h;
  double net = spread_projected(s, pos);

  double* phi_p = s->work;
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) phi_p[n] = 2.0 * s->phi_k[n] - s->phi_km1[n];
  oracle_apply_M(N, phi_p, s->sigma);
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n)
    s->sigma[n] = (h / (4.0 * M_PI)) * s->sigma[n] + s->q[n];

  /* (-M) y = -sigma_p */
  double* b = (double*)malloc(sizeof(double) * (size_t)G);
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) b[n] = -s->sigma[n];
  double qn = l2norm(G, s->q);
  double thr = (s->cfg.residual_norm == ORACLE_NORM_ABSMAX) ? s->cfg.tol
                                                             : s->cfg.tol * qn;
  int iters = 0;
  int ok = oracle_pcg(N, b, s->y, thr, s->cfg.residual_norm, s->cfg.max_iter,
                      &iters);
  oracle_project_mean(N, s->y);

  /* true residual M y - sigma_p */
  double* r = (double*)malloc(sizeof(double) * (size_t)G);
  oracle_apply_M(N, s->y, r);
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n) r[n] = r[n] - s->sigma[n];
  double l2 = l2norm(G, r);
  double amax = max_abs(G, r);
  free(r);
  free(b);

  /* phi^{k+1} = phi_p - (4 pi / h) y, stored over phi^{k-1} */
  ORACLE_PARALLEL_FOR
  for (long long n = 0; n < G; ++n)
    s->phi_km1[n] = phi_p[n] - (4.0 * M_PI / h) * s->y[n];
  oracle_project_mean(N, s->phi_km1);
  double* t = s->phi_k;
  s->phi_k = s->phi_km1;
  s->phi_km1 = t;
  s->step += 1;

  double e = oracle_energy(N, s->phi_k, s->q, s->cfg.coulomb_k);
  if (field) memcpy(field, s->phi_k, sizeof(double) * (size_t)G);
  if (forces)
    oracle_gather(s->cfg.n_ions, pos, s->Q, s->cfg.box, N, s->cfg.order,
                  s->phi_k, s->cfg.coulomb_k, forces);
  if (energy) *energy = e;
  fill_stats(st, s, iters, ok, (qn > 0.0) ? l2 / qn : l2, amax, net, e);
  return ok ? ORACLE_OK : ORACLE_NOT_CONVERGED;
}

/* Direct solution of equation "linearproblem" from the guesses compared in
 * the convergence subsection: zero, "static" (phi^k) or "time-propagated"
 * (2 phi^k - phi^{k-1}). The MaZe history is left untouched. */
int oracle_solve(oracle_session* s, int guess, const double* pos,
                 double* field, double* forces, double* energy,
                 oracle_stats* st) {
  if (!s || !pos) return ORACLE_E_INVALID;
  if (guess < ORACLE_GUESS_ZERO || guess > ORACLE_GUESS_TIMEPROP)
    return ORACLE_E_INVALID;
  if (!check_positions(s->cfg.n_ions, pos)) return ORACLE_E_INVALID;
  int N = s->N;
  long long G = grid_points(N);
  /* the direct solve must not disturb the step state: use private copies */
  double* q_save = (double*)malloc(sizeof(double) * (size_t)G);
  double* sig_save = (double*)malloc(sizeof(double) * (size_t)G);
  memcpy(q_save, s->q, sizeof(double) * (size_t)G);
  memcpy(sig_save, s->sigma, sizeof(double) * (size_t)G);
  double* phi = (double*)malloc(sizeof(double) * (size_t)G);
  for (long long n = 0; n < G; ++n) {
    if (guess == ORACLE_GUESS_ZERO) phi[n] = 0.0;
    else if (guess == ORACLE_GUESS_STATIC) phi[n] = s->phi_k[n];
    else phi[n] = 2.0 * s->phi_k[n] - s->phi_km1[n];
  }
  double net = spread_projected(s, pos);
  int iters = 0;
  double rel, amax;
  int ok = poisson_solve(s, phi, &iters, &rel, &amax);
  double e = oracle_energy(N, phi, s->q, s->cfg.coulomb_k);
  if (field) memcpy(field, phi, sizeof(double) * (size_t)G);
  if (forces)
    oracle_gather(s->cfg.n_ions, pos, s->Q, s->cfg.box, N, s->cfg.order, phi,
                  s->cfg.coulomb_k, forces);
  if (energy) *energy = e;
  fill_stats(st, s, iters, ok, rel, amax, net, e);
  memcpy(s->q, q_save, sizeof(double) * (size_t)G);
  memcpy(s->sigma, sig_save, sizeof(double) * (size_t)G);
  free(q_save); free(sig_save); free(phi);
  return ok ? ORACLE_OK : ORACLE_NOT_CONVERGED;
}

void oracle_get_state(const oracle_session* s, double* phi_k, double* phi_km1,
                      double* y, double* q, double* sigma_p) {
  size_t bytes = sizeof(double) * (size_t)grid_points(s->N);
  if (phi_k) memcpy(phi_k, s->phi_k, bytes);
  if (phi_km1) memcpy(phi_km1, s->phi_km1, bytes);
  if (y) memcpy(y, s->y, bytes);
  if (q) memcpy(q, s->q, bytes);
  if (sigma_p) memcpy(sigma_p, s->sigma, bytes);
}

int oracle_grid_of(const oracle_session* s) { return s ? s->N : 0; }

void oracle_destroy(oracle_session* s) {
  if (!s) return;
  free(s->Q); free(s->phi_k); free(s->phi_km1); free(s->y); free(s->q);
  free(s->sigma); free(s->work);
  free(s);
}

/* ------------------------------------------------------------------ */
/* MD driver pieces: Born-Huggins-Mayer short range (Results section,  */
/* Tosi-Fumi form with the electrostatic term removed) and velocity    */
/* Verlet for the ions (Section 2).                                    */
/* ------------------------------------------------------------------ */
static double bmh_pair(const double* row, double r) {
  double A = row[0], B = row[1], s = row[2], C = row[3], D = row[4];
  double r2 = r * r;
  double r6 = r2 * r2 * r2;
  double r8 = r6 * r2;
  return A * exp(B * (s - r)) - C / r6 - D / r8;
}

static double bmh_pair_dvdr(const double* row, double r) {
  double A = row[0], B = row[1], s = row[2], C = row[3], D = row[4];
  double r2 = r * r;
  double r7 = r2 * r2 * r2 * r;
  double r9 = r7 * r2;
  return -A * B * exp(B * (s - r)) + 6.0 * C / r7 + 8.0 * D / r9;
}

void oracle_bmh(int n, const double* pos, const int32_t* species, double box,
                const double* table, double cutoff, double* F,
                double* energy) {
  double e = 0.0;
  for (int i = 0; i < 3 * n; ++i) F[i] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double d[3];
      for (int c = 0; c < 3; ++c) {
        double x = pos[3 * i + c] - pos[3 * j + c];
        d[c] = x - box * floor(x / box + 0.5);  /* minimum image */
      }
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (r >= cutoff) continue;
      const double* row = table + 5 * (species[i] + species[j]);
      e += bmh_pair(row, r) - bmh_pair(row, cutoff);
      double f = -bmh_pair_dvdr(row, r) / r;
      for (int c = 0; c < 3; ++c) {
        F[3 * i + c] += f * d[c];
        F[3 * j + c] -= f * d[c];
      }
    }
  if (energy) *energy = e;
}

int oracle_md_step(oracle_session* s, int n, double* pos, double* vel,
                   const double* masses, const int32_t* species,
                   const double* table, double cutoff, double dt,
                   double accel_factor, double* F_es, double* F_sr,
                   double* work, double* v_sr, double* energy_c,
                   oracle_stats* st) {
  double* old = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  double* fold = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < 3; ++c) {
      int i = 3 * a + c;
      vel[i] += 0.5 * dt * (F_es[i] + F_sr[i]) / masses[a] * accel_factor;
      old[i] = pos[i];
      fold[i] = F_es[i];
      pos[i] += dt * vel[i];
    }
  int rc = oracle_step(s, pos, NULL, F_es, energy_c, st);
  oracle_bmh(n, pos, species, s->cfg.box, table, cutoff, F_sr, v_sr);
  double dw = 0.0;
  for (int i = 0; i < 3 * n; ++i) dw += 0.5 * (fold[i] + F_es[i]) * (pos[i] - old[i]);
  *work -= dw;
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < 3; ++c) {
      int i = 3 * a + c;
      vel[i] += 0.5 * dt * (F_es[i] + F_sr[i]) / masses[a] * accel_factor;
    }
  free(old);
  free(fold);
  return rc;
}
