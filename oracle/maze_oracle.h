/*
 * Plain FP64 CPU oracle of the Poisson MaZe per-timestep path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this code: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no code with the HIP implementation.
 *
 * Conventions (all functions):
 *   - cubic periodic box of side `box`; N = lround(box / grid_spacing) grid
 *     points per side; effective spacing h = box / N;
 *   - grid point (i, j, k) sits at (i h, j h, k h) and is stored at flat
 *     index (i*N + j)*N + k (z fastest);
 *   - positions are (n, 3) row-major, x y z per ion;
 *   - Gaussian units inside (charges in e, lengths in A, potential in e/A);
 *     `coulomb_k` multiplies energies and forces (14.3996454784 gives eV and
 *     eV/A, 1.0 keeps e^2/A).
 */
#ifndef MAZE_ORACLE_H
#define MAZE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_OK = 0, ORACLE_NOT_CONVERGED = 1, ORACLE_E_INVALID = -1,
       ORACLE_E_NOT_NEUTRAL = -2 };
enum { ORACLE_GUESS_ZERO = 0, ORACLE_GUESS_STATIC = 1, ORACLE_GUESS_TIMEPROP = 2 };
enum { ORACLE_NORM_REL2 = 0, ORACLE_NORM_ABSMAX = 1 };

typedef struct {
  int32_t n_ions;
  int32_t order;          /* 2: linear (8 points), 4: cubic B-spline (64) */
  double  box;
  double  grid_spacing;
  double  tol;
  int32_t max_iter;
  int32_t residual_norm;  /* ORACLE_NORM_* */
  double  coulomb_k;
} oracle_config;

typedef struct {
  int32_t grid_n;
  int32_t iters;
  int32_t converged;
  int32_t pad;
  double  h;
  double  rel_residual;      /* ||true residual||_2 / ||rhs scale||_2 */
  double  max_abs_residual;  /* max |true residual| */
  double  net_charge;        /* sum of spread charge before projection */
  double  energy;            /* (1/2) k phi.q */
} oracle_stats;

typedef struct oracle_session oracle_session;

/* ---- building blocks ---- */
int    oracle_grid_n(double box, double grid_spacing);
/* 1-D assignment weights of one coordinate: writes `order` grid indices
 * (already taken mod N) and weights. */
void   oracle_axis_weights(int order, double coord, double box, int N,
                           int32_t* idx, double* w);
/* Spread without the mean projection. */
void   oracle_spread_raw(int n, const double* pos, const double* Q, double box,
                         int N, int order, double* q);
/* Subtract the mean of an N^3 vector; returns the mean removed. */
double oracle_project_mean(int N, double* x);
/* out = M x, the 7-point periodic stencil (diagonal -6, six +1). */
void   oracle_apply_M(int N, const double* x, double* out);
/* Jacobi-preconditioned CG for (-M) x = b, preconditioner diag(-M) = 6 I.
 * Stops when ||r||_2 <= thr (norm 0) or max|r| <= thr (norm 1), or after
 * max_iter iterations. Returns 1 if the stopping test was met. */
int    oracle_pcg(int N, const double* b, double* x, double thr, int norm,
                  int max_iter, int* iters);
/* Central-difference forces interpolated with the assignment weights. */
void   oracle_gather(int n, const double* pos, const double* Q, double box,
                     int N, int order, const double* phi, double coulomb_k,
                     double* F);
/* Im-style force: gradient of the assignment weights times phi. */
void   oracle_gather_weight_gradient(int n, const double* pos, const double* Q,
                     double box, int N, int order, const double* phi,
                     double coulomb_k, double* F);
double oracle_energy(int N, const double* phi, const double* q, double coulomb_k);

/* ---- session API (same shape as the device C ABI, on host pointers) ---- */
int  oracle_init(const oracle_config* cfg, const double* charges,
                 const double* pos0, oracle_session** out, oracle_stats* st);
int  oracle_step(oracle_session* s, const double* pos, double* field,
                 double* forces, double* energy, oracle_stats* st);
int  oracle_solve(oracle_session* s, int guess, const double* pos,
                  double* field, double* forces, double* energy,
                  oracle_stats* st);
/* Copies of the internal state (any pointer may be NULL). */
void oracle_get_state(const oracle_session* s, double* phi_k, double* phi_km1,
                      double* y, double* q, double* sigma_p);
int  oracle_grid_of(const oracle_session* s);
void oracle_destroy(oracle_session* s);

/* ---- MD driver pieces (not part of the electrostatic path) ---- */
/* Born-Huggins-Mayer short range, minimum image, energy shifted at cutoff.
 * table: 3 rows (pair type species_i + species_j) of A, B, s, C, D. */
void oracle_bmh(int n, const double* pos, const int32_t* species, double box,
                const double* table, double cutoff, double* F, double* energy);
/* One velocity-Verlet step of ions under MaZe electrostatics + BMH.
 * On entry F_es and F_sr hold the forces at pos; on exit the new ones.
 * work accumulates the trapezoid work of the electrostatic force. */
int  oracle_md_step(oracle_session* s, int n, double* pos, double* vel,
                    const double* masses, const int32_t* species,
                    const double* table, double cutoff, double dt,
                    double accel_factor, double* F_es, double* F_sr,
                    double* work, double* v_sr, double* energy_c,
                    oracle_stats* st);

#ifdef __cplusplus
}
#endif
#endif
