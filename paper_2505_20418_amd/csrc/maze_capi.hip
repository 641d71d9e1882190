// Runtime and C ABI of the MI355X Poisson MaZe library: session
// allocation, the per-step launch sequence, the host loop that polls the
// device convergence flag, the mixed-precision refinement loop, checkpoints
// and the MD driver entry points.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "maze_internal.h"

using namespace maze;

namespace {

constexpr int kPollBatch = 8;          // CG iterations queued between polls
constexpr int kMaxRefinements = 40;    // mixed precision outer iterations
// Mixed precision: one FP32 inner solve may reduce the residual it starts
// from by at most kInnerReduction, and aims at kInnerMargin times the final
// threshold. The FP32 recursive residual tracks the FP64 true residual to a
// few parts in 1e4 over such a reduction (measured at 256^3), so a warm step
// normally finishes in one pass; restarting the inner CG earlier discards its
// Krylov space and costs iterations.
constexpr double kInnerReduction = 1e-7;
constexpr double kInnerMargin = 0.95;
constexpr uint64_t kMagic = 0x4d415a4531534553ull;  // "MAZE1SES"
constexpr int kProfMax = 512;          // sweeps timed per solve
constexpr int kProfStride = 4;         // every kProfStride-th sweep is timed

struct SaveHeader {
  uint64_t magic;
  int32_t abi, N, n_ions, order;
  int32_t precision, pad;
  int64_t step;
  double box, h;
};

}  // namespace

struct maze_session {
  maze_config cfg{};
  DeviceState d;
  MarchGeom geom{};
  SweepGeom sweep{};
  hipStream_t stream = nullptr;
  int device = 0;
  Scalars* host_sc = nullptr;   // pinned, 2 slots for pipelined polling
  hipEvent_t ev[2] = {nullptr, nullptr};
  long long step = 0;
  int last_iters = 0;
  // results of the last solve, filled by the host loop
  int iters = 0, refinements = 0, converged = 0;
  // inner iteration counts of the previous mixed solve, per refinement
  int last_inner[kMaxRefinements] = {0};
  char* base = nullptr;         // the session's single device allocation
  // optional sweep timing: event pairs around sampled sweeps
  bool prof = false;
  std::vector<hipEvent_t> pev;
  double prof_acc[8] = {0};
  // optional residual trace of the last solve: rows (pass, iteration, rel)
  bool trace = false;
  int trace_pass = 0;
  std::vector<double> trace_rows;
  std::vector<double> hist_host;
};

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return MAZE_E_DEVICE; \
  } while (0)

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static int grid_of(const maze_config* c) {
  if (!finite_pos(c->box) || !finite_pos(c->grid_spacing)) return 0;
  const double n = std::round(c->box / c->grid_spacing);
  if (!(n >= 4 && n <= 1024)) return 0;
  return (int)std::lround(c->box / c->grid_spacing);
}

static int validate(const maze_config* c) {
  if (!c) return MAZE_E_INVALID;
  if (c->n_ions <= 0 || (c->order != 2 && c->order != 4)) return MAZE_E_INVALID;
  if (!finite_pos(c->tol) || c->max_iter < 0) return MAZE_E_INVALID;
  if (c->precision != MAZE_FP64 && c->precision != MAZE_MIXED) return MAZE_E_INVALID;
  if (c->residual_norm != MAZE_NORM_REL2 && c->residual_norm != MAZE_NORM_ABSMAX)
    return MAZE_E_INVALID;
  if (c->flags != 0 || !finite_pos(c->coulomb_k)) return MAZE_E_INVALID;
  if (grid_of(c) == 0) return MAZE_E_INVALID;
  return MAZE_OK;
}

// Launch shape of the marching passes by grid size: enough workgroups to
// fill 256 CUs several times over, long enough x runs to amortise the two
// halo planes of each run.
static MarchGeom choose_geom(int N) {
  if (N >= 192) return make_march_geom(N, 4, 16);
  if (N >= 96) return make_march_geom(N, 2, 8);
  if (N >= 48) return make_march_geom(N, 1, 4);
  return make_march_geom(N, 1, 2);
}

// Launch shape of the fused CG sweep. A run of cx planes re-reads four halo
// planes of p and two of r, so runs are long; segments are sized to give
// about two workgroups per CU at 256^3.
static SweepGeom choose_sweep(int N) {
  if (N >= 192) return make_sweep_geom(N, 4, 32);
  if (N >= 96) return make_sweep_geom(N, 2, 16);
  if (N >= 48) return make_sweep_geom(N, 1, 8);
  return make_sweep_geom(N, 1, 4);
}

static int part_stride_for(const DeviceState& d, const MarchGeom& g, const SweepGeom& w) {
  return std::max({g.nwg, w.nwg, update_blocks(d.G), d.ntiles, 1});
}

struct Layout {
  size_t off[32];
  size_t total = 0;
  int n = 0;
  size_t add(size_t bytes) {
    const size_t o = total;
    off[n++] = o;
    total += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

// One device allocation per session, carved into the buffers below.
static Layout layout_for(const maze_config* c, int N, int* ntx_out, int* ntiles_out,
                         int* stride_out) {
  const long long G = (long long)N * N * N;
  const int ntx = (N + kTile - 1) / kTile;
  const int ntiles = ntx * ntx * ntx;
  DeviceState tmp;
  tmp.G = G;
  tmp.ntiles = ntiles;
  const int stride = part_stride_for(tmp, choose_geom(N), choose_sweep(N));
  const bool mixed = c->precision == MAZE_MIXED;
  const size_t n = (size_t)c->n_ions;
  Layout L;
  const size_t gd = sizeof(double) * (size_t)G, gf = sizeof(float) * (size_t)G;
  L.add(gd);                 // 0 phi_cur
  L.add(gd);                 // 1 phi_prev
  L.add(gd);                 // 2 y
  L.add(gd);                 // 3 q
  L.add(gd);                 // 4 sigma
  L.add(gd);                 // 5 xsolve
  L.add(mixed ? 0 : 2 * gd); // 6 r (two buffers)
  L.add(mixed ? 0 : 2 * gd); // 7 p (two buffers)
  L.add(mixed ? 2 * gf : 0); // 8 r32 (two buffers)
  L.add(mixed ? 2 * gf : 0); // 9 p32 (two buffers)
  L.add(mixed ? gf : 0);     // 10 e32
  L.add(sizeof(double) * (size_t)SL_COUNT * stride);  // 11 partials
  L.add(sizeof(Scalars));    // 12 scalars
  L.add(sizeof(double) * n); // 13 Q
  L.add(sizeof(int32_t) * ntiles);        // 14 tile_count
  L.add(sizeof(int32_t) * (ntiles + 1));  // 15 tile_start
  L.add(sizeof(int32_t) * ntiles);        // 16 tile_cursor
  L.add(sizeof(int32_t) * 3 * n);         // 17 ion_cell
  L.add(sizeof(double) * 3 * n);          // 18 ion_t
  L.add(sizeof(int32_t) * n);             // 19 sorted_idx
  L.add(sizeof(int32_t) * 3 * n);         // 20 s_cell
  L.add(sizeof(double) * 3 * n * c->order);  // 21 s_w
  L.add(sizeof(double) * n);              // 22 s_Q
  L.add(sizeof(double) * (n + 1));        // 23 md_epart
  L.add(sizeof(double) * kHistCap);       // 24 residual history
  if (ntx_out) *ntx_out = ntx;
  if (ntiles_out) *ntiles_out = ntiles;
  if (stride_out) *stride_out = stride;
  return L;
}

// ---------------------------------------------------------------------------
// Host loop of one CG solve: queue sweeps in batches, copy the device
// scalars to pinned memory after each batch, and stop queueing once a
// completed batch reports done (sweeps queued after convergence return at
// once). At most max_iter + 1 sweeps are queued (sweep 0 only forms p_0);
// after the last one a check kernel applies the stopping test.
// ---------------------------------------------------------------------------
static void prof_collect(maze_session* s, int timed, int iters, bool fp32) {
  double* acc = s->prof_acc + (fp32 ? 2 : 0);
  for (int j = 0; j < timed; ++j) {
    // sample j timed sweep k = 1 + j * kProfStride; sweeps past `iters`
    // returned without work and are not counted
    if (1 + j * kProfStride > iters) break;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->pev[2 * j], s->pev[2 * j + 1]) == hipSuccess) {
      acc[0] += 1;
      acc[1] += ms;
    }
  }
  s->prof_acc[fp32 ? 5 : 4] += iters;
}

static int run_cg(maze_session* s, void* x, bool fp32, bool zero_x, int max_iter,
                  int first_batch, int* iters, int* done_code) {
  DeviceState& d = s->d;
  const SweepGeom& w = s->sweep;
  const long long cap = (long long)max_iter + 1;
  long long k = 0;
  int batch = 0, timed = 0;
  bool have_prev = false, capped = false;
  const bool prof = s->prof;
  for (;;) {
    const int nb = (batch == 0) ? std::max(kPollBatch, first_batch) : kPollBatch;
    for (int b = 0; b < nb && k < cap; ++b, ++k) {
      const int nprev = (k == 0) ? s->geom.nwg : w.nwg;
      const bool timeit = prof && k >= 1 && (k - 1) % kProfStride == 0 && timed < kProfMax;
      if (timeit) HIP_TRY(hipEventRecord(s->pev[2 * timed], s->stream));
      HIP_TRY(launch_cg_sweep(d, w, (int)k, nprev, x, fp32, zero_x, s->stream));
      if (timeit) {
        HIP_TRY(hipEventRecord(s->pev[2 * timed + 1], s->stream));
        ++timed;
      }
    }
    if (k == cap && !capped) {
      HIP_TRY(launch_cg_check(d, (int)(k & 1), w.nwg, s->stream));
      capped = true;
    }
    const int slot = batch & 1;
    HIP_TRY(hipMemcpyAsync(&s->host_sc[slot], d.sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipEventRecord(s->ev[slot], s->stream));
    const int wait_slot = capped ? slot : (slot ^ 1);
    if (have_prev || capped) {
      HIP_TRY(hipEventSynchronize(s->ev[wait_slot]));
      const Scalars& h = s->host_sc[wait_slot];
      if (h.err) return MAZE_E_NONFINITE;
      if (h.done || capped) {
        *iters = h.iters;
        *done_code = h.done ? h.done : 3;
        if (prof) prof_collect(s, timed, h.iters, fp32);
        if (s->trace) {
          const int n = std::min(h.iters + 1, s->d.hist_cap);
          s->hist_host.resize(n);
          HIP_TRY(hipMemcpyAsync(s->hist_host.data(), s->d.hist, sizeof(double) * n,
                                 hipMemcpyDeviceToHost, s->stream));
          HIP_TRY(hipStreamSynchronize(s->stream));
          const double qn = h.qnorm > 0 ? h.qnorm : 1.0;
          for (int t = 0; t < n; ++t) {
            s->trace_rows.push_back(s->trace_pass);
            s->trace_rows.push_back(t);
            s->trace_rows.push_back(s->hist_host[t] / qn);
          }
        }
        return MAZE_OK;
      }
    }
    have_prev = true;
    ++batch;
  }
}

static int read_scalars(maze_session* s, Scalars* out) {
  HIP_TRY(hipMemcpyAsync(&s->host_sc[0], s->d.sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  *out = s->host_sc[0];
  return MAZE_OK;
}

// Resets the binning counters and the error flag after a rejected input.
static int recover_error(maze_session* s) {
  DeviceState& d = s->d;
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemsetAsync(d.tile_count, 0, sizeof(int32_t) * d.ntiles, s->stream));
  HIP_TRY(hipMemsetAsync(&d.sc->err, 0, sizeof(int32_t), s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MAZE_E_NONFINITE;
}

// Solve of M x = s (s already in d.sigma, first residual and its partials
// written by a right-hand-side kernel, thresholds set by FIN_SOLVE_START).
// Leaves the true residual and mean of x in the scalars (FIN_SOLVE_END).
static int solve(maze_session* s, double* x) {
  DeviceState& d = s->d;
  const MarchGeom& g = s->geom;
  const bool mixed = s->cfg.precision == MAZE_MIXED;
  s->iters = 0;
  s->refinements = 0;
  s->converged = 0;
  s->trace_rows.clear();
  s->trace_pass = 0;
  if (!mixed) {
    int it = 0, code = 0;
    const int rc = run_cg(s, x, false, false, s->cfg.max_iter,
                          std::max(0, s->last_iters - 2 * kPollBatch), &it, &code);
    if (rc != MAZE_OK) return rc;
    s->iters = it;
    s->converged = (code == 1);
    HIP_TRY(launch_true_residual(d, g, x, s->stream));
    HIP_TRY(launch_finalize(d, FIN_SOLVE_END, g.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0, s->stream));
    return MAZE_OK;
  }
  // Mixed precision: FP32 inner CG on the correction, FP64 outer residual.
  Scalars h;
  int rc = read_scalars(s, &h);
  if (rc != MAZE_OK) return rc;
  if (h.err) return MAZE_E_NONFINITE;
  const double thr = h.thr;
  const bool absmax = s->cfg.residual_norm == MAZE_NORM_ABSMAX;
  int total = 0;
  for (;;) {
    const double res = absmax ? h.true_max : std::sqrt(h.true_rr);
    if (s->trace) {
      s->trace_rows.push_back(s->refinements);
      s->trace_rows.push_back(-1);
      s->trace_rows.push_back(std::sqrt(h.true_rr) / (h.qnorm > 0 ? h.qnorm : 1.0));
    }
    s->trace_pass = s->refinements;
    if (res <= thr) {
      s->converged = 1;
      break;
    }
    if (s->refinements >= kMaxRefinements || total >= s->cfg.max_iter) break;
    const double inner = std::max(kInnerReduction * res, kInnerMargin * thr);
    HIP_TRY(launch_finalize(d, FIN_INNER_START, 0, 0.0, inner, 0.0, nullptr,
                            s->cfg.max_iter - total, s->cfg.residual_norm, s->stream));
    int it = 0, code = 0;
    const int guess_it = s->last_inner[s->refinements];
    rc = run_cg(s, d.e32, true, true, s->cfg.max_iter - total,
                std::max(0, guess_it - 2 * kPollBatch), &it, &code);
    if (rc != MAZE_OK) return rc;
    s->last_inner[s->refinements] = it;
    total += it;
    s->refinements += 1;
    HIP_TRY(launch_add_correction(d, x, s->stream));
    HIP_TRY(launch_refine(d, g, x, true, s->stream));
    HIP_TRY(launch_finalize(d, FIN_SOLVE_END, g.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0, s->stream));
    rc = read_scalars(s, &h);
    if (rc != MAZE_OK) return rc;
    if (code == 2 && it == 0) break;  // breakdown without progress
  }
  s->iters = total;
  return MAZE_OK;
}

static void fill_stats(maze_session* s, const Scalars& h, maze_stats* st) {
  st->grid_n = s->d.N;
  st->iters = s->iters;
  st->refinements = s->refinements;
  st->converged = s->converged;
  st->h = s->d.h;
  st->rel_residual = (h.qnorm > 0) ? std::sqrt(h.true_rr) / h.qnorm : std::sqrt(h.true_rr);
  st->max_abs_residual = h.true_max;
  st->net_charge = h.qsum;
  st->energy = h.energy;
}

static int finish_call(maze_session* s, maze_stats* st) {
  if (st) {
    Scalars h;
    const int rc = read_scalars(s, &h);
    if (rc != MAZE_OK) return rc;
    fill_stats(s, h, st);
  }
  return s->converged ? MAZE_OK : MAZE_NOT_CONVERGED;
}

// Assignment of the charge of `pos` into d.q and its raw sum.
static int assign(maze_session* s, const double* pos) {
  DeviceState& d = s->d;
  HIP_TRY(launch_bin(d, pos, s->stream));
  HIP_TRY(launch_spread(d, s->stream));
  HIP_TRY(launch_finalize(d, FIN_QSUM, d.ntiles, 0.0, 0.0, 0.0, nullptr, 0, 0, s->stream));
  return MAZE_OK;
}

// Direct Poisson solve into x from the given guess; projects x, energy,
// optional field and forces.
static int direct_solve(maze_session* s, int guess, const double* pos, double* x,
                        double* field, double* forces, double* energy) {
  DeviceState& d = s->d;
  const bool mixed = s->cfg.precision == MAZE_MIXED;
  int rc = assign(s, pos);
  if (rc != MAZE_OK) return rc;
  HIP_TRY(launch_rhs_poisson(d, s->geom, guess, x, mixed, s->stream));
  HIP_TRY(launch_finalize(d, FIN_SOLVE_START, s->geom.nwg, s->cfg.tol, 0.0, 0.0, nullptr,
                          s->cfg.max_iter, s->cfg.residual_norm, s->stream));
  rc = solve(s, x);
  if (rc == MAZE_E_NONFINITE) return recover_error(s);
  if (rc != MAZE_OK) return rc;
  HIP_TRY(launch_project(d, x, field, s->stream));
  HIP_TRY(launch_finalize(d, FIN_ENERGY, update_blocks(d.G), 0.0, 0.0, s->cfg.coulomb_k,
                          energy, 0, 0, s->stream));
  if (forces) HIP_TRY(launch_gather(d, x, s->cfg.coulomb_k, forces, s->stream));
  return MAZE_OK;
}

extern "C" {

int maze_abi_version(void) { return MAZE_ABI_VERSION; }

const char* maze_strerror(int status) {
  switch (status) {
    case MAZE_OK: return "ok";
    case MAZE_NOT_CONVERGED: return "solver did not reach the tolerance (outputs written)";
    case MAZE_E_INVALID: return "invalid argument";
    case MAZE_E_NOT_NEUTRAL: return "charges are not neutral";
    case MAZE_E_OOM: return "device allocation failed";
    case MAZE_E_DEVICE: return "HIP runtime error";
    case MAZE_E_NONFINITE: return "non-finite position";
    default: return "unknown status";
  }
}

size_t maze_device_bytes(const maze_config* cfg) {
  if (validate(cfg) != MAZE_OK) return 0;
  const Layout L = layout_for(cfg, grid_of(cfg), nullptr, nullptr, nullptr);
  return L.total;
}

int maze_grid_n(const maze_session* s) { return s ? s->d.N : 0; }

void maze_destroy(maze_session* s) {
  if (!s) return;
  hipSetDevice(s->device);
  if (s->stream) hipStreamSynchronize(s->stream);
  else hipDeviceSynchronize();
  if (s->base) hipFree(s->base);
  if (s->host_sc) hipHostFree(s->host_sc);
  for (auto& e : s->pev)
    if (e) hipEventDestroy(e);
  for (auto& e : s->ev)
    if (e) hipEventDestroy(e);
  delete s;
}

int maze_init(const maze_config* cfg, const double* charges_dev, const double* pos0_dev,
              maze_session** out, maze_stats* st) {
  if (!out) return MAZE_E_INVALID;
  *out = nullptr;
  int rc = validate(cfg);
  if (rc != MAZE_OK) return rc;
  if (!charges_dev || !pos0_dev) return MAZE_E_INVALID;
  const int n = cfg->n_ions;
  const hipStream_t stream = (hipStream_t)cfg->stream;

  // neutrality check on a host copy of the charges
  double* hq = new (std::nothrow) double[n];
  if (!hq) return MAZE_E_OOM;
  if (hipMemcpyAsync(hq, charges_dev, sizeof(double) * n, hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    delete[] hq;
    return MAZE_E_DEVICE;
  }
  double qs = 0, qa = 0;
  bool qfin = true;
  for (int i = 0; i < n; ++i) {
    qs += hq[i];
    qa += std::fabs(hq[i]);
    qfin &= std::isfinite(hq[i]);
  }
  delete[] hq;
  if (!qfin) return MAZE_E_INVALID;
  if (std::fabs(qs) > 1e-10 * qa) return MAZE_E_NOT_NEUTRAL;

  maze_session* s = new (std::nothrow) maze_session();
  if (!s) return MAZE_E_OOM;
  s->cfg = *cfg;
  s->stream = stream;
  hipGetDevice(&s->device);
  DeviceState& d = s->d;
  d.N = grid_of(cfg);
  d.G = (long long)d.N * d.N * d.N;
  d.n_ions = n;
  d.order = cfg->order;
  d.box = cfg->box;
  d.h = cfg->box / d.N;
  s->geom = choose_geom(d.N);
  s->sweep = choose_sweep(d.N);
  const Layout L = layout_for(cfg, d.N, &d.ntx, &d.ntiles, &d.part_stride);
  char* base = nullptr;
  if (hipMalloc((void**)&base, L.total) != hipSuccess) {
    hipGetLastError();
    delete s;
    return MAZE_E_OOM;
  }
  s->base = base;
  auto at = [&](int i) { return (void*)(base + L.off[i]); };
  const bool mixed = cfg->precision == MAZE_MIXED;
  d.phi_cur = (double*)at(0);
  d.phi_prev = (double*)at(1);
  d.y = (double*)at(2);
  d.q = (double*)at(3);
  d.sigma = (double*)at(4);
  d.xsolve = (double*)at(5);
  d.r = mixed ? nullptr : (double*)at(6);
  d.p = mixed ? nullptr : (double*)at(7);
  d.r32 = mixed ? (float*)at(8) : nullptr;
  d.p32 = mixed ? (float*)at(9) : nullptr;
  d.e32 = mixed ? (float*)at(10) : nullptr;
  d.part = (double*)at(11);
  d.sc = (Scalars*)at(12);
  d.Q = (double*)at(13);
  d.tile_count = (int32_t*)at(14);
  d.tile_start = (int32_t*)at(15);
  d.tile_cursor = (int32_t*)at(16);
  d.ion_cell = (int32_t*)at(17);
  d.ion_t = (double*)at(18);
  d.sorted_idx = (int32_t*)at(19);
  d.s_cell = (int32_t*)at(20);
  d.s_w = (double*)at(21);
  d.s_Q = (double*)at(22);
  d.md_epart = (double*)at(23);
  d.hist = (double*)at(24);
  d.hist_cap = kHistCap;
  if (hipHostMalloc((void**)&s->host_sc, 2 * sizeof(Scalars), hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreateWithFlags(&s->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev[1], hipEventDisableTiming) != hipSuccess) {
    maze_destroy(s);
    return MAZE_E_DEVICE;
  }
  // zero everything once (not part of any step, so never graph-captured)
  if (hipMemsetAsync(base, 0, L.total, stream) != hipSuccess ||
      hipMemcpyAsync(d.Q, charges_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, stream) !=
          hipSuccess) {
    maze_destroy(s);
    return MAZE_E_DEVICE;
  }
  Scalars init{};
  init.max_iter = cfg->max_iter;
  init.norm = cfg->residual_norm;
  if (hipMemcpy(d.sc, &init, sizeof(Scalars), hipMemcpyHostToDevice) != hipSuccess) {
    maze_destroy(s);
    return MAZE_E_DEVICE;
  }
  // cold Poisson solve for phi^0 from zero; phi^{-1} = phi^0; y = 0
  rc = direct_solve(s, MAZE_GUESS_ZERO, pos0_dev, d.phi_cur, nullptr, nullptr, nullptr);
  if (rc < 0) {
    maze_destroy(s);
    return rc;
  }
  if (hipMemcpyAsync(d.phi_prev, d.phi_cur, sizeof(double) * d.G, hipMemcpyDeviceToDevice,
                     stream) != hipSuccess) {
    maze_destroy(s);
    return MAZE_E_DEVICE;
  }
  s->last_iters = 0;
  rc = finish_call(s, st);
  if (rc < 0) {
    maze_destroy(s);
    return rc;
  }
  *out = s;
  return rc;
}

int maze_step(maze_session* s, const double* pos_dev, double* field_dev, double* forces_dev,
              double* energy_dev, maze_stats* st) {
  if (!s || !pos_dev) return MAZE_E_INVALID;
  hipSetDevice(s->device);
  DeviceState& d = s->d;
  const bool mixed = s->cfg.precision == MAZE_MIXED;
  int rc = assign(s, pos_dev);
  if (rc != MAZE_OK) return rc;
  HIP_TRY(launch_rhs_maze(d, s->geom, mixed, s->stream));
  HIP_TRY(launch_finalize(d, FIN_SOLVE_START, s->geom.nwg, s->cfg.tol, 0.0, 0.0, nullptr,
                          s->cfg.max_iter, s->cfg.residual_norm, s->stream));
  rc = solve(s, d.y);
  if (rc == MAZE_E_NONFINITE) return recover_error(s);
  if (rc != MAZE_OK) return rc;
  s->last_iters = s->iters;
  HIP_TRY(launch_update(d, field_dev, s->stream));
  HIP_TRY(launch_finalize(d, FIN_ENERGY, update_blocks(d.G), 0.0, 0.0, s->cfg.coulomb_k,
                          energy_dev, 0, 0, s->stream));
  if (forces_dev) HIP_TRY(launch_gather(d, d.phi_prev, s->cfg.coulomb_k, forces_dev, s->stream));
  std::swap(d.phi_cur, d.phi_prev);
  s->step += 1;
  return finish_call(s, st);
}

int maze_solve(maze_session* s, int guess, const double* pos_dev, double* field_dev,
               double* forces_dev, double* energy_dev, maze_stats* st) {
  if (!s || !pos_dev) return MAZE_E_INVALID;
  if (guess < MAZE_GUESS_ZERO || guess > MAZE_GUESS_TIMEPROP) return MAZE_E_INVALID;
  hipSetDevice(s->device);
  const int keep = s->last_iters;
  s->last_iters = 0;
  const int rc = direct_solve(s, guess, pos_dev, s->d.xsolve, field_dev, forces_dev, energy_dev);
  s->last_iters = keep;
  if (rc != MAZE_OK) return rc;
  return finish_call(s, st);
}

int maze_step_batch(maze_session* const* sessions, int32_t count, const double* const* pos_dev,
                    double* const* forces_dev, double* energies_dev, maze_stats* st) {
  if (!sessions || count <= 0 || !pos_dev) return MAZE_E_INVALID;
  int worst = MAZE_OK;
  for (int i = 0; i < count; ++i) {
    const int rc = maze_step(sessions[i], pos_dev[i], nullptr, forces_dev ? forces_dev[i] : nullptr,
                             energies_dev ? energies_dev + i : nullptr, st ? st + i : nullptr);
    if (rc < 0 && (worst >= 0 || rc < worst)) worst = rc;
    else if (worst >= 0 && rc > worst) worst = rc;
  }
  return worst;
}

int maze_get_grid(const maze_session* s, int which, double* out_dev) {
  if (!s || !out_dev) return MAZE_E_INVALID;
  const DeviceState& d = s->d;
  const double* src = nullptr;
  switch (which) {
    case 0: src = d.phi_cur; break;
    case 1: src = d.phi_prev; break;
    case 2: src = d.y; break;
    case 3: src = d.q; break;
    case 4: src = d.sigma; break;
    default: return MAZE_E_INVALID;
  }
  hipSetDevice(s->device);
  HIP_TRY(hipMemcpyAsync(out_dev, src, sizeof(double) * d.G, hipMemcpyDeviceToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MAZE_OK;
}

size_t maze_state_bytes(const maze_session* s) {
  if (!s) return 0;
  return sizeof(SaveHeader) + 3 * sizeof(double) * (size_t)s->d.G;
}

int maze_save(const maze_session* s, void* host_buf, size_t bytes) {
  if (!s || !host_buf || bytes < maze_state_bytes(s)) return MAZE_E_INVALID;
  hipSetDevice(s->device);
  const DeviceState& d = s->d;
  SaveHeader h{};
  h.magic = kMagic;
  h.abi = MAZE_ABI_VERSION;
  h.N = d.N;
  h.n_ions = d.n_ions;
  h.order = d.order;
  h.precision = s->cfg.precision;
  h.step = s->step;
  h.box = d.box;
  h.h = d.h;
  char* p = (char*)host_buf;
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  const size_t gb = sizeof(double) * (size_t)d.G;
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemcpy(p, d.phi_cur, gb, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(p + gb, d.phi_prev, gb, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(p + 2 * gb, d.y, gb, hipMemcpyDeviceToHost));
  return MAZE_OK;
}

int maze_load(maze_session* s, const void* host_buf, size_t bytes) {
  if (!s || !host_buf || bytes < sizeof(SaveHeader)) return MAZE_E_INVALID;
  SaveHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  DeviceState& d = s->d;
  if (h.magic != kMagic || h.abi != MAZE_ABI_VERSION || h.N != d.N || h.n_ions != d.n_ions ||
      h.order != d.order || h.box != d.box || bytes < maze_state_bytes(s))
    return MAZE_E_INVALID;
  hipSetDevice(s->device);
  const char* p = (const char*)host_buf + sizeof(h);
  const size_t gb = sizeof(double) * (size_t)d.G;
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemcpy(d.phi_cur, p, gb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d.phi_prev, p + gb, gb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d.y, p + 2 * gb, gb, hipMemcpyHostToDevice));
  s->step = h.step;
  s->last_iters = 0;
  return MAZE_OK;
}

int maze_profile_enable(maze_session* s, int on) {
  if (!s) return MAZE_E_INVALID;
  hipSetDevice(s->device);
  if (on && s->pev.empty()) {
    s->pev.assign(2 * kProfMax, nullptr);
    for (auto& e : s->pev)
      if (hipEventCreate(&e) != hipSuccess) return MAZE_E_DEVICE;
  }
  s->prof = on != 0;
  for (double& v : s->prof_acc) v = 0.0;
  return MAZE_OK;
}

int maze_profile_read(maze_session* s, double* out8) {
  if (!s || !out8) return MAZE_E_INVALID;
  for (int i = 0; i < 8; ++i) {
    out8[i] = s->prof_acc[i];
    s->prof_acc[i] = 0.0;
  }
  return MAZE_OK;
}

int maze_trace_enable(maze_session* s, int on) {
  if (!s) return MAZE_E_INVALID;
  s->trace = on != 0;
  s->trace_rows.clear();
  return MAZE_OK;
}

int maze_trace_read(const maze_session* s, double* out, int max_rows, int* n_rows) {
  if (!s || (!out && max_rows > 0) || max_rows < 0) return MAZE_E_INVALID;
  const int n = (int)(s->trace_rows.size() / 3);
  const int m = std::min(n, max_rows);
  if (m > 0) std::memcpy(out, s->trace_rows.data(), sizeof(double) * 3 * (size_t)m);
  if (n_rows) *n_rows = n;
  return MAZE_OK;
}

static int md_check(const maze_session* s, const maze_md_state* md) {
  if (!s || !md || md->n_ions != s->d.n_ions || !md->pos_dev || !md->vel_dev || !md->mass_dev ||
      !md->species_dev || !md->f_es_dev || !md->f_sr_dev || !md->scratch_dev || !md->scalars_dev)
    return MAZE_E_INVALID;
  if (!(md->dt > 0) || !(md->accel > 0) || !(md->cutoff > 0) || md->cutoff > 0.5 * s->d.box)
    return MAZE_E_INVALID;
  return MAZE_OK;
}

int maze_md_prime(maze_session* s, const maze_md_state* md, maze_stats* st) {
  int rc = md_check(s, md);
  if (rc != MAZE_OK) return rc;
  rc = maze_step(s, md->pos_dev, nullptr, md->f_es_dev, md->scalars_dev + 6, nullptr);
  if (rc < 0) return rc;
  HIP_TRY(launch_md_bmh(*md, s->d, s->stream));
  HIP_TRY(launch_md_prime(*md, s->d, s->stream));
  const int rc2 = finish_call(s, st);
  return rc2 < 0 ? rc2 : rc;
}

int maze_md_step(maze_session* s, const maze_md_state* md, maze_stats* st) {
  int rc = md_check(s, md);
  if (rc != MAZE_OK) return rc;
  hipSetDevice(s->device);
  HIP_TRY(launch_md_kick_drift(*md, s->stream));
  rc = maze_step(s, md->pos_dev, nullptr, md->f_es_dev, md->scalars_dev + 6, nullptr);
  if (rc < 0) return rc;
  HIP_TRY(launch_md_bmh(*md, s->d, s->stream));
  HIP_TRY(launch_md_finish(*md, s->d, s->stream));
  const int rc2 = finish_call(s, st);
  return rc2 < 0 ? rc2 : rc;
}

}  // extern "C"
