// Runtime and C ABI of the MI355X Poisson MaZe library: session
// allocation, the per-step launch sequence, the host loop that polls the
// device convergence flag, the mixed-precision refinement loop, checkpoints
// and the MD driver entry points.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
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
// threshold. Restarting the inner CG early discards its Krylov space and
// costs iterations. With the two-iteration CG the FP32 recursive residual
// ends 10-14% below the FP64 true residual at 256^3, so a first pass aimed at
// 0.95 of the threshold was followed by a short second pass in nearly every
// step; aimed at 0.92 it is in about a quarter of the steps (measured mixed
// 256^3 MD steps/s: 0.95 63.54, 0.92 64.00, 0.90 63.87, 0.88 63.60, 0.85
// 63.16).
constexpr double kInnerReduction = 1e-7;
constexpr double kInnerMargin = 0.92;
constexpr uint64_t kMagic = 0x4d415a4531534553ull;  // "MAZE1SES"
constexpr int kProfMax = 512;          // sweeps timed per solve
constexpr int kProfStride = 16;        // every kProfStride-th sweep is timed

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
  SweepGeom sweep{};     // latency shape: alone and in batches below the fill level
  SweepGeom sweep_tp{};  // throughput shape: batches that fill the GPU
  SweepGeom sbasis{};    // basis kernel of the two-iteration CG (own shape)
  hipStream_t stream = nullptr;
  // captured chunks of kPollBatch sweeps, [fp32][parity of the first sweep]
  // [slot]: a graph holds its kernels' arguments, and the solution vector
  // differs between solves (y for MaZe steps, the direct-solve buffer, the
  // field for the cold solve), so each graph is kept with the x it updates
  struct ChunkGraph {
    hipGraphExec_t exec = nullptr;
    void* x = nullptr;
  };
  static constexpr int kChunkSlots = 4;
  ChunkGraph chunk[2][2][kChunkSlots];
  int chunk_next[2][2] = {{0, 0}, {0, 0}};
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
  const int32_t known = MAZE_FLAG_MULTIGRID | MAZE_FLAG_WEIGHT_GRADIENT_FORCE |
                        MAZE_FLAG_ALLOW_NET_CHARGE | MAZE_FLAG_GRAPH_CHUNKS | MAZE_FLAG_SSTEP;
  if ((c->flags & ~known) != 0 || !finite_pos(c->coulomb_k)) return MAZE_E_INVALID;
  if ((c->flags & MAZE_FLAG_SSTEP) && (c->flags & MAZE_FLAG_MULTIGRID)) return MAZE_E_INVALID;
  // the null stream cannot be captured
  if ((c->flags & MAZE_FLAG_GRAPH_CHUNKS) && c->stream == nullptr) return MAZE_E_INVALID;
  if (grid_of(c) == 0) return MAZE_E_INVALID;
  if (c->flags & MAZE_FLAG_MULTIGRID) {
    int Ns[kMgMaxLevels];
    if (mg_plan(grid_of(c), Ns, kMgMaxLevels) == 0) return MAZE_E_INVALID;
  }
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
  if (N >= 128) return make_sweep_geom(N, 2, 16);
  if (N >= 48) return make_sweep_geom(N, 1, 8);
  return make_sweep_geom(N, 1, 4);
}

// Launch shapes the autotuner times: segments of 256, 512 or 1024 points
// of the (y, z) plane, runs of 4 to 64 x planes (1 and 2 as well on grids up
// to 96^3), and the runs that make the
// workgroup count k times the device's CU count (k = 1..8), since a launch
// whose last round of workgroups only partly fills the CUs leaves them idle
// for that round. Shapes whose halo slots or LDS do not fit a kernel
// instantiation are left out; of runs giving the same number of chunks only
// the most even split is kept.
static std::vector<SweepGeom> sweep_candidates(int N, bool fp32, int cus) {
  std::vector<SweepGeom> out;
  const int P = N * N;
  for (int ppt : {1, 2, 4}) {
    if (ppt > 1 && kThreads * ppt / 2 >= P) continue;  // segment longer than a plane
    const int nseg = (P + kThreads * ppt - 1) / (kThreads * ppt);
    std::vector<int> cxs = {4, 8, 16, 32, 64};
    // small grids are bound by the latency of a workgroup's serial plane
    // steps (run + 2), not by bandwidth: shorter runs, more workgroups
    if (N <= 96) {
      cxs.push_back(1);
      cxs.push_back(2);
    }
    for (int k = 1; k <= 8 && cus > 0; ++k) {
      const int nchunk = (k * cus + nseg - 1) / nseg;
      if (nchunk >= 1 && nchunk <= N) cxs.push_back((N + nchunk - 1) / nchunk);
    }
    for (int cx : cxs) {
      if (cx > N && cx != 4) continue;
      const SweepGeom g0 = make_sweep_geom(N, ppt, cx);
      const SweepGeom g = make_sweep_geom(N, ppt, (N + g0.nchunk - 1) / g0.nchunk);
      if (sweep_nh_class(g.nh) == 0) continue;
      if (sweep_lds_bytes(g, fp32, false) > 159 * 1024) continue;
      bool dup = false;
      for (const SweepGeom& o : out) dup |= (o.ppt == g.ppt && o.nchunk == g.nchunk);
      if (!dup) out.push_back(g);
    }
  }
  return out;
}

// CUs of the current device (0 if it cannot be read).
static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

static int part_stride_for(const DeviceState& d, const MarchGeom& g, const SweepGeom& w) {
  int m = std::max({g.nwg, w.nwg, update_blocks(d.G), d.ntiles, 1});
  const int N = g.N;
  // sized for the fixed list; CU-multiple candidates that would not fit are
  // skipped by the tuner
  for (bool f : {false, true})
    for (const SweepGeom& c : sweep_candidates(N, f, 0)) m = std::max(m, c.nwg);
  return m;
}

struct Layout {
  size_t off[64];
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
  const bool mg = (c->flags & MAZE_FLAG_MULTIGRID) != 0;
  // the multigrid-preconditioned CG is FP64 outside the V-cycle; the mixed
  // mode runs its V-cycle in FP32
  const bool mixed = c->precision == MAZE_MIXED && !mg;
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
  L.add(sizeof(double) * (size_t)SL_COUNT * stride);  // partial-sum table
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
  L.add(sizeof(int32_t) * (size_t)ntx * (1 + kMaxCandAxis));  // 25 spreading candidates
  if (mg) {
    int Ns[kMgMaxLevels];
    const int levels = mg_plan(N, Ns, kMgMaxLevels);
    const size_t es = (c->precision == MAZE_MIXED) ? sizeof(float) : sizeof(double);
    const bool f32 = es == sizeof(float);
    L.add(f32 ? es * (size_t)G : 0);  // 26 z (FP64 uses the second r buffer)
    L.add(f32 ? es * (size_t)G : 0);  // 27 rounded level-0 right-hand side
    L.add(es * (size_t)G);            // 28 level-0 residual
    for (int l = 1; l < levels; ++l) {
      const size_t gl = (size_t)Ns[l] * Ns[l] * Ns[l];
      L.add(es * gl);  // x_l
      L.add(es * gl);  // b_l
      L.add(es * gl);  // r_l
    }
  }
  if (ntx_out) *ntx_out = ntx;
  if (ntiles_out) *ntiles_out = ntiles;
  if (stride_out) *stride_out = stride;
  return L;
}

// ---------------------------------------------------------------------------
// CG host loops. Sweeps are queued in groups of kPollBatch; after each group
// the solve's status is copied to pinned memory, and the status of the group
// before is waited for, so the device always has a group queued. Sweeps
// queued after convergence return at once. The device applies the stopping
// test and the iteration cap itself (sweep k stops when k - 1 updates reach
// max_iter), so the host only counts sweeps as a guard.
// ---------------------------------------------------------------------------
// last: index of the last unit that did work in the solve. Sweep k applies
// iteration k, so a solve of n iterations ends with sweep n; outer step k of
// the two-iteration form applies iterations 2k+1 and 2k+2, so it ends with
// outer step (n + 1) / 2 - 1.
static void prof_collect(maze_session* s, int timed, int last, int iters, bool fp32,
                         bool sstep) {
  double* acc = s->prof_acc + (fp32 ? 2 : 0);
  for (int j = 0; j < timed; ++j) {
    // sample j timed unit k = 1 + j * kProfStride; units past `last`
    // returned without work and are not counted
    if (1 + j * kProfStride > last) break;
    float ms = 0.f, mu = 0.f;
    if (hipEventElapsedTime(&ms, s->pev[3 * j], s->pev[3 * j + 2]) == hipSuccess &&
        (!sstep || hipEventElapsedTime(&mu, s->pev[3 * j + 1], s->pev[3 * j + 2]) == hipSuccess)) {
      acc[0] += 1;
      acc[1] += ms;
      s->prof_acc[fp32 ? 7 : 6] += mu;
    }
  }
  s->prof_acc[fp32 ? 5 : 4] += iters;
}

// Appends the residual history of the solve that just ended to the trace.
static int trace_collect(maze_session* s, int iters, double qnorm) {
  const int n = std::min(iters + 1, s->d.hist_cap);
  s->hist_host.resize(n);
  HIP_TRY(hipMemcpyAsync(s->hist_host.data(), s->d.hist, sizeof(double) * n,
                         hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const double qn = qnorm > 0 ? qnorm : 1.0;
  for (int t = 0; t < n; ++t) {
    s->trace_rows.push_back(s->trace_pass);
    s->trace_rows.push_back(t);
    s->trace_rows.push_back(s->hist_host[t] / qn);
  }
  return MAZE_OK;
}

// One CG solve on one session: x is double* (FP64) or float* (FP32, then
// zero_x starts it from zero). max_iter bounds the host guard only.
struct CgJob {
  maze_session* s;
  void* x;
  int max_iter;
  int iters = 0, code = 0, err = 0;
};

static long long sweep_guard(int max_iter, int first_batch) {
  return (long long)max_iter + 4LL * kPollBatch + first_batch + 64;
}

// Captures one poll group of units starting at parity par0 (never the first sweep
// of a solve) on the session's stream into a graph. The sweeps' arguments
// depend only on the session, the precision and the parity, so one graph
// serves every later chunk of every solve.
static bool sstep_of(const maze_session* s) { return (s->cfg.flags & MAZE_FLAG_SSTEP) != 0; }
// Iterations to queue before the first poll of a solve, from the iteration
// count of the same solve in the previous step: short of it by an eighth
// (at least two poll groups of sweeps), since iteration counts move by a
// few percent from step to step and units queued past convergence run for
// nothing, while the rest of the solve is queued in poll groups.
static int first_batch_of(int last_iters) {
  return std::max(0, last_iters - std::max(2 * kPollBatch, last_iters / 8));
}

// CG units queued between polls: sweeps, or two-iteration outer steps.
// Enough for about 100 us (sweeps) or 200 us (outer steps) of device work (a
// unit moves 24-64 B per point at some 5 TB/s, plus about 10 us of launch
// and reduction latency), so the device stays busy through the host's poll;
// no more, because the units queued after convergence run for nothing (at
// 256^3 a group of four outer steps left about eight such launches per
// solve). At 256^3 the FP32 outer steps go two to a group instead of one
// (mixed MD steps/s 64.55 -> 64.68; FP64 outer steps stay one to a group).
static int poll_units(const maze_session* s, bool fp32) {
  const bool ss = sstep_of(s);
  const double bytes = (ss ? 32.0 : 24.0) * (fp32 ? 1.0 : 2.0);
  const double unit_us = (double)s->d.G * bytes / 5.0e6 + 10.0;
  const int cap = ss ? kPollBatch / 2 : kPollBatch;
  const double target_us = ss ? 200.0 : 100.0;
  return std::max(1, std::min(cap, (int)std::ceil(target_us / unit_us)));
}

// Unit k of a solve: sweep k, or outer step k of the two-iteration form.
static hipError_t launch_unit(maze_session* s, long long k, void* x, bool fp32, bool zero_x) {
  const int kk = (int)(k & 0x7fffffff);
  if (sstep_of(s))
    return launch_sstep_outer(s->d, s->sbasis, s->sweep, kk, x, fp32, zero_x, s->stream);
  return launch_cg_sweep(s->d, s->sweep, kk, s->geom.nwg, x, fp32, zero_x, s->stream);
}

static int chunk_graph(maze_session* s, bool fp32, int par0, void* x, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int b = 0; b < poll_units(s, fp32) && e == hipSuccess; ++b)
    e = launch_unit(s, 2 + par0 + b, x, fp32, false);
  const hipError_t e2 = hipStreamEndCapture(s->stream, &g);
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return MAZE_E_DEVICE;
  }
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return MAZE_E_DEVICE;
  }
  return MAZE_OK;
}

static int run_cg(CgJob& job, bool fp32, bool zero_x, int first_batch) {
  maze_session* s = job.s;
  DeviceState& d = s->d;
  const SweepGeom& w = s->sweep;
  const long long guard = sweep_guard(job.max_iter, first_batch);
  const bool ss = sstep_of(s);
  const int per = poll_units(s, fp32);
  // first_batch counts iterations; a two-iteration unit covers two
  const int first_units = ss ? first_batch / 2 : first_batch;
  long long k = 0;
  int batch = 0, timed = 0;
  bool have_prev = false;
  const bool prof = s->prof;
  const bool graphs = (s->cfg.flags & MAZE_FLAG_GRAPH_CHUNKS) && !prof;
  for (;;) {
    const int nb = (batch == 0) ? std::max(per, first_units) : per;
    if (graphs && batch > 0) {
      const int f = fp32 ? 1 : 0, par = (int)(k & 1);
      maze_session::ChunkGraph* hit = nullptr;
      for (auto& c : s->chunk[f][par])
        if (c.exec && c.x == job.x) hit = &c;
      if (!hit) {
        hit = &s->chunk[f][par][s->chunk_next[f][par]];
        s->chunk_next[f][par] = (s->chunk_next[f][par] + 1) % maze_session::kChunkSlots;
        if (hit->exec) {
          (void)hipGraphExecDestroy(hit->exec);
          hit->exec = nullptr;
        }
        const int rc = chunk_graph(s, fp32, par, job.x, &hit->exec);
        if (rc != MAZE_OK) return rc;
        hit->x = job.x;
      }
      HIP_TRY(hipGraphLaunch(hit->exec, s->stream));
      k += nb;
    }
    for (int b = 0; b < nb && !(graphs && batch > 0); ++b, ++k) {
      const bool timeit = prof && k >= 1 && (k - 1) % kProfStride == 0 && timed < kProfMax;
      if (timeit) HIP_TRY(hipEventRecord(s->pev[3 * timed], s->stream));
      if (ss && timeit) {
        // basis and update kernels timed apart
        const int kk = (int)(k & 0x7fffffff);
        HIP_TRY(launch_sstep_half(d, s->sbasis, w, kk, job.x, fp32, zero_x, false, s->stream));
        HIP_TRY(hipEventRecord(s->pev[3 * timed + 1], s->stream));
        HIP_TRY(launch_sstep_half(d, s->sbasis, w, kk, job.x, fp32, zero_x, true, s->stream));
      } else {
        HIP_TRY(launch_unit(s, k, job.x, fp32, zero_x));
      }
      if (timeit) {
        HIP_TRY(hipEventRecord(s->pev[3 * timed + 2], s->stream));
        ++timed;
      }
    }
    const bool last = k > guard;
    const int slot = batch & 1;
    HIP_TRY(hipMemcpyAsync(&s->host_sc[slot], d.sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipEventRecord(s->ev[slot], s->stream));
    if (have_prev || last) {
      const int ws = last ? slot : (slot ^ 1);
      HIP_TRY(hipEventSynchronize(s->ev[ws]));
      const Scalars& h = s->host_sc[ws];
      if (h.err) {
        job.err = 1;
        return MAZE_OK;
      }
      if (h.done || last) {
        job.iters = h.iters;
        job.code = h.done ? h.done : 3;
        if (prof) prof_collect(s, timed, ss ? (h.iters + 1) / 2 - 1 : h.iters, h.iters, fp32, ss);
        if (s->trace) return trace_collect(s, h.iters, h.qnorm);
        return MAZE_OK;
      }
    }
    have_prev = true;
    ++batch;
  }
}

// ---- batch tables: device arrays describing the sessions of a batched
// launch, with a pinned host mirror; one per device, grown on demand ----------
static_assert(sizeof(SweepArgs<float>) == sizeof(SweepArgs<double>),
              "batched sweep arguments share one layout");

struct BatchTable {
  int cap = 0;
  char* dev = nullptr;
  char* host = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // o_geom2 / o_wgb2: the update kernels' shapes of a two-iteration batch
  size_t o_args = 0, o_geom = 0, o_wgb = 0, o_scs = 0, o_poll = 0, o_sco = 0, bytes = 0;
  size_t o_geom2 = 0, o_wgb2 = 0;
};
static BatchTable g_tables[64];

static constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Offsets of a batch table for cap sessions (and its total size).
static constexpr BatchTable table_layout(int cap) {
  BatchTable n;
  n.cap = cap;
  size_t o = 0;
  n.o_args = o; o = align256(o + sizeof(SweepArgs<double>) * cap);
  n.o_geom = o; o = align256(o + sizeof(SweepGeom) * cap);
  n.o_wgb = o;  o = align256(o + sizeof(int) * (2 * cap + 16));
  n.o_geom2 = o; o = align256(o + sizeof(SweepGeom) * cap);
  n.o_wgb2 = o; o = align256(o + sizeof(int) * (2 * cap + 16));
  n.o_scs = o;  o = align256(o + sizeof(Scalars*) * cap);
  n.o_poll = o; o = align256(o + sizeof(int32_t) * 6 * cap);
  n.o_sco = o;  o = align256(o + sizeof(Scalars) * cap);
  n.bytes = o;
  return n;
}

// ---- fixed batch table of maze_step_batch_noalloc -----------------------------
// The non-allocating batch entry point keeps its batch table (session
// descriptors, launch geometries, workgroup prefixes, the poll and scalar
// staging arrays) in `scratch`, one copy per GPU for the life of the process,
// sized for kNoAllocMaxSessions sessions; its host mirror is a static array
// per device. In host code `scratch` names a host-side stand-in, not a device
// address: g_scratch_dev[device] holds the address hipGetSymbolAddress gives
// for that device, and only that address is passed to kernels and copies.
// Every table entry is written before a kernel or a copy reads it, so the
// array needs no clearing between calls.
constexpr int kNoAllocMaxSessions = 256;
constexpr int kNoAllocMaxDevices = 64;
constexpr size_t kNoAllocBytes = table_layout(kNoAllocMaxSessions).bytes;
static __device__ __align__(256) char scratch[kNoAllocBytes];
static char* g_scratch_dev[kNoAllocMaxDevices];
static bool g_scratch_looked_up[kNoAllocMaxDevices];
static std::mutex g_scratch_mu;
alignas(256) static char g_noalloc_host[kNoAllocMaxDevices][kNoAllocBytes];

// Looks up this device's address of `scratch`, once per device, with that
// device current (maze_init calls it for every session's device).
static void scratch_setup(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_looked_up[device]) return;
  g_scratch_looked_up[device] = true;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    ptr = nullptr;
  }
  g_scratch_dev[device] = static_cast<char*>(ptr);
}

// While set, every batch table request of this thread is served by the fixed
// table (a request for more sessions than it holds fails with
// MAZE_E_CAPACITY) instead of the grow-on-demand table of the device.
static thread_local BatchTable* tl_fixed_table = nullptr;

static int ensure_table(int device, int count, BatchTable** out) {
  if (tl_fixed_table) {
    if (count > tl_fixed_table->cap) return MAZE_E_CAPACITY;
    *out = tl_fixed_table;
    return MAZE_OK;
  }
  if (device < 0 || device >= 64) return MAZE_E_DEVICE;
  BatchTable& t = g_tables[device];
  if (t.cap < count) {
    int cap = std::max(64, t.cap);
    while (cap < count) cap *= 2;
    BatchTable n = table_layout(cap);
    if (hipMalloc((void**)&n.dev, n.bytes) != hipSuccess) {
      hipGetLastError();
      return MAZE_E_OOM;
    }
    if (hipHostMalloc((void**)&n.host, n.bytes, hipHostMallocDefault) != hipSuccess) {
      hipFree(n.dev);
      return MAZE_E_OOM;
    }
    if (hipEventCreateWithFlags(&n.ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&n.ev[1], hipEventDisableTiming) != hipSuccess)
      return MAZE_E_DEVICE;
    if (t.dev) {
      hipDeviceSynchronize();
      hipFree(t.dev);
      hipHostFree(t.host);
      hipEventDestroy(t.ev[0]);
      hipEventDestroy(t.ev[1]);
    }
    t = n;
  }
  *out = &t;
  return MAZE_OK;
}

// Scalars of several sessions (one device copy and one transfer).
static int gather_scalars(std::vector<maze_session*>& ss, std::vector<Scalars>& out) {
  const int n = (int)ss.size();
  out.resize(n);
  if (n == 1) {
    maze_session* s = ss[0];
    HIP_TRY(hipMemcpyAsync(&s->host_sc[0], s->d.sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    out[0] = s->host_sc[0];
    return MAZE_OK;
  }
  BatchTable* t = nullptr;
  int rc = ensure_table(ss[0]->device, n, &t);
  if (rc != MAZE_OK) return rc;
  hipStream_t st = ss[0]->stream;
  Scalars** hs = (Scalars**)(t->host + t->o_scs);
  for (int i = 0; i < n; ++i) hs[i] = ss[i]->d.sc;
  HIP_TRY(hipMemcpyAsync(t->dev + t->o_scs, hs, sizeof(Scalars*) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_batch_scalars((Scalars* const*)(t->dev + t->o_scs), n,
                               (Scalars*)(t->dev + t->o_sco), st));
  HIP_TRY(hipMemcpyAsync(t->host + t->o_sco, t->dev + t->o_sco, sizeof(Scalars) * n,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::memcpy(out.data(), t->host + t->o_sco, sizeof(Scalars) * n);
  return MAZE_OK;
}

// A batch whose sessions need at least kThroughputWgs workgroups in their
// throughput shapes (one per CU) is swept in those shapes; a smaller one in
// each session's latency shape, so that a session swept in it sums its
// partials in the same order as when stepped alone. Measured on molten-NaCl
// batches of 2 to 64 sessions (32^3 to 192^3 grids): below one workgroup
// per CU the latency shapes are up to 2.6x faster per step, above it the
// throughput shapes up to 1.8x. MAZE_BATCH_MODE=latency or =throughput in
// the environment forces one mode.
constexpr long long kThroughputWgs = 256;

static bool batch_throughput_mode(const std::vector<CgJob>& jobs) {
  const char* e = std::getenv("MAZE_BATCH_MODE");
  if (e && std::strcmp(e, "latency") == 0) return false;
  if (e && std::strcmp(e, "throughput") == 0) return true;
  long long w = 0;
  for (const CgJob& j : jobs) w += j.s->sweep_tp.nwg;
  return w >= kThroughputWgs;
}

// ---- graph-captured poll groups of batched solves ----------------------------
// A poll group of a batched solve (its units after the first one) depends on
// the sessions only through the batch table, which the kernels read at run
// time: the launch structure (the kernel classes with their table ranges,
// workgroup counts and LDS), the table's device address, the parity of the
// group's first unit and the number of units fix every launch. So a group
// captured once into a HIP graph is replayed for every later group with the
// same key, in this solve and in later calls, whatever sessions fill the
// table. Graphs are kept per device, at most kBatchGraphMax (then all are
// dropped and recaptured as needed).
constexpr size_t kBatchGraphMax = 64;
static std::map<std::vector<long long>, hipGraphExec_t> g_batch_graphs[64];
static std::mutex g_batch_graph_mu;

// Replays (capturing on first use) nb units from k0 through launch(k).
template <class F>
static hipError_t batch_graph_group(int device, std::vector<long long> key, long long k0, int nb,
                                    hipStream_t st, F& launch) {
  if (device < 0 || device >= 64) return hipErrorInvalidValue;
  key.push_back(k0 & 1);
  key.push_back(nb);
  std::lock_guard<std::mutex> lk(g_batch_graph_mu);
  auto& cache = g_batch_graphs[device];
  auto it = cache.find(key);
  hipGraphExec_t exec = nullptr;
  if (it != cache.end()) {
    exec = it->second;
  } else {
    if (cache.size() >= kBatchGraphMax) {
      for (auto& kv : cache) (void)hipGraphExecDestroy(kv.second);
      cache.clear();
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int b = 0; b < nb && e == hipSuccess; ++b) e = launch(k0 + b);
    const hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess && g) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
    cache[key] = exec;
  }
  return hipGraphLaunch(exec, st);
}

// The polling loop of a batched solve: queues `per` units (first call:
// at least first_units) through launch(k), then copies every session's
// status to pinned memory and waits for the copy of the group before, so
// the device always has a group queued; returns once every session is done
// (or the guard is reached), with iterations and codes in the jobs. With a
// graph key (non-empty), the groups after the first (which holds the first
// unit of every solve) are replayed from captured graphs.
template <class F>
static int batch_loop(std::vector<CgJob>& jobs, const std::vector<int>& order, BatchTable* t,
                      hipStream_t st, long long guard, int per, int first_units, F launch,
                      const std::vector<long long>& graph_key = {}) {
  const int n = (int)jobs.size();
  char* H = t->host;
  int32_t* poll_h = (int32_t*)(H + t->o_poll);
  int32_t* poll_d = (int32_t*)(t->dev + t->o_poll);
  long long k = 0;
  int batch = 0;
  bool have_prev = false;
  for (;;) {
    const int nb = (batch == 0) ? std::max(per, first_units) : per;
    if (batch > 0 && !graph_key.empty()) {
      HIP_TRY(batch_graph_group(jobs[0].s->device, graph_key, k, nb, st, launch));
      k += nb;
    } else {
      for (int b = 0; b < nb; ++b, ++k) HIP_TRY(launch(k));
    }
    const bool last = k > guard;
    const int slot = batch & 1;
    HIP_TRY(launch_batch_poll((Scalars* const*)(t->dev + t->o_scs), n, poll_d + 3 * n * slot, st));
    HIP_TRY(hipMemcpyAsync(poll_h + 3 * n * slot, poll_d + 3 * n * slot, sizeof(int32_t) * 3 * n,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(t->ev[slot], st));
    if (have_prev || last) {
      const int ws = last ? slot : (slot ^ 1);
      HIP_TRY(hipEventSynchronize(t->ev[ws]));
      const int32_t* p = poll_h + 3 * n * ws;
      bool all = true;
      for (int q = 0; q < n; ++q) all &= (p[3 * q] != 0 || p[3 * q + 2] != 0);
      if (all || last) {
        for (int q = 0; q < n; ++q) {
          CgJob& j = jobs[order[q]];
          j.err = p[3 * q + 2] != 0;
          j.iters = p[3 * q + 1];
          j.code = p[3 * q] ? p[3 * q] : 3;
        }
        for (CgJob& j : jobs) {
          if (!j.err && j.s->trace) {
            std::vector<maze_session*> one{j.s};
            std::vector<Scalars> h;
            int rc = gather_scalars(one, h);
            if (rc != MAZE_OK) return rc;
            rc = trace_collect(j.s, j.iters, h[0].qnorm);
            if (rc != MAZE_OK) return rc;
          }
        }
        return MAZE_OK;
      }
    }
    have_prev = true;
    ++batch;
  }
}

static int run_sstep_batch(std::vector<CgJob>& jobs, bool fp32, bool zero_x, int first_batch);

// Batched solves replay their poll groups from captured graphs when every
// session asks for graph chunks (MAZE_FLAG_GRAPH_CHUNKS), the stream can be
// captured and no session samples its timing.
static bool batch_graphs(const std::vector<CgJob>& jobs, hipStream_t st) {
  if (st == nullptr) return false;
  for (const CgJob& j : jobs)
    if (!(j.s->cfg.flags & MAZE_FLAG_GRAPH_CHUNKS) || j.s->prof) return false;
  return true;
}

// Batched CG solves: one launch per sweep and template class covers every
// session; a compact status array is polled.
static int run_cg_batch(std::vector<CgJob>& jobs, bool fp32, bool zero_x, int first_batch) {
  const int n = (int)jobs.size();
  if (n == 1) return run_cg(jobs[0], fp32, zero_x, first_batch);
  // two-iteration sessions run in batches of their own
  {
    std::vector<CgJob> ss, one;
    for (const CgJob& j : jobs) (sstep_of(j.s) ? ss : one).push_back(j);
    if (!ss.empty()) {
      int rc = MAZE_OK;
      if (one.empty()) return run_sstep_batch(jobs, fp32, zero_x, first_batch);
      rc = run_cg_batch(one, fp32, zero_x, first_batch);
      if (rc != MAZE_OK) return rc;
      rc = run_cg_batch(ss, fp32, zero_x, first_batch);
      if (rc != MAZE_OK) return rc;
      size_t a = 0, b = 0;  // results back into the caller's order
      for (CgJob& j : jobs) j = sstep_of(j.s) ? ss[b++] : one[a++];
      return MAZE_OK;
    }
  }
  BatchTable* t = nullptr;
  int rc = ensure_table(jobs[0].s->device, n, &t);
  if (rc != MAZE_OK) return rc;
  hipStream_t st = jobs[0].s->stream;
  const bool tp = batch_throughput_mode(jobs);
  auto shape = [&](int i) -> const SweepGeom& { return tp ? jobs[i].s->sweep_tp : jobs[i].s->sweep; };
  // order the sessions by template class (ppt, nh)
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cls = [&](int i) {
    const SweepGeom& g = shape(i);
    return g.ppt * 16 + sweep_nh_class(g.nh);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cls(a) < cls(b); });
  struct Cls { int c0, c1, wgb0, nwg, ppt, nh; size_t lds; };
  std::vector<Cls> classes;
  char* H = t->host;
  SweepGeom* hg = (SweepGeom*)(H + t->o_geom);
  int* hw = (int*)(H + t->o_wgb);
  Scalars** hs = (Scalars**)(H + t->o_scs);
  int wpos = 0;
  long long guard = 0;
  for (int q = 0; q < n; ++q) {
    const int i = order[q];
    maze_session* s = jobs[i].s;
    const SweepGeom& g = shape(i);
    if (g.nwg > s->d.part_stride) return MAZE_E_INVALID;
    if (classes.empty() || cls(order[classes.back().c0]) != cls(i)) {
      if (!classes.empty()) hw[wpos++] = classes.back().nwg;
      classes.push_back({q, q, wpos, 0, g.ppt, sweep_nh_class(g.nh), 0});
    }
    Cls& c = classes.back();
    hw[wpos++] = c.nwg;
    c.nwg += g.nwg;
    c.c1 = q + 1;
    c.lds = std::max(c.lds, sweep_lds_bytes(g, fp32, false));
    hg[q] = g;
    hs[q] = s->d.sc;
    if (fp32) {
      ((SweepArgs<float>*)(H + t->o_args))[q] =
          make_sweep_args<float>(s->d, (float*)jobs[i].x, s->geom.nwg, g.nwg, zero_x);
    } else {
      ((SweepArgs<double>*)(H + t->o_args))[q] =
          make_sweep_args<double>(s->d, (double*)jobs[i].x, s->geom.nwg, g.nwg, zero_x);
    }
    guard = std::max(guard, sweep_guard(jobs[i].max_iter, first_batch));
  }
  hw[wpos++] = classes.back().nwg;
  for (const Cls& c : classes)
    if (c.nh == 0 || c.lds > 160 * 1024 - 1024) return MAZE_E_INVALID;
  HIP_TRY(hipMemcpyAsync(t->dev, H, t->o_poll, hipMemcpyHostToDevice, st));
  std::vector<long long> gkey;
  if (batch_graphs(jobs, st)) {
    gkey = {0, (long long)(uintptr_t)t->dev, fp32 ? 1 : 0, n};
    for (const Cls& c : classes)
      gkey.insert(gkey.end(), {c.c0, c.c1, c.wgb0, c.nwg, c.ppt, c.nh, (long long)c.lds});
  }
  return batch_loop(jobs, order, t, st, guard, kPollBatch, first_batch, [&](long long k) {
    for (const Cls& c : classes) {
      SweepLaunch L{};
      L.batch = true;
      L.par = (int)(k & 1);
      L.ppt = c.ppt;
      L.nh = c.nh;
      L.args = t->dev + t->o_args + (size_t)c.c0 * sizeof(SweepArgs<double>);
      L.geoms = (const SweepGeom*)(t->dev + t->o_geom) + c.c0;
      L.wg_begin = (const int*)(t->dev + t->o_wgb) + c.wgb0;
      L.count = c.c1 - c.c0;
      L.nwg_total = c.nwg;
      L.lds = c.lds;
      const hipError_t e = launch_sweep(L, fp32, k == 0, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }, gkey);
}

// Batched two-iteration solves. The sessions are ordered by the template
// class of their basis kernel, then of their update kernel; each kernel
// runs one launch per run of equal class. In latency mode the shapes are
// the sessions' own (basis and latency shapes), so a session's result is
// bitwise the one it gets alone; in throughput mode both kernels take the
// throughput shape.
static int run_sstep_batch(std::vector<CgJob>& jobs, bool fp32, bool zero_x, int first_batch) {
  const int n = (int)jobs.size();
  BatchTable* t = nullptr;
  int rc = ensure_table(jobs[0].s->device, n, &t);
  if (rc != MAZE_OK) return rc;
  hipStream_t st = jobs[0].s->stream;
  const bool tp = batch_throughput_mode(jobs);
  auto gb = [&](int i) -> const SweepGeom& { return tp ? jobs[i].s->sweep_tp : jobs[i].s->sbasis; };
  auto gu = [&](int i) -> const SweepGeom& { return tp ? jobs[i].s->sweep_tp : jobs[i].s->sweep; };
  // The row-owning layout changes which points a thread's Gram sums cover,
  // so a latency-mode batch keeps each session's own layout (its results
  // are bitwise those it gets alone) and a throughput-mode batch, whose
  // partials are summed in another order anyway, runs every member in the
  // flat layout: fewer classes, fewer launches.
  auto rows = [tp](const SweepGeom& g) { return !tp && sstep_rows(g); };
  auto cls = [&rows](const SweepGeom& g) {
    return ((((sstep_threads(g)) * 8 + g.ppt) * 16 + sweep_nh_class(g.nh)) * 2 +
            (rows(g) ? 1 : 0)) * 32 + g.zv;
  };
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int ca = cls(gb(a)), cb = cls(gb(b));
    return ca != cb ? ca < cb : cls(gu(a)) < cls(gu(b));
  });
  struct Grp { int c0, c1, wgb0, nwg, nt, ppt, nh; bool rows; size_t lds; int zv; };
  std::vector<Grp> gbs, gus;
  char* H = t->host;
  SweepGeom* hg = (SweepGeom*)(H + t->o_geom);
  SweepGeom* hg2 = (SweepGeom*)(H + t->o_geom2);
  int* hw = (int*)(H + t->o_wgb);
  int* hw2 = (int*)(H + t->o_wgb2);
  Scalars** hs = (Scalars**)(H + t->o_scs);
  int wpos = 0, wpos2 = 0;
  long long guard = 0;
  for (int q = 0; q < n; ++q) {
    const int i = order[q];
    maze_session* s = jobs[i].s;
    const SweepGeom& b = gb(i);
    const SweepGeom& u = gu(i);
    if (b.nwg > s->d.part_stride || u.nwg > s->d.part_stride) return MAZE_E_INVALID;
    if (!sstep_basis_shape_ok(b, fp32) || !sstep_update_shape_ok(u, fp32)) return MAZE_E_INVALID;
    const int cb = cls(b), cu = cls(u);
    if (gbs.empty() || cls(hg[gbs.back().c0]) != cb) {
      if (!gbs.empty()) hw[wpos++] = gbs.back().nwg;
      gbs.push_back({q, q, wpos, 0, sstep_threads(b), b.ppt, sweep_nh_class(b.nh), rows(b), 0,
                     b.zv});
    }
    if (gus.empty() || cls(hg2[gus.back().c0]) != cu) {
      if (!gus.empty()) hw2[wpos2++] = gus.back().nwg;
      gus.push_back({q, q, wpos2, 0, sstep_threads(u), u.ppt, sweep_nh_class(u.nh), rows(u), 0,
                     u.zv});
    }
    hg[q] = b;
    hg2[q] = u;
    Grp& B = gbs.back();
    hw[wpos++] = B.nwg;
    B.nwg += b.nwg;
    B.c1 = q + 1;
    B.lds = std::max(B.lds, sstep_lds_bytes(b, fp32));
    Grp& U = gus.back();
    hw2[wpos2++] = U.nwg;
    U.nwg += u.nwg;
    U.c1 = q + 1;
    U.lds = std::max(U.lds, sstep_lds_bytes(u, fp32));
    hs[q] = s->d.sc;
    // the update kernel reads one partial per basis workgroup
    if (fp32) {
      ((SweepArgs<float>*)(H + t->o_args))[q] =
          make_sweep_args<float>(s->d, (float*)jobs[i].x, 0, b.nwg, zero_x);
    } else {
      ((SweepArgs<double>*)(H + t->o_args))[q] =
          make_sweep_args<double>(s->d, (double*)jobs[i].x, 0, b.nwg, zero_x);
    }
    guard = std::max(guard, sweep_guard(jobs[i].max_iter, first_batch));
  }
  // at most one start per session and one total per run: 2n + 1 entries
  hw[wpos++] = gbs.back().nwg;
  hw2[wpos2++] = gus.back().nwg;
  for (const std::vector<Grp>* gs : {&gbs, &gus})
    for (const Grp& g : *gs)
      if (g.nh == 0 || g.lds > 160 * 1024 - 2048) return MAZE_E_INVALID;
  HIP_TRY(hipMemcpyAsync(t->dev, H, t->o_poll, hipMemcpyHostToDevice, st));
  std::vector<long long> gkey;
  if (batch_graphs(jobs, st)) {
    gkey = {1, (long long)(uintptr_t)t->dev, fp32 ? 1 : 0, n};
    for (const std::vector<Grp>* gs : {&gbs, &gus})
      for (const Grp& g : *gs)
        gkey.insert(gkey.end(),
                    {g.c0, g.c1, g.wgb0, g.nwg, g.nt, g.ppt, g.nh, g.rows ? 1 : 0,
                     (long long)g.lds, g.zv});
  }
  return batch_loop(jobs, order, t, st, guard, kPollBatch / 2, first_batch / 2, [&](long long k) {
    for (int half = 0; half < 2; ++half) {
      const bool update = half == 1;
      for (const Grp& g : update ? gus : gbs) {
        SweepLaunch L{};
        L.batch = true;
        L.par = (int)(k & 1);
        L.ppt = g.ppt;
        L.nh = g.nh;
        L.zv = g.zv;
        L.args = t->dev + t->o_args + (size_t)g.c0 * sizeof(SweepArgs<double>);
        L.geoms = (const SweepGeom*)(t->dev + (update ? t->o_geom2 : t->o_geom)) + g.c0;
        L.wg_begin = (const int*)(t->dev + (update ? t->o_wgb2 : t->o_wgb)) + g.wgb0;
        L.count = g.c1 - g.c0;
        L.nwg_total = g.nwg;
        L.lds = g.lds;
        const hipError_t e = launch_sstep_batch(L, g.nt, g.rows, fp32, k == 0, update, st);
        if (e != hipSuccess) return e;
      }
    }
    return hipSuccess;
  }, gkey);
}

// Multigrid-preconditioned CG of one session on x (FP64): per iteration a
// V-cycle z = B r, rho = <r, z>, the direction pass p = z + beta p with
// <p, A p>, the update pass x += alpha p, r -= alpha A p with ||r||; the
// device applies the stopping test. Iteration i is queued before the status
// of iteration i - 1 is waited for.
static int run_mgcg(maze_session* s, double* x, CgJob& job) {
  DeviceState& d = s->d;
  const MarchGeom& g = s->geom;
  const MgHierarchy& m = d.mg;
  hipStream_t st = s->stream;
  HIP_TRY(launch_finalize(d, FIN_MG_CHECK0, g.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0, st));
  const long long guard = (long long)s->cfg.max_iter + 8;
  for (long long i = 0;; ++i) {
    HIP_TRY(launch_mg_vcycle(d, m, d.r, m.z, m.fp32, st));
    HIP_TRY(launch_mg_dot(d, d.r, m.z, m.fp32, st));
    HIP_TRY(launch_finalize(d, FIN_MG_RHO, mg_dot_blocks(d.G), 0.0, 0.0, 0.0, nullptr, 0, 0, st));
    double* pnew = d.p + (size_t)(i & 1) * d.G;
    const double* pold = d.p + (size_t)((i & 1) ^ 1) * d.G;
    HIP_TRY(launch_mg_dir(d, g, m.z, m.fp32, pold, pnew, st));
    HIP_TRY(launch_finalize(d, FIN_MG_MU, g.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0, st));
    HIP_TRY(launch_mg_upd(d, g, pnew, x, st));
    HIP_TRY(launch_finalize(d, FIN_MG_CONV, g.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0, st));
    const int slot = (int)(i & 1);
    HIP_TRY(hipMemcpyAsync(&s->host_sc[slot], d.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(s->ev[slot], st));
    const bool last = i > guard;
    if (i > 0 || last) {
      const int ws = last ? slot : (slot ^ 1);
      HIP_TRY(hipEventSynchronize(s->ev[ws]));
      const Scalars& h = s->host_sc[ws];
      if (h.err) {
        job.err = 1;
        return MAZE_OK;
      }
      if (h.done || last) {
        job.iters = h.iters;
        job.code = h.done ? h.done : 3;
        if (s->trace) return trace_collect(s, h.iters, h.qnorm);
        return MAZE_OK;
      }
    }
  }
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

// Solves M x = s for every session (s in d.sigma, the first residual and its
// partials written by a right-hand-side kernel, thresholds set by
// FIN_SOLVE_START). Sessions of one precision are solved together. Leaves
// the true residual and the mean of x in each session's scalars
// (FIN_SOLVE_END). rcs[i]: MAZE_OK or MAZE_E_NONFINITE for session i.
static int solve_multi(std::vector<maze_session*>& ss, std::vector<double*>& xs,
                       std::vector<int>& rcs) {
  const int n = (int)ss.size();
  rcs.assign(n, MAZE_OK);
  for (maze_session* s : ss) {
    s->iters = 0;
    s->refinements = 0;
    s->converged = 0;
    s->trace_rows.clear();
    s->trace_pass = 0;
  }
  // multigrid-preconditioned sessions: one solve each
  std::vector<bool> is_mg(n, false);
  for (int i = 0; i < n; ++i) {
    if (ss[i]->d.mg.levels == 0) continue;
    is_mg[i] = true;
    maze_session* s = ss[i];
    CgJob j;
    j.s = s;
    j.x = xs[i];
    j.max_iter = s->cfg.max_iter;
    const int rc = run_mgcg(s, xs[i], j);
    if (rc != MAZE_OK) return rc;
    if (j.err) {
      rcs[i] = MAZE_E_NONFINITE;
      continue;
    }
    s->iters = j.iters;
    s->converged = (j.code == 1);
    HIP_TRY(launch_true_residual(s->d, s->geom, xs[i], s->stream));
    HIP_TRY(launch_finalize(s->d, FIN_SOLVE_END, s->geom.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0,
                            s->stream));
  }
  // FP64 sessions: one CG solve each, batched
  {
    std::vector<CgJob> jobs;
    std::vector<int> idx;
    int fb = 1 << 30;
    for (int i = 0; i < n; ++i)
      if (ss[i]->cfg.precision != MAZE_MIXED && !is_mg[i]) {
        CgJob j;
        j.s = ss[i];
        j.x = xs[i];
        j.max_iter = ss[i]->cfg.max_iter;
        jobs.push_back(j);
        idx.push_back(i);
        fb = std::min(fb, first_batch_of(ss[i]->last_iters));
      }
    if (!jobs.empty()) {
      const int rc = run_cg_batch(jobs, false, false, fb);
      if (rc != MAZE_OK) return rc;
      for (size_t q = 0; q < jobs.size(); ++q) {
        maze_session* s = jobs[q].s;
        if (jobs[q].err) {
          rcs[idx[q]] = MAZE_E_NONFINITE;
          continue;
        }
        s->iters = jobs[q].iters;
        s->converged = (jobs[q].code == 1);
        HIP_TRY(launch_true_residual(s->d, s->geom, xs[idx[q]], s->stream));
        HIP_TRY(launch_finalize(s->d, FIN_SOLVE_END, s->geom.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0,
                                s->stream));
      }
    }
  }
  // Mixed sessions: FP32 inner CG on the correction, FP64 outer residual.
  std::vector<int> act;
  for (int i = 0; i < n; ++i)
    if (ss[i]->cfg.precision == MAZE_MIXED && !is_mg[i]) act.push_back(i);
  if (act.empty()) return MAZE_OK;
  std::vector<Scalars> h;
  std::vector<double> thr(n, 0.0);
  std::vector<int> total(n, 0);
  std::vector<Scalars> hs(n);
  int rc = MAZE_OK;
  // After an inner solve of session i (job j): the FP64 correction and
  // residual; returns whether another pass may follow.
  auto after_pass = [&](int i, const CgJob& j, bool* more) -> int {
    maze_session* s = ss[i];
    *more = false;
    if (j.err) {
      rcs[i] = MAZE_E_NONFINITE;
      return MAZE_OK;
    }
    const int it = j.iters;
    s->last_inner[s->refinements] = it;
    total[i] += it;
    s->refinements += 1;
    HIP_TRY(launch_add_correction(s->d, xs[i], s->stream));
    HIP_TRY(launch_refine(s->d, s->geom, xs[i], true, s->stream));
    HIP_TRY(launch_finalize(s->d, FIN_SOLVE_END, s->geom.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0,
                            s->stream));
    *more = !(j.code == 2 && it == 0);  // breakdown without progress
    return MAZE_OK;
  };
  // The first pass is decided on the device (FIN_INNER_FIRST, the same
  // test and tolerance as below), so no host round trip precedes it, unless
  // a session records a residual trace or allows no iteration.
  bool dev_first = true;
  for (int i : act)
    if (ss[i]->trace || ss[i]->cfg.max_iter <= 0) dev_first = false;
  if (dev_first) {
    std::vector<CgJob> jobs;
    int fb = 1 << 30;
    for (int i : act) {
      maze_session* s = ss[i];
      s->trace_pass = 0;
      HIP_TRY(launch_finalize(s->d, FIN_INNER_FIRST, 0, kInnerReduction, kInnerMargin, 0.0,
                              nullptr, s->cfg.max_iter, s->cfg.residual_norm, s->stream));
      CgJob j;
      j.s = s;
      j.x = s->d.e32;
      j.max_iter = s->cfg.max_iter;
      jobs.push_back(j);
      fb = std::min(fb, first_batch_of(s->last_inner[0]));
    }
    rc = run_cg_batch(jobs, true, true, fb);
    if (rc != MAZE_OK) return rc;
    std::vector<int> keep;
    std::vector<maze_session*> ks;
    for (size_t q = 0; q < act.size(); ++q) {
      const int i = act[q];
      if (!jobs[q].err && jobs[q].code == 4) {  // the right-hand side's residual met thr
        ss[i]->converged = 1;
        continue;
      }
      bool more = false;
      rc = after_pass(i, jobs[q], &more);
      if (rc != MAZE_OK) return rc;
      if (more) {
        keep.push_back(i);
        ks.push_back(ss[i]);
      }
    }
    if (!ks.empty()) {
      rc = gather_scalars(ks, h);
      if (rc != MAZE_OK) return rc;
    }
    for (size_t q = 0; q < keep.size(); ++q) {
      hs[keep[q]] = h[q];
      thr[keep[q]] = h[q].thr_outer;
    }
    act = keep;
  } else {
    std::vector<maze_session*> as;
    for (int i : act) as.push_back(ss[i]);
    rc = gather_scalars(as, h);
    if (rc != MAZE_OK) return rc;
    for (size_t q = 0; q < act.size(); ++q) {
      hs[act[q]] = h[q];
      thr[act[q]] = h[q].thr;
    }
  }
  while (!act.empty()) {
    std::vector<int> next;
    for (int i : act) {
      maze_session* s = ss[i];
      const Scalars& hh = hs[i];
      if (hh.err) {
        rcs[i] = MAZE_E_NONFINITE;
        continue;
      }
      const bool absmax = s->cfg.residual_norm == MAZE_NORM_ABSMAX;
      const double res = absmax ? hh.true_max : std::sqrt(hh.true_rr);
      if (s->trace) {
        s->trace_rows.push_back(s->refinements);
        s->trace_rows.push_back(-1);
        s->trace_rows.push_back(std::sqrt(hh.true_rr) / (hh.qnorm > 0 ? hh.qnorm : 1.0));
      }
      s->trace_pass = s->refinements;
      if (res <= thr[i]) {
        s->converged = 1;
        continue;
      }
      if (s->refinements >= kMaxRefinements || total[i] >= s->cfg.max_iter) continue;
      const double inner = std::max(kInnerReduction * res, kInnerMargin * thr[i]);
      HIP_TRY(launch_finalize(s->d, FIN_INNER_START, 0, 0.0, inner, 0.0, nullptr,
                              s->cfg.max_iter - total[i], s->cfg.residual_norm, s->stream));
      next.push_back(i);
    }
    if (next.empty()) break;
    std::vector<CgJob> jobs;
    int fb = 1 << 30;
    for (int i : next) {
      maze_session* s = ss[i];
      CgJob j;
      j.s = s;
      j.x = s->d.e32;
      j.max_iter = s->cfg.max_iter - total[i];
      jobs.push_back(j);
      fb = std::min(fb, first_batch_of(s->last_inner[s->refinements]));
    }
    rc = run_cg_batch(jobs, true, true, fb);
    if (rc != MAZE_OK) return rc;
    std::vector<int> keep;
    std::vector<maze_session*> ks;
    for (size_t q = 0; q < next.size(); ++q) {
      bool more = false;
      rc = after_pass(next[q], jobs[q], &more);
      if (rc != MAZE_OK) return rc;
      if (more) {
        keep.push_back(next[q]);
        ks.push_back(ss[next[q]]);
      }
    }
    if (keep.empty()) break;
    rc = gather_scalars(ks, h);
    if (rc != MAZE_OK) return rc;
    for (size_t q = 0; q < keep.size(); ++q) hs[keep[q]] = h[q];
    act = keep;
  }
  for (int i = 0; i < n; ++i)
    if (ss[i]->cfg.precision == MAZE_MIXED && !is_mg[i]) ss[i]->iters = total[i];
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
    std::vector<maze_session*> one{s};
    std::vector<Scalars> h;
    const int rc = gather_scalars(one, h);
    if (rc != MAZE_OK) return rc;
    fill_stats(s, h[0], st);
    st->status = s->converged ? MAZE_OK : MAZE_NOT_CONVERGED;
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
  HIP_TRY(launch_rhs_poisson(d, s->geom, guess, x, mixed && d.mg.levels == 0, s->stream));
  HIP_TRY(launch_finalize(d, FIN_SOLVE_START, s->geom.nwg, s->cfg.tol, 0.0, 0.0, nullptr,
                          s->cfg.max_iter, s->cfg.residual_norm, s->stream));
  std::vector<maze_session*> one{s};
  std::vector<double*> xs{x};
  std::vector<int> rcs;
  rc = solve_multi(one, xs, rcs);
  if (rc != MAZE_OK) return rc;
  if (rcs[0] == MAZE_E_NONFINITE) return recover_error(s);
  HIP_TRY(launch_project(d, x, field, s->stream));
  HIP_TRY(launch_finalize(d, FIN_ENERGY, update_blocks(d.G), 0.0, 0.0, s->cfg.coulomb_k,
                          energy, 0, 0, s->stream));
  if (forces) HIP_TRY(launch_gather(d, x, s->cfg.coulomb_k, forces, s->stream));
  return MAZE_OK;
}

// One MaZe step of every session (all on one stream). Per-session status in
// rcs (MAZE_OK, or an error that left the session unchanged).
static int step_multi(std::vector<maze_session*>& ss, const double* const* pos,
                      double* const* field, double* const* forces, double* const* energies,
                      std::vector<int>& rcs) {
  const int n = (int)ss.size();
  std::vector<double*> ys(n);
  for (int i = 0; i < n; ++i) {
    maze_session* s = ss[i];
    DeviceState& d = s->d;
    const int rc = assign(s, pos[i]);
    if (rc != MAZE_OK) return rc;
    HIP_TRY(launch_rhs_maze(d, s->geom, s->cfg.precision == MAZE_MIXED && d.mg.levels == 0,
                            s->stream));
    HIP_TRY(launch_finalize(d, FIN_SOLVE_START, s->geom.nwg, s->cfg.tol, 0.0, 0.0, nullptr,
                            s->cfg.max_iter, s->cfg.residual_norm, s->stream));
    ys[i] = d.y;
  }
  int rc = solve_multi(ss, ys, rcs);
  if (rc != MAZE_OK) return rc;
  for (int i = 0; i < n; ++i) {
    maze_session* s = ss[i];
    DeviceState& d = s->d;
    if (rcs[i] == MAZE_E_NONFINITE) {
      rcs[i] = recover_error(s);
      continue;
    }
    s->last_iters = s->iters;
    HIP_TRY(launch_update(d, field ? field[i] : nullptr, s->stream));
    HIP_TRY(launch_finalize(d, FIN_ENERGY, update_blocks(d.G), 0.0, 0.0, s->cfg.coulomb_k,
                            energies ? energies[i] : nullptr, 0, 0, s->stream));
    if (forces && forces[i])
      HIP_TRY(launch_gather(d, d.phi_prev, s->cfg.coulomb_k, forces[i], s->stream));
    std::swap(d.phi_cur, d.phi_prev);
    s->step += 1;
  }
  return MAZE_OK;
}

// ---- launch-shape autotuner -------------------------------------------------
// At session creation, before the buffers are cleared for the first solve,
// each candidate shape runs the first sweep, 3 warm-up sweeps and 8 timed
// sweeps on a fixed pattern (thresholds set so that nothing converges); the
// fastest shape is kept for the session and cached per (device, N,
// precision), so later sessions of that size reuse it without timing and
// sessions of equal size share one shape (and one summation order).
// MAZE_AUTOTUNE=0 in the environment selects the fixed default shapes.
struct TuneKey {
  int device, N, fp32;
  bool operator<(const TuneKey& o) const {
    return device != o.device ? device < o.device : (N != o.N ? N < o.N : fp32 < o.fp32);
  }
};
static std::map<TuneKey, SweepGeom> g_tuned;
static std::mutex g_tune_mu;

static bool autotune_enabled() {
  const char* e = std::getenv("MAZE_AUTOTUNE");
  return !(e && e[0] == '0');
}

// MAZE_SWEEP_SHAPE="ppt:cx" forces one launch shape (points per thread 1, 2
// or 4; x planes per workgroup) for every session that admits it: its halo
// width and LDS must fit a kernel instantiation and its workgroups the rows
// of the session's partials buffer.
static bool forced_shape(const DeviceState& d, bool fp32, SweepGeom* out) {
  const char* e = std::getenv("MAZE_SWEEP_SHAPE");
  int ppt = 0, cx = 0;
  if (!e || std::sscanf(e, "%d:%d", &ppt, &cx) != 2) return false;
  if ((ppt != 1 && ppt != 2 && ppt != 4) || cx < 1) return false;
  const SweepGeom g = make_sweep_geom(d.N, ppt, cx);
  if (sweep_nh_class(g.nh) == 0 || sweep_lds_bytes(g, fp32, false) > 159 * 1024) return false;
  if (g.nwg > d.part_stride) return false;
  *out = g;
  return true;
}

// Throughput shape: the admissible shape with the least re-read traffic per
// point among runs of 16 x planes and 1024-point segments (then shorter
// segments and runs). Within a batch that fills the GPU many times over,
// workgroups are not the limit and the halo re-reads of short runs are.
static SweepGeom throughput_sweep(const DeviceState& d, bool fp32) {
  const int N = d.N;
  SweepGeom g;
  if (forced_shape(d, fp32, &g)) return g;
  const std::vector<SweepGeom> cand = sweep_candidates(N, fp32, 0);
  for (int ppt : {4, 2, 1})
    for (int cx : {16, 8, 4})
      for (const SweepGeom& c : cand)
        if (c.ppt == ppt && c.nchunk == (N + cx - 1) / cx) return c;
  return choose_sweep(N);
}

static SweepGeom autotune_sweep(maze_session* s) {
  DeviceState& d = s->d;
  const bool fp32 = s->cfg.precision == MAZE_MIXED;
  SweepGeom def = choose_sweep(d.N);
  if (forced_shape(d, fp32, &def)) return def;
  if (d.mg.levels > 0 || !autotune_enabled()) return def;
  const TuneKey key{s->device, d.N, fp32 ? 1 : 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  std::vector<SweepGeom> cand;
  for (const SweepGeom& g : sweep_candidates(d.N, fp32, device_cus()))
    if (g.nwg <= d.part_stride) cand.push_back(g);
  if (cand.size() <= 1) return def;
  hipStream_t st = s->stream;
  void* x = fp32 ? (void*)d.e32 : (void*)d.xsolve;
  void* r0 = fp32 ? (void*)d.r32 : (void*)d.r;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return def;
  Scalars sc{};
  sc.thr = -1.0;  // never converged
  sc.max_iter = 1 << 30;
  sc.norm = MAZE_NORM_REL2;
  SweepGeom best = def;
  float best_ms = 1e30f;
  bool ok = true;
  for (const SweepGeom& g : cand) {
    ok = ok && hipMemcpyAsync(d.sc, &sc, sizeof(Scalars), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && launch_fill_pattern(r0, d.G, fp32, st) == hipSuccess;
    for (int k = 0; k < 4 && ok; ++k)
      ok = launch_cg_sweep(d, g, k, s->geom.nwg, x, fp32, true, st) == hipSuccess;
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    for (int k = 4; k < 12 && ok; ++k)
      ok = launch_cg_sweep(d, g, k, s->geom.nwg, x, fp32, true, st) == hipSuccess;
    ok = ok && hipEventRecord(e1, st) == hipSuccess;
    Scalars h{};
    ok = ok && hipMemcpyAsync(&h, d.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) break;
    float ms = 0.f;
    if (h.done == 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = g;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!ok) {
    hipGetLastError();
    return def;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

// Shape of the basis kernel of the two-iteration CG. It only reads r and p
// and is bound by its per-plane steps rather than by HBM, so it prefers
// larger workgroups (512 or 1024 threads, segments of 1024 to 4096 points:
// less halo work per point). Candidates are the session's latency shape
// and the spill-free 512- and 1024-thread shapes; each runs 2 warm-up and
// 6 timed outer steps (basis and update kernel) on a fill pattern of the
// session's r and p. MAZE_BASIS_SHAPE="threads:ppt:cx" forces one.

// "zv:wavefronts:cx": a wavefront-row shape
static bool forced_zv(const char* e, const DeviceState& d, SweepGeom* out) {
  int wv = 0, cx = 0;
  if (!e || std::sscanf(e, "zv:%d:%d", &wv, &cx) != 2 || wv < 3 || cx < 1 || d.N % 64 != 0)
    return false;
  *out = make_sstep_zv_geom(d.N, cx, wv);
  return true;
}

// Wavefront-row basis candidates of a grid (N = 64, 128 or 256): with
// workgroups of 8 wavefronts, a list of x runs and the shortest runs whose
// grid fits the device's CUs in one round at one and at two workgroups per
// CU (FP64 kernels hold one per CU, FP32 kernels two; at 256^3 x runs of 52
// and 24 planes); with workgroups of 16 (FP32, 256^3), the shortest
// one-round run at one per CU (20 planes).
static void zv_candidates(const DeviceState& d, bool fp32, int device,
                          std::vector<SweepGeom>* cand) {
  const char* e = std::getenv("MAZE_ZV");
  if (d.N % 64 != 0 || (e && std::strcmp(e, "0") == 0)) return;
  std::vector<int> cxs{6, 8, 10, 12, 16, 20, 24, 32, 48, 64};
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    (void)hipGetLastError();
    cus = 0;
  }
  const int nseg = make_sstep_zv_geom(d.N, 1, 8).nseg;
  for (int k : {1, 2}) {
    const int nch = (k * cus) / nseg;
    if (nch >= 1) cxs.push_back((d.N + nch - 1) / nch);
  }
  std::sort(cxs.begin(), cxs.end());
  int last = -1;
  for (int cx : cxs) {
    const SweepGeom g = make_sstep_zv_geom(d.N, cx, 8);
    if (g.nchunk == last || !sstep_basis_shape_ok(g, fp32) || g.nwg > d.part_stride) continue;
    last = g.nchunk;
    cand->push_back(g);
  }
  const int nseg16 = make_sstep_zv_geom(d.N, 1, 16).nseg;
  if (cus >= nseg16) {
    const int nch = cus / nseg16;
    const SweepGeom g = make_sstep_zv_geom(d.N, (d.N + nch - 1) / nch, 16);
    if (sstep_basis_shape_ok(g, fp32) && g.nwg <= d.part_stride) cand->push_back(g);
  }
}

static bool forced_basis(const DeviceState& d, bool fp32, SweepGeom* out) {
  const char* e = std::getenv("MAZE_BASIS_SHAPE");
  SweepGeom z;
  if (forced_zv(e, d, &z)) {
    if (!sstep_basis_shape_ok(z, fp32) || z.nwg > d.part_stride) return false;
    *out = z;
    return true;
  }
  int nt = 0, ppt = 0, cx = 0;
  if (!e || std::sscanf(e, "%d:%d:%d", &nt, &ppt, &cx) != 3) return false;
  if ((nt != kThreads && nt != 512 && nt != 1024) || (ppt != 1 && ppt != 2 && ppt != 4) || cx < 1)
    return false;
  const SweepGeom g = make_sstep_geom(d.N, ppt, cx, nt);
  if (!sstep_basis_shape_ok(g, fp32) || g.nwg > d.part_stride) return false;
  *out = g;
  return true;
}

// Times the basis candidates with the update kernel in shape `upd`.
static SweepGeom tune_basis(maze_session* s, const SweepGeom& upd) {
  DeviceState& d = s->d;
  const bool fp32 = s->cfg.precision == MAZE_MIXED;
  const SweepGeom def = s->sweep;
  std::vector<SweepGeom> cand{def};
  const long long P = (long long)d.N * d.N;
  for (int nt : {512, 1024})
    for (int ppt : {1, 2, 4}) {
      if ((long long)nt * ppt > P) continue;  // segments longer than a plane
      int last = -1;
      for (int cx : {8, 12, 16, 24, 32, 48, 64}) {
        const SweepGeom g = make_sstep_geom(d.N, ppt, cx, nt);
        if (g.nchunk == last || !sstep_basis_shape_ok(g, fp32) || g.nwg > d.part_stride)
          continue;
        last = g.nchunk;
        cand.push_back(g);
      }
    }
  zv_candidates(d, fp32, s->device, &cand);
  if (cand.size() <= 1) return def;
  hipStream_t st = s->stream;
  void* r0 = fp32 ? (void*)d.r32 : (void*)d.r;
  void* p0 = fp32 ? (void*)d.p32 : (void*)d.p;
  void* x = fp32 ? (void*)d.e32 : (void*)d.xsolve;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return def;
  Scalars sc{};
  sc.thr = -1.0;
  sc.max_iter = 1 << 30;
  sc.norm = MAZE_NORM_REL2;
  bool ok = hipMemcpyAsync(d.sc, &sc, sizeof(Scalars), hipMemcpyHostToDevice, st) == hipSuccess &&
            launch_fill_pattern(r0, d.G, fp32, st) == hipSuccess &&
            launch_fill_pattern(p0, d.G, fp32, st) == hipSuccess;
  SweepGeom best = def;
  float best_ms = 1e30f;
  for (const SweepGeom& g : cand) {
    // outer step 2 (parity 0, not the first: reads r[0], p[0], x; the
    // update writes r[1], p[1] and x), whole outer steps: a basis kernel
    // timed alone, on data it has just read, ranks the shapes differently
    for (int k = 0; k < 2 && ok; ++k)
      ok = launch_sstep_outer(d, g, upd, 2, x, fp32, false, st) == hipSuccess;
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    for (int k = 0; k < 6 && ok; ++k)
      ok = launch_sstep_outer(d, g, upd, 2, x, fp32, false, st) == hipSuccess;
    ok = ok && hipEventRecord(e1, st) == hipSuccess;
    Scalars h{};
    ok = ok && hipMemcpyAsync(&h, d.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) break;
    float ms = 0.f;
    if (h.done == 0 && h.err == 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
        ms < best_ms) {
      best_ms = ms;
      best = g;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!ok) {
    hipGetLastError();
    return def;
  }
  return best;
}

// Shape of the update kernel of the two-iteration CG: the session's
// latency sweep shape (256 threads) or a 512-thread shape (segments of 1024
// or 2048 points: half the halo rows per point, at fewer waves per CU).
// Each candidate runs 2 warm-up and 6 timed outer steps (basis kernel,
// then the update kernel in that shape) on a fill of the session's r and
// p. MAZE_UPDATE_SHAPE="threads:ppt:cx" forces one; a forced
// MAZE_SWEEP_SHAPE keeps the sweep shape.

static bool forced_update(const DeviceState& d, bool fp32, SweepGeom* out) {
  const char* e = std::getenv("MAZE_UPDATE_SHAPE");
  int nt = 0, ppt = 0, cx = 0;
  if (!e || std::sscanf(e, "%d:%d:%d", &nt, &ppt, &cx) != 3) return false;
  if ((nt != kThreads && nt != 512) || (ppt != 1 && ppt != 2 && ppt != 4) || cx < 1) return false;
  const SweepGeom g = make_sstep_geom(d.N, ppt, cx, nt);
  if (!sstep_update_shape_ok(g, fp32) || g.nwg > d.part_stride) return false;
  *out = g;
  return true;
}

// Times the update candidates with the basis kernel in shape `basis`.
static SweepGeom tune_update(maze_session* s, const SweepGeom& basis) {
  DeviceState& d = s->d;
  const bool fp32 = s->cfg.precision == MAZE_MIXED;
  const SweepGeom def = s->sweep;
  std::vector<SweepGeom> cand{def};
  const long long P = (long long)d.N * d.N;
  for (int ppt : {2, 4}) {
    if (512LL * ppt > P) continue;  // segments longer than a plane
    int last = -1;
    for (int cx : {8, 12, 16, 24, 32, 48, 64}) {
      const SweepGeom g = make_sstep_geom(d.N, ppt, cx, 512);
      if (g.nchunk == last || !sstep_update_shape_ok(g, fp32) || g.nwg > d.part_stride) continue;
      last = g.nchunk;
      cand.push_back(g);
    }
  }
  if (cand.size() <= 1) return def;
  hipStream_t st = s->stream;
  void* r0 = fp32 ? (void*)d.r32 : (void*)d.r;
  void* p0 = fp32 ? (void*)d.p32 : (void*)d.p;
  void* x = fp32 ? (void*)d.e32 : (void*)d.xsolve;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return def;
  Scalars sc{};
  sc.thr = -1.0;  // never converged
  sc.max_iter = 1 << 30;
  sc.norm = MAZE_NORM_REL2;
  // outer step 2: parity 0, not the first (reads r[0], p[0] and x)
  bool ok = hipMemcpyAsync(d.sc, &sc, sizeof(Scalars), hipMemcpyHostToDevice, st) == hipSuccess &&
            launch_fill_pattern(r0, d.G, fp32, st) == hipSuccess &&
            launch_fill_pattern(p0, d.G, fp32, st) == hipSuccess;
  SweepGeom best = def;
  float best_ms = 1e30f;
  for (const SweepGeom& g : cand) {
    for (int k = 0; k < 2 && ok; ++k)
      ok = launch_sstep_outer(d, basis, g, 2, x, fp32, false, st) == hipSuccess;
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    for (int k = 0; k < 6 && ok; ++k)
      ok = launch_sstep_outer(d, basis, g, 2, x, fp32, false, st) == hipSuccess;
    ok = ok && hipEventRecord(e1, st) == hipSuccess;
    Scalars h{};
    ok = ok && hipMemcpyAsync(&h, d.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) break;
    float ms = 0.f;
    if (h.done == 0 && h.err == 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
        ms < best_ms) {
      best_ms = ms;
      best = g;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!ok) {
    hipGetLastError();
    return def;
  }
  return best;
}

// Basis and update shapes of a two-iteration session. Each kernel's best
// shape depends on the other's (the basis kernel reads what the update
// kernel has just written), so the update shape is timed with the latency
// basis, the basis shape with that update, and the update shape again with
// the chosen basis. The pair is cached per (device, N, precision); a forced
// shape is kept and the other tuned around it; MAZE_AUTOTUNE=0 keeps the
// latency shape for both.
struct SstepShapes {
  SweepGeom basis, update;
};
static std::map<TuneKey, SstepShapes> g_tuned_sstep;

static void autotune_sstep(maze_session* s) {
  DeviceState& d = s->d;
  const bool fp32 = s->cfg.precision == MAZE_MIXED;
  SweepGeom b = s->sweep, u = s->sweep, fs;
  const bool fb = forced_basis(d, fp32, &b);
  // a forced sweep shape (MAZE_SWEEP_SHAPE) is the update shape as well
  const bool fu = forced_update(d, fp32, &u) || forced_shape(d, fp32, &fs);
  if (autotune_enabled() && !(fb && fu)) {
    const TuneKey key{s->device, d.N, fp32 ? 1 : 0};
    bool hit = false;
    if (!fb && !fu) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tuned_sstep.find(key);
      if (it != g_tuned_sstep.end()) {
        b = it->second.basis;
        u = it->second.update;
        hit = true;
      }
    }
    if (!hit) {
      if (!fu) u = tune_update(s, b);
      if (!fb) b = tune_basis(s, u);
      if (!fu && !fb) u = tune_update(s, b);
      if (!fb && !fu) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned_sstep[key] = SstepShapes{b, u};
      }
    }
  }
  s->sbasis = b;
  s->sweep = u;
}


// ---- continuous batches -------------------------------------------------------
// A maze_batch holds the MaZe steps of many sessions in flight on one stream.
// Adding a step queues its assignment, right-hand side and the first unit of
// its solve at once; each advance queues one poll group of CG units in which
// one batched launch per kernel class covers every session whose solve is
// running, then copies every in-flight session's scalars to pinned memory and
// acts on the copy of the group before (the device always has a group
// queued). A session whose solve ends leaves the launches: an FP64 step queues
// its finishing kernels (true residual, field update, energy, forces, the MD
// short range and closing kick); a mixed step queues its FP64 refinement, and
// the next poll decides from its true residual whether another FP32 pass joins
// the launches. A step is handed back once a poll queued after its finishing
// kernels has completed. Each session keeps its own latency shapes (the
// basis, update and sweep shapes it uses alone) and the same per-workgroup
// code, and the sessions' iterations are independent, so a step's result is
// bitwise the one it gets stepped alone, whatever else is in flight.
namespace {
enum BatchPhase { kBatchCg = 0, kBatchCheck = 1, kBatchFinish = 2 };

struct BatchJob {
  maze_session* s = nullptr;
  uint64_t tag = 0;
  bool has_md = false;
  maze_md_state md{};
  const double* pos = nullptr;
  double* forces = nullptr;
  double* energy = nullptr;
  long long md_step = 0;
  int phase = kBatchCg;
  bool fp32 = false;       // precision of the solve in flight
  void* x = nullptr;       // its solution vector
  long long k = 0;         // units of that solve issued so far (the next one's index)
  long long guard = 0;     // host guard on k
  int total = 0;           // CG iterations over the refinement passes
  int refinements = 0;
  long long ready = 0;     // first poll whose copy reflects the work queued last
  int rc = MAZE_OK;
  bool have_thr = false;   // mixed: the step's FP64 threshold, read at its first check
  double thr = 0.0;
  bool stop = false;       // mixed: a pass broke down without progress
  bool tp = false;         // the solve in flight runs in the throughput shapes
};

struct BatchLaunch {
  int kind;  // 0 sweep, 1 basis, 2 update
  bool fp32;
  int c0, c1, wgb0, nwg, nt, ppt, nh;
  bool rows;
  size_t lds;
  int zv;
};
}  // namespace

struct maze_batch {
  hipStream_t stream = nullptr;
  int device = 0;
  int cap = 0;
  std::vector<BatchJob> jobs;
  std::vector<std::pair<uint64_t, maze_stats>> done;
  // launch tables, double-buffered: a table is rewritten only after the poll
  // queued behind the launches that read it has completed
  BatchTable tab[2];
  int tab_cur = 1;
  bool dirty = true;
  std::vector<BatchLaunch> launches;
  std::vector<int> members;  // jobs in the current table, in table order
  long long unit = 0;        // batched units issued (their parity)
  // polls, double-buffered: device list of scalar pointers, device and
  // pinned host copies of the scalars
  struct Poll {
    char* dev = nullptr;
    Scalars* host = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<maze_session*> list;
    long long seq = -1;
  } poll[2];
  long long polls = 0;       // polls queued
  bool have_prev = false;
};

namespace {

size_t batch_poll_bytes(int cap) { return align256(sizeof(Scalars*) * cap) + sizeof(Scalars) * cap; }

// Shapes of a solve that starts now: the session's latency shapes (its
// result is then bitwise the one it gets alone) while the running solves
// together with it need fewer than kThroughputWgs workgroups in their
// throughput shapes, else the throughput shapes (its result then meets its
// tolerance, summed in another order), as maze_step_batch decides for a
// whole batch; MAZE_BATCH_MODE=latency or =throughput forces one. A solve
// keeps its shapes to its end.
bool batch_solve_tp(const maze_batch* b, const maze_session* s) {
  const char* e = std::getenv("MAZE_BATCH_MODE");
  if (e && std::strcmp(e, "latency") == 0) return false;
  if (e && std::strcmp(e, "throughput") == 0) return true;
  long long w = s->sweep_tp.nwg;
  for (const BatchJob& j : b->jobs)
    if (j.phase == kBatchCg && j.s != s) w += j.s->sweep_tp.nwg;
  return w >= kThroughputWgs;
}

// Queues the first unit of a solve of job j, in the shapes chosen for it.
int batch_first_unit(maze_batch* b, BatchJob& j, bool zero_x) {
  maze_session* s = j.s;
  j.tp = batch_solve_tp(b, s);
  if (!j.tp) {
    HIP_TRY(launch_unit(s, 0, j.x, j.fp32, zero_x));
  } else if (sstep_of(s)) {
    HIP_TRY(launch_sstep_outer(s->d, s->sweep_tp, s->sweep_tp, 0, j.x, j.fp32, zero_x, s->stream));
  } else {
    HIP_TRY(launch_cg_sweep(s->d, s->sweep_tp, 0, s->geom.nwg, j.x, j.fp32, zero_x, s->stream));
  }
  j.k = 1;
  j.guard = sweep_guard(s->cfg.max_iter - j.total, 0);
  j.phase = kBatchCg;
  // polls queued before this solve started still show the status of the
  // session's previous solve
  j.ready = b->polls;
  b->dirty = true;
  return MAZE_OK;
}

// Queues the kernels that end a step (after its solve) and marks it to be
// handed back after the next poll.
int batch_finish(maze_batch* b, BatchJob& j, long long next_poll) {
  maze_session* s = j.s;
  DeviceState& d = s->d;
  hipStream_t st = s->stream;
  HIP_TRY(launch_update(d, nullptr, st));
  HIP_TRY(launch_finalize(d, FIN_ENERGY, update_blocks(d.G), 0.0, 0.0, s->cfg.coulomb_k,
                          j.has_md ? j.md.scalars_dev + 6 : j.energy, 0, 0, st));
  double* F = j.has_md ? j.md.f_es_dev : j.forces;
  if (F) HIP_TRY(launch_gather(d, d.phi_prev, s->cfg.coulomb_k, F, st));
  std::swap(d.phi_cur, d.phi_prev);
  s->step += 1;
  if (j.has_md) {
    HIP_TRY(launch_md_bmh(j.md, d, st));
    HIP_TRY(launch_md_finish(j.md, d, j.md_step, st));
  }
  j.phase = kBatchFinish;
  j.ready = next_poll;
  return MAZE_OK;
}

// Rebuilds the launch table from the jobs whose solve is running: ordered by
// (form, precision, template classes), one launch per run of equal class.
int batch_rebuild(maze_batch* b) {
  b->tab_cur ^= 1;
  BatchTable& t = b->tab[b->tab_cur];
  b->launches.clear();
  b->members.clear();
  for (int i = 0; i < (int)b->jobs.size(); ++i)
    if (b->jobs[i].phase == kBatchCg && b->jobs[i].rc == MAZE_OK) b->members.push_back(i);
  b->dirty = false;
  if (b->members.empty()) return MAZE_OK;
  auto job = [&](int q) -> BatchJob& { return b->jobs[b->members[q]]; };
  auto cls = [](const SweepGeom& g, bool rows) {
    return ((((sstep_threads(g)) * 8 + g.ppt) * 16 + sweep_nh_class(g.nh)) * 2 + (rows ? 1 : 0)) *
               32 + g.zv;
  };
  // shapes of a job's solve: basis (or sweep) and update; the flat layout
  // in the throughput shapes, as in a throughput-mode maze_step_batch
  auto geo_a = [](const BatchJob& j) -> const SweepGeom& {
    return j.tp ? j.s->sweep_tp : (sstep_of(j.s) ? j.s->sbasis : j.s->sweep);
  };
  auto geo_u = [](const BatchJob& j) -> const SweepGeom& {
    return j.tp ? j.s->sweep_tp : j.s->sweep;
  };
  auto rows_of = [](const BatchJob& j, const SweepGeom& g) {
    return !j.tp && sstep_of(j.s) && sstep_rows(g);
  };
  auto key = [&](int q) {
    BatchJob& j = job(q);
    const bool ss = sstep_of(j.s);
    const SweepGeom& g0 = geo_a(j);
    const long long a = (ss ? 2 : 0) + (j.fp32 ? 1 : 0);
    const long long c0 = cls(g0, rows_of(j, g0));
    const long long c1 = ss ? cls(geo_u(j), rows_of(j, geo_u(j))) : 0;
    return (a << 40) | (c0 << 20) | c1;
  };
  std::vector<int> order(b->members.size());
  for (size_t q = 0; q < order.size(); ++q) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
  std::vector<int> sorted;
  for (int q : order) sorted.push_back(b->members[q]);
  b->members = sorted;
  char* H = t.host;
  SweepGeom* hg = (SweepGeom*)(H + t.o_geom);
  SweepGeom* hg2 = (SweepGeom*)(H + t.o_geom2);
  int* hw = (int*)(H + t.o_wgb);
  int* hw2 = (int*)(H + t.o_wgb2);
  int wpos = 0, wpos2 = 0;
  // open groups: index into launches of the last basis/sweep and update group
  int gA = -1, gB = -1;
  long long kA = -1, kB = -1;
  for (int q = 0; q < (int)b->members.size(); ++q) {
    BatchJob& j = job(q);
    maze_session* s = j.s;
    const bool ss = sstep_of(s);
    const SweepGeom& ga = geo_a(j);
    const bool ra = rows_of(j, ga);
    const long long ka = ((ss ? 2LL : 0LL) + (j.fp32 ? 1 : 0)) * 1000000007LL + cls(ga, ra);
    if (gA < 0 || ka != kA) {
      if (gA >= 0) hw[wpos++] = b->launches[gA].nwg;
      b->launches.push_back({ss ? 1 : 0, j.fp32, q, q, wpos, 0, sstep_threads(ga), ga.ppt,
                             sweep_nh_class(ga.nh), ra, 0, ss ? ga.zv : 0});
      gA = (int)b->launches.size() - 1;
      kA = ka;
    }
    BatchLaunch& A = b->launches[gA];
    hw[wpos++] = A.nwg;
    A.nwg += ga.nwg;
    A.c1 = q + 1;
    A.lds = std::max(A.lds, ss ? sstep_lds_bytes(ga, j.fp32) : sweep_lds_bytes(ga, j.fp32, false));
    hg[q] = ga;
    if (ss) {
      const SweepGeom& gu = geo_u(j);
      const bool ru = rows_of(j, gu);
      const long long kb = (j.fp32 ? 1 : 0) * 1000000007LL + cls(gu, ru);
      if (gB < 0 || kb != kB || b->launches[gB].c1 != q) {
        if (gB >= 0) hw2[wpos2++] = b->launches[gB].nwg;
        b->launches.push_back({2, j.fp32, q, q, wpos2, 0, sstep_threads(gu), gu.ppt,
                               sweep_nh_class(gu.nh), ru, 0, gu.zv});
        gB = (int)b->launches.size() - 1;
        kB = kb;
      }
      BatchLaunch& B = b->launches[gB];
      hw2[wpos2++] = B.nwg;
      B.nwg += gu.nwg;
      B.c1 = q + 1;
      B.lds = std::max(B.lds, sstep_lds_bytes(gu, j.fp32));
      hg2[q] = gu;
    }
    if (ga.nwg > s->d.part_stride || (ss && (!sstep_basis_shape_ok(ga, j.fp32) ||
                                             !sstep_update_shape_ok(geo_u(j), j.fp32))))
      return MAZE_E_INVALID;
    const int flip = (int)((b->unit ^ j.k) & 1);
    const int nprev = ga.nwg;
    if (j.fp32) {
      SweepArgs<float> a = make_sweep_args<float>(s->d, (float*)j.x, s->geom.nwg, nprev, false);
      a.par_flip = flip;
      ((SweepArgs<float>*)(H + t.o_args))[q] = a;
    } else {
      SweepArgs<double> a = make_sweep_args<double>(s->d, (double*)j.x, s->geom.nwg, nprev, false);
      a.par_flip = flip;
      ((SweepArgs<double>*)(H + t.o_args))[q] = a;
    }
  }
  if (gA >= 0) hw[wpos++] = b->launches[gA].nwg;
  if (gB >= 0) hw2[wpos2++] = b->launches[gB].nwg;
  for (const BatchLaunch& L : b->launches)
    if (L.nh == 0 || L.lds > 160 * 1024 - 2048) return MAZE_E_INVALID;
  HIP_TRY(hipMemcpyAsync(t.dev, H, t.o_scs, hipMemcpyHostToDevice, b->stream));
  return MAZE_OK;
}

// One unit of every running solve: the sweep launches, then the basis
// launches, then the update launches.
int batch_unit(maze_batch* b) {
  BatchTable& t = b->tab[b->tab_cur];
  const int par = (int)(b->unit & 1);
  for (int pass = 0; pass < 3; ++pass)
    for (const BatchLaunch& G : b->launches) {
      if (G.kind != pass) continue;
      SweepLaunch L{};
      L.batch = true;
      L.par = par;
      L.ppt = G.ppt;
      L.nh = G.nh;
      L.zv = G.zv;
      L.args = t.dev + t.o_args + (size_t)G.c0 * sizeof(SweepArgs<double>);
      L.geoms = (const SweepGeom*)(t.dev + (G.kind == 2 ? t.o_geom2 : t.o_geom)) + G.c0;
      L.wg_begin = (const int*)(t.dev + (G.kind == 2 ? t.o_wgb2 : t.o_wgb)) + G.wgb0;
      L.count = G.c1 - G.c0;
      L.nwg_total = G.nwg;
      L.lds = G.lds;
      const hipError_t e = G.kind == 0
                               ? launch_sweep(L, G.fp32, false, b->stream)
                               : launch_sstep_batch(L, G.nt, G.rows, G.fp32, false, G.kind == 2,
                                                    b->stream);
      if (e != hipSuccess) return MAZE_E_DEVICE;
    }
  b->unit += 1;
  for (int i : b->members) b->jobs[i].k += 1;
  return MAZE_OK;
}

// Queues a copy of the scalars of every job in flight into poll slot
// polls % 2.
int batch_queue_poll(maze_batch* b) {
  maze_batch::Poll& P = b->poll[b->polls & 1];
  P.list.clear();
  for (const BatchJob& j : b->jobs) P.list.push_back(j.s);
  P.seq = b->polls;
  const int n = (int)P.list.size();
  b->polls += 1;
  if (n == 0) return MAZE_OK;
  std::vector<Scalars*> ptrs(n);
  for (int i = 0; i < n; ++i) ptrs[i] = P.list[i]->d.sc;
  HIP_TRY(hipMemcpyAsync(P.dev, ptrs.data(), sizeof(Scalars*) * n, hipMemcpyHostToDevice,
                         b->stream));
  Scalars* out_d = (Scalars*)(P.dev + align256(sizeof(Scalars*) * b->cap));
  HIP_TRY(launch_batch_scalars((Scalars* const*)P.dev, n, out_d, b->stream));
  HIP_TRY(hipMemcpyAsync(P.host, out_d, sizeof(Scalars) * n, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipEventRecord(P.ev, b->stream));
  return MAZE_OK;
}

// Acts on a completed poll: solves that ended, refinement decisions, steps
// whose finishing kernels have run.
int batch_process(maze_batch* b, const maze_batch::Poll& P) {
  std::map<maze_session*, const Scalars*> sc;
  for (size_t i = 0; i < P.list.size(); ++i) sc[P.list[i]] = &P.host[i];
  const long long next_poll = b->polls;  // the next poll queued reflects work queued now
  std::vector<BatchJob> keep;
  for (BatchJob& j : b->jobs) {
    auto it = sc.find(j.s);
    if (it == sc.end() || P.seq < j.ready) {
      keep.push_back(j);
      continue;
    }
    const Scalars& h = *it->second;
    maze_session* s = j.s;
    if (h.err) {
      // a rejected position: nothing was advanced beyond the MD drift
      const int rc = recover_error(s);
      maze_stats st{};
      st.grid_n = s->d.N;
      st.status = rc;
      b->done.push_back({j.tag, st});
      b->dirty = true;
      continue;
    }
    if (j.phase == kBatchCg) {
      const bool ended = h.done != 0 || j.k > j.guard;
      if (!ended) {
        keep.push_back(j);
        continue;
      }
      const int code = h.done ? h.done : 3;
      b->dirty = true;
      if (!j.fp32) {
        s->iters = h.iters;
        s->converged = (code == 1);
        s->refinements = 0;
        HIP_TRY(launch_true_residual(s->d, s->geom, s->d.y, s->stream));
        HIP_TRY(launch_finalize(s->d, FIN_SOLVE_END, s->geom.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0,
                                s->stream));
        const int rc = batch_finish(b, j, next_poll);
        if (rc != MAZE_OK) return rc;
        keep.push_back(j);
        continue;
      }
      // mixed: FP64 refinement with the correction of this pass
      s->last_inner[std::min(j.refinements, kMaxRefinements - 1)] = h.iters;
      j.total += h.iters;
      j.refinements += 1;
      HIP_TRY(launch_add_correction(s->d, s->d.y, s->stream));
      HIP_TRY(launch_refine(s->d, s->geom, s->d.y, true, s->stream));
      HIP_TRY(launch_finalize(s->d, FIN_SOLVE_END, s->geom.nwg, 0.0, 0.0, 0.0, nullptr, 0, 0,
                              s->stream));
      j.phase = kBatchCheck;
      j.ready = next_poll;
      // a breakdown without progress ends the step, unconverged
      if (code == 2 && h.iters == 0) j.stop = true;
      keep.push_back(j);
      continue;
    }
    if (j.phase == kBatchCheck) {
      const bool absmax = s->cfg.residual_norm == MAZE_NORM_ABSMAX;
      const double res = absmax ? h.true_max : std::sqrt(h.true_rr);
      if (!j.have_thr) {
        j.thr = h.thr;  // set by the step's solve start, before any inner pass
        j.have_thr = true;
      }
      const double thr = j.thr;
      s->refinements = j.refinements;
      s->iters = j.total;
      if (j.stop || res <= thr || j.refinements >= kMaxRefinements ||
          j.total >= s->cfg.max_iter) {
        s->converged = !j.stop && res <= thr;
        const int rc = batch_finish(b, j, next_poll);
        if (rc != MAZE_OK) return rc;
        keep.push_back(j);
        continue;
      }
      const double inner = std::max(kInnerReduction * res, kInnerMargin * thr);
      HIP_TRY(launch_finalize(s->d, FIN_INNER_START, 0, 0.0, inner, 0.0, nullptr,
                              s->cfg.max_iter - j.total, s->cfg.residual_norm, s->stream));
      j.fp32 = true;
      j.x = s->d.e32;
      const int rc = batch_first_unit(b, j, true);
      if (rc != MAZE_OK) return rc;
      keep.push_back(j);
      continue;
    }
    // kBatchFinish: the poll ran after the finishing kernels
    s->last_iters = s->iters;
    maze_stats st{};
    fill_stats(s, h, &st);
    st.status = s->converged ? MAZE_OK : MAZE_NOT_CONVERGED;
    b->done.push_back({j.tag, st});
  }
  // the table's members are indices into jobs: rebuild it after a removal
  if (keep.size() != b->jobs.size()) b->dirty = true;
  b->jobs.swap(keep);
  return MAZE_OK;
}

}  // namespace

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
    case MAZE_E_CAPACITY:
      return "request exceeds the fixed capacity of maze_step_batch_noalloc (256 sessions)";
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
  for (auto& byf : s->chunk)
    for (auto& bypar : byf)
      for (auto& c : bypar)
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
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
  if (!(cfg->flags & MAZE_FLAG_ALLOW_NET_CHARGE) && std::fabs(qs) > 1e-10 * qa)
    return MAZE_E_NOT_NEUTRAL;

  maze_session* s = new (std::nothrow) maze_session();
  if (!s) return MAZE_E_OOM;
  s->cfg = *cfg;
  s->stream = stream;
  hipGetDevice(&s->device);
  scratch_setup(s->device);
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
  const bool mg = (cfg->flags & MAZE_FLAG_MULTIGRID) != 0;
  const bool mixed = cfg->precision == MAZE_MIXED && !mg;
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
  d.cand = (int32_t*)at(25);
  d.weight_gradient_force = (cfg->flags & MAZE_FLAG_WEIGHT_GRADIENT_FORCE) ? 1 : 0;
  if (mg) {
    MgHierarchy& m = d.mg;
    int Ns[kMgMaxLevels];
    m.levels = mg_plan(d.N, Ns, kMgMaxLevels);
    m.fp32 = cfg->precision == MAZE_MIXED;
    for (int l = 0; l < m.levels; ++l) {
      m.N[l] = Ns[l];
      m.G[l] = (long long)Ns[l] * Ns[l] * Ns[l];
      m.c[l] = std::pow(0.25, l);
    }
    m.z = m.fp32 ? at(26) : (void*)(d.r + d.G);
    m.b[0] = m.fp32 ? at(27) : nullptr;
    m.r[0] = at(28);
    for (int l = 1; l < m.levels; ++l) {
      m.x[l] = at(29 + 3 * (l - 1));
      m.b[l] = at(30 + 3 * (l - 1));
      m.r[l] = at(31 + 3 * (l - 1));
    }
  }
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
  // launch shape of the CG sweep (timed on the still-unused buffers), then
  // clear them again for the first solve
  s->sweep = autotune_sweep(s);
  s->sweep_tp = throughput_sweep(s->d, s->cfg.precision == MAZE_MIXED);
  if (sstep_of(s)) {
    // the two-iteration kernels stage one more array in LDS than the sweep:
    // on the largest grids keep the x run and shorten the segments until
    // they fit
    const bool f32 = s->cfg.precision == MAZE_MIXED;
    for (SweepGeom* g : {&s->sweep, &s->sweep_tp}) {
      if (sstep_basis_shape_ok(*g, f32)) continue;
      for (int ppt : {2, 1}) {
        const SweepGeom h = make_sweep_geom(d.N, ppt, g->cx);
        if (h.ppt < g->ppt && sstep_basis_shape_ok(h, f32) && h.nwg <= d.part_stride) {
          *g = h;
          break;
        }
      }
      if (!sstep_basis_shape_ok(*g, f32)) {
        maze_destroy(s);
        return MAZE_E_INVALID;
      }
    }
  }
  if (sstep_of(s)) autotune_sstep(s);
  else s->sbasis = s->sweep;
  if (hipMemsetAsync(base, 0, L.total, stream) != hipSuccess ||
      hipMemcpyAsync(d.Q, charges_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, stream) !=
          hipSuccess ||
      launch_cand_table(d, stream) != hipSuccess) {
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
  std::vector<maze_session*> one{s};
  std::vector<int> rcs;
  const int rc = step_multi(one, &pos_dev, &field_dev, &forces_dev, &energy_dev, rcs);
  if (rc != MAZE_OK) return rc;
  if (rcs[0] != MAZE_OK) return rcs[0];
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

// Checks of a batch call: distinct sessions on one device and stream.
static int check_batch(maze_session* const* sessions, int32_t count, const double* const* pos_dev) {
  if (!sessions || count <= 0 || !pos_dev) return MAZE_E_INVALID;
  for (int i = 0; i < count; ++i) {
    if (!sessions[i] || !pos_dev[i]) return MAZE_E_INVALID;
    if (sessions[i]->stream != sessions[0]->stream || sessions[i]->device != sessions[0]->device)
      return MAZE_E_INVALID;
    for (int j = 0; j < i; ++j)
      if (sessions[j] == sessions[i]) return MAZE_E_INVALID;
  }
  return MAZE_OK;
}

static int step_batch_impl(maze_session* const* sessions, int32_t count,
                           const double* const* pos_dev, double* const* forces_dev,
                           double* energies_dev, maze_stats* st) {
  std::vector<maze_session*> ss(sessions, sessions + count);
  std::vector<int> rcs;
  std::vector<double*> eptr(count, nullptr);
  if (energies_dev)
    for (int i = 0; i < count; ++i) eptr[i] = energies_dev + i;
  int rc = step_multi(ss, pos_dev, nullptr, forces_dev, eptr.data(), rcs);
  if (rc != MAZE_OK) return rc;
  int worst = MAZE_OK;
  std::vector<Scalars> h;
  if (st) {
    rc = gather_scalars(ss, h);
    if (rc != MAZE_OK) return rc;
  }
  for (int i = 0; i < count; ++i) {
    int r = rcs[i];
    if (r == MAZE_OK && !ss[i]->converged) r = MAZE_NOT_CONVERGED;
    if (st) {
      std::memset(&st[i], 0, sizeof(maze_stats));
      if (r >= 0) fill_stats(ss[i], h[i], &st[i]);
      st[i].status = r;
    }
    if (r < 0 && (worst >= 0 || r < worst)) worst = r;
    else if (worst >= 0 && r > worst) worst = r;
  }
  return worst;
}

int maze_step_batch(maze_session* const* sessions, int32_t count, const double* const* pos_dev,
                    double* const* forces_dev, double* energies_dev, maze_stats* st) {
  const int rc = check_batch(sessions, count, pos_dev);
  if (rc != MAZE_OK) return rc;
  hipSetDevice(sessions[0]->device);
  return step_batch_impl(sessions, count, pos_dev, forces_dev, energies_dev, st);
}

int maze_step_batch_noalloc(maze_session* const* sessions, int32_t count,
                            const double* const* pos_dev, double* const* forces_dev,
                            double* energies_dev, maze_stats* st) {
  if (count > kNoAllocMaxSessions) return MAZE_E_CAPACITY;
  const int rc = check_batch(sessions, count, pos_dev);
  if (rc != MAZE_OK) return rc;
  const int device = sessions[0]->device;
  if (device < 0 || device >= kNoAllocMaxDevices) return MAZE_E_CAPACITY;
  hipSetDevice(device);
  scratch_setup(device);  // a no-op after maze_init on this device
  if (!g_scratch_dev[device]) return MAZE_E_DEVICE;
  BatchTable t = table_layout(kNoAllocMaxSessions);
  t.dev = g_scratch_dev[device];
  t.host = g_noalloc_host[device];
  // the first session's poll events, idle while its solve runs in a batch
  t.ev[0] = sessions[0]->ev[0];
  t.ev[1] = sessions[0]->ev[1];
  tl_fixed_table = &t;
  const int r = step_batch_impl(sessions, count, pos_dev, forces_dev, energies_dev, st);
  tl_fixed_table = nullptr;
  return r;
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
    // timing only: without the system-scope fence at each record, which
    // writes back and invalidates caches between the kernels it brackets
    s->pev.assign(3 * kProfMax, nullptr);
    for (auto& e : s->pev)
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
        return MAZE_E_DEVICE;
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

int maze_launch_shape(const maze_session* s, int32_t* out8) {
  if (!s || !out8) return MAZE_E_INVALID;
  const SweepGeom* g[2] = {&s->sweep, &s->sweep_tp};
  for (int i = 0; i < 2; ++i) {
    out8[4 * i + 0] = g[i]->ppt;
    out8[4 * i + 1] = g[i]->cx;
    out8[4 * i + 2] = g[i]->nwg;
    out8[4 * i + 3] = g[i]->S;
  }
  return MAZE_OK;
}

int maze_sstep_layout(const maze_session* s, int32_t* out2) {
  if (!s || !out2) return MAZE_E_INVALID;
  out2[0] = s->sbasis.zv;
  out2[1] = s->sweep.zv;
  return MAZE_OK;
}

int maze_basis_shape(const maze_session* s, int32_t* out4) {
  if (!s || !out4) return MAZE_E_INVALID;
  out4[0] = sstep_threads(s->sbasis);
  out4[1] = s->sbasis.ppt;
  out4[2] = s->sbasis.cx;
  out4[3] = s->sbasis.nwg;
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
  if (!(md->gamma >= 0) || !std::isfinite(md->gamma) ||
      (md->gamma > 0 && (!(md->kT >= 0) || !std::isfinite(md->kT))))
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
  const long long k = s->step;  // noise counter of the Langevin half steps
  HIP_TRY(launch_md_kick_drift(*md, k, s->stream));
  rc = maze_step(s, md->pos_dev, nullptr, md->f_es_dev, md->scalars_dev + 6, nullptr);
  if (rc < 0) return rc;
  HIP_TRY(launch_md_bmh(*md, s->d, s->stream));
  HIP_TRY(launch_md_finish(*md, s->d, k, s->stream));
  const int rc2 = finish_call(s, st);
  return rc2 < 0 ? rc2 : rc;
}

int maze_md_step_batch(maze_session* const* sessions, const maze_md_state* const* mds,
                       int32_t count, maze_stats* st) {
  if (!sessions || !mds || count <= 0) return MAZE_E_INVALID;
  std::vector<maze_session*> ss(sessions, sessions + count);
  for (int i = 0; i < count; ++i) {
    const int rc = md_check(ss[i], mds[i]);
    if (rc != MAZE_OK) return rc;
    if (ss[i]->stream != ss[0]->stream || ss[i]->device != ss[0]->device) return MAZE_E_INVALID;
    for (int j = 0; j < i; ++j)
      if (ss[j] == ss[i]) return MAZE_E_INVALID;
  }
  hipSetDevice(ss[0]->device);
  std::vector<const double*> pos(count);
  std::vector<double*> forces(count), energies(count);
  std::vector<long long> steps(count);
  for (int i = 0; i < count; ++i) {
    steps[i] = ss[i]->step;
    HIP_TRY(launch_md_kick_drift(*mds[i], steps[i], ss[i]->stream));
    pos[i] = mds[i]->pos_dev;
    forces[i] = mds[i]->f_es_dev;
    energies[i] = mds[i]->scalars_dev + 6;
  }
  std::vector<int> rcs;
  int rc = step_multi(ss, pos.data(), nullptr, forces.data(), energies.data(), rcs);
  if (rc != MAZE_OK) return rc;
  for (int i = 0; i < count; ++i) {
    if (rcs[i] != MAZE_OK) continue;
    HIP_TRY(launch_md_bmh(*mds[i], ss[i]->d, ss[i]->stream));
    HIP_TRY(launch_md_finish(*mds[i], ss[i]->d, steps[i], ss[i]->stream));
  }
  std::vector<Scalars> h;
  if (st) {
    rc = gather_scalars(ss, h);
    if (rc != MAZE_OK) return rc;
  }
  int worst = MAZE_OK;
  for (int i = 0; i < count; ++i) {
    int r = rcs[i];
    if (r == MAZE_OK && !ss[i]->converged) r = MAZE_NOT_CONVERGED;
    if (st) {
      std::memset(&st[i], 0, sizeof(maze_stats));
      if (r >= 0) fill_stats(ss[i], h[i], &st[i]);
      st[i].status = r;
    }
    if (r < 0 && (worst >= 0 || r < worst)) worst = r;
    else if (worst >= 0 && r > worst) worst = r;
  }
  return worst;
}

// ---- continuous batches -------------------------------------------------------
int maze_batch_create(void* stream, int32_t max_sessions, maze_batch** out) {
  if (!out) return MAZE_E_INVALID;
  *out = nullptr;
  if (max_sessions < 1 || max_sessions > 4096) return MAZE_E_INVALID;
  maze_batch* b = new (std::nothrow) maze_batch();
  if (!b) return MAZE_E_OOM;
  b->stream = (hipStream_t)stream;
  b->cap = max_sessions;
  hipGetDevice(&b->device);
  bool ok = true;
  for (BatchTable& t : b->tab) {
    t = table_layout(max_sessions);
    ok = ok && hipMalloc((void**)&t.dev, t.bytes) == hipSuccess &&
         hipHostMalloc((void**)&t.host, t.bytes, hipHostMallocDefault) == hipSuccess;
  }
  for (maze_batch::Poll& P : b->poll) {
    ok = ok && hipMalloc((void**)&P.dev, batch_poll_bytes(max_sessions)) == hipSuccess &&
         hipHostMalloc((void**)&P.host, sizeof(Scalars) * max_sessions, hipHostMallocDefault) ==
             hipSuccess &&
         hipEventCreateWithFlags(&P.ev, hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    maze_batch_destroy(b);
    return MAZE_E_OOM;
  }
  *out = b;
  return MAZE_OK;
}

int maze_batch_add(maze_batch* b, maze_session* s, const maze_md_state* md,
                   const double* pos_dev, double* forces_dev, double* energy_dev, uint64_t tag) {
  if (!b || !s) return MAZE_E_INVALID;
  if (s->stream != b->stream || s->device != b->device || s->d.mg.levels > 0)
    return MAZE_E_INVALID;
  for (const BatchJob& j : b->jobs)
    if (j.s == s) return MAZE_E_INVALID;
  if ((int)b->jobs.size() >= b->cap) return MAZE_E_CAPACITY;
  if (md) {
    const int rc = md_check(s, md);
    if (rc != MAZE_OK) return rc;
  } else if (!pos_dev) {
    return MAZE_E_INVALID;
  }
  hipSetDevice(b->device);
  BatchJob j;
  j.s = s;
  j.tag = tag;
  DeviceState& d = s->d;
  if (md) {
    j.has_md = true;
    j.md = *md;
    j.md_step = s->step;
    HIP_TRY(launch_md_kick_drift(*md, s->step, s->stream));
    pos_dev = md->pos_dev;
  } else {
    j.pos = pos_dev;
    j.forces = forces_dev;
    j.energy = energy_dev;
  }
  s->iters = 0;
  s->refinements = 0;
  s->converged = 0;
  int rc = assign(s, pos_dev);
  if (rc != MAZE_OK) return rc;
  const bool mixed = s->cfg.precision == MAZE_MIXED;
  HIP_TRY(launch_rhs_maze(d, s->geom, mixed, s->stream));
  HIP_TRY(launch_finalize(d, FIN_SOLVE_START, s->geom.nwg, s->cfg.tol, 0.0, 0.0, nullptr,
                          s->cfg.max_iter, s->cfg.residual_norm, s->stream));
  if (mixed) {
    // the first poll after this decides whether an FP32 pass is needed
    j.phase = kBatchCheck;
    j.ready = b->polls;
  } else {
    j.fp32 = false;
    j.x = d.y;
    rc = batch_first_unit(b, j, false);
    if (rc != MAZE_OK) return rc;
  }
  b->jobs.push_back(j);
  return MAZE_OK;
}

int maze_batch_advance(maze_batch* b, int32_t* n_ready) {
  if (!b) return MAZE_E_INVALID;
  hipSetDevice(b->device);
  if (b->dirty) {
    const int rc = batch_rebuild(b);
    if (rc != MAZE_OK) return rc;
  }
  const bool running = !b->members.empty();
  if (running) {
    // one poll per kPollBatch sweeps or half as many two-iteration units:
    // a unit covers every running solve, and units queued after a solve has
    // ended return at once
    bool any_ss = false;
    for (int i : b->members) any_ss |= sstep_of(b->jobs[i].s);
    const int per = any_ss ? kPollBatch / 2 : kPollBatch;
    for (int u = 0; u < per; ++u) {
      const int rc = batch_unit(b);
      if (rc != MAZE_OK) return rc;
    }
  }
  if (!b->jobs.empty() || b->have_prev) {
    int rc = batch_queue_poll(b);
    if (rc != MAZE_OK) return rc;
    const long long cur = b->polls - 1;
    if (b->have_prev) {
      const maze_batch::Poll& P = b->poll[(cur - 1) & 1];
      HIP_TRY(hipEventSynchronize(P.ev));
      rc = batch_process(b, P);
      if (rc != MAZE_OK) return rc;
    }
    if (running) {
      b->have_prev = true;
    } else {
      // nothing on the device to overlap with: act on this poll at once
      const maze_batch::Poll& P = b->poll[cur & 1];
      if (!P.list.empty()) HIP_TRY(hipEventSynchronize(P.ev));
      rc = batch_process(b, P);
      if (rc != MAZE_OK) return rc;
      b->have_prev = false;
    }
  }
  if (n_ready) *n_ready = (int32_t)b->done.size();
  return MAZE_OK;
}

int maze_batch_take(maze_batch* b, int32_t max, uint64_t* tags, maze_stats* st, int32_t* n) {
  if (!b || max < 0 || (max > 0 && !tags)) return MAZE_E_INVALID;
  const int m = std::min<int>(max, (int)b->done.size());
  for (int i = 0; i < m; ++i) {
    tags[i] = b->done[i].first;
    if (st) st[i] = b->done[i].second;
  }
  b->done.erase(b->done.begin(), b->done.begin() + m);
  if (n) *n = m;
  return MAZE_OK;
}

int maze_batch_in_flight(const maze_batch* b) { return b ? (int)b->jobs.size() : 0; }

void maze_batch_destroy(maze_batch* b) {
  if (!b) return;
  hipSetDevice(b->device);
  // finish the steps in flight, so that their sessions stay consistent
  for (int guard = 0; !b->jobs.empty() && guard < (1 << 22); ++guard)
    if (maze_batch_advance(b, nullptr) != MAZE_OK) break;
  if (b->stream) hipStreamSynchronize(b->stream);
  else hipDeviceSynchronize();
  for (BatchTable& t : b->tab) {
    if (t.dev) hipFree(t.dev);
    if (t.host) hipHostFree(t.host);
  }
  for (maze_batch::Poll& P : b->poll) {
    if (P.dev) hipFree(P.dev);
    if (P.host) hipHostFree(P.host);
    if (P.ev) hipEventDestroy(P.ev);
  }
  delete b;
}

// ---- measurement ---------------------------------------------------------------
int maze_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, void* stream) {
  if (!dst_dev || !src_dev || bytes % 16 != 0 || ((uintptr_t)dst_dev | (uintptr_t)src_dev) % 16)
    return MAZE_E_INVALID;
  HIP_TRY(launch_stream_copy(dst_dev, src_dev, bytes, device_cus(), (hipStream_t)stream));
  return MAZE_OK;
}

}  // extern "C"
