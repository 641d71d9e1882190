// Internal declarations of the MI355X Poisson MaZe library: device state of
// a session, the per-kernel launch geometry and the launch wrappers that
// the runtime (maze_capi.hip) calls.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>

#include "../../include/maze.h"

namespace maze {

constexpr int kThreads = 256;   // threads per workgroup everywhere
constexpr int kTile = 8;        // binning / spreading tile edge (grid points)
constexpr int kMaxOrder = 4;
constexpr int kMaxCandAxis = 4;  // spreading: candidate tiles per axis of a tile

// Slots of the per-workgroup partial-sum table. Every kernel that reduces
// writes one double per workgroup into a slot; the consumer sums the slot in
// a fixed order, so all reductions are deterministic and atomic-free.
enum PartialSlot : int {
  SL_QSUM = 0,     // sum of raw assigned charge (spread)
  SL_PHIP,         // sum of phi_p, or of the start vector of a direct solve
  SL_QQ,           // ||q - qbar||^2, or ||rhs||^2 of a direct solve
  SL_RR0,          // ||r||^2, parity 0 (SL_RR0 + 1: parity 1)
  SL_RR1,
  SL_RMAX0,        // max |r|, parity 0 / 1
  SL_RMAX1,
  SL_MU0,          // <p, A p> of a CG sweep, parity 0 / 1
  SL_MU1,
  SL_RW0,          // <r, A p>, parity 0 / 1
  SL_RW1,
  SL_WW0,          // <A p, A p>, parity 0 / 1
  SL_WW1,
  SL_MGRZ,         // <r, z> of the multigrid-preconditioned CG
  SL_XSUM,         // sum of the solution vector (y or phi)
  SL_TRR,          // true FP64 residual ||M x - s||^2
  SL_TMAX,         // true FP64 residual max
  SL_ENERGY,       // phi . (q - qbar)
  SL_PHISUM,       // sum of phi^{k+1}
  SL_SG0,          // two-iteration CG: the 12 Gram moments of its basis
  SL_SGMAX = SL_SG0 + 12,  // two-iteration CG: max |r|
  SL_COUNT
};

// Device-resident solver scalars. Written only by workgroup 0 of the kernel
// that owns each field, read by later kernels (stream order makes writes
// visible at kernel boundaries).
struct alignas(64) Scalars {
  // control, polled by the host
  int32_t done;        // 0 running, 1 converged, 2 breakdown, 3 max_iter
  int32_t iters;       // iterations when done was set
  int32_t err;         // nonzero: non-finite input seen
  int32_t itp[2];      // updates done in the current solve, as read by the
                       // sweep of parity 0 / 1 (written by the sweep before)
  // solve parameters and results
  double thr;          // stopping threshold of the current solve
  double gamma[2];     // ||r||^2 by iteration parity
  double qsum;         // raw charge sum of the last assignment
  double qbar;         // qsum / G
  double qnorm;        // ||q - qbar||_2 (or ||rhs||_2 of a direct solve)
  double xbar;         // mean of the solution vector at exit
  double pbar;         // mean of phi_p (or the direct-solve start)
  double true_rr;      // true residual ||.||_2^2 (FP64)
  double true_max;     // true residual max
  double energy;       // (1/2) k phi . q
  int32_t max_iter;
  int32_t norm;        // MAZE_NORM_*
  int32_t pend;        // two-iteration CG: stop code left by an update that
                       // ended the solve, turned into done by the next kernel
  double mg_rho;       // multigrid-preconditioned CG: <r, z>
  double mg_alpha;     // rho / <p, A p>
  double mg_beta;      // rho / rho of the previous iteration (0 first)
  double thr_outer;    // mixed step: the step's threshold, kept by
                       // FIN_INNER_FIRST while thr holds the inner one
  double pad[1];
};

// Geometry of a marching stencil launch: each workgroup owns a contiguous
// segment of S points of the (y, z) plane (flattened, z fastest) and a run
// of cx consecutive x planes; it walks the x planes keeping the x
// neighbours in registers and the y/z neighbours of one plane in LDS.
struct MarchGeom {
  int N;
  int S;          // segment length = kThreads * PPT
  int nseg;       // ceil(N*N / S)
  int cx;         // planes per workgroup
  int nchunk;     // ceil(N / cx)
  int nwg;        // nseg * nchunk
  int ppt;        // points per thread per plane
  int nh;         // halo elements per thread per plane: ceil(2N / kThreads)
  long long P;    // N*N
};

MarchGeom make_march_geom(int N, int ppt, int cx);

// Geometry of a fused CG sweep (k_cg.hip): segments of S = kThreads * ppt
// points of the (y, z) plane times runs of cx x planes; nh = halo slots per
// thread for one row on each side of the segment.
struct SweepGeom {
  int N;
  int P;          // N*N
  int S;
  int nseg;
  int cx;
  int nchunk;
  int nwg;
  int ppt;
  int nh;
  // two-iteration kernels only: wavefronts per workgroup of the
  // wavefront-row layout (N = 64 ppt; S = (zv - 2) N points of zv - 2 rows
  // per segment), 0 for the segment layouts
  int zv = 0;
};

SweepGeom make_sweep_geom(int N, int ppt, int cx);
size_t sweep_lds_bytes(const SweepGeom& g, bool fp32, bool first);

// Multigrid hierarchy of a session (preconditioner of the PLCG solve).
// Level 0 is the fine grid: its right-hand side is the CG residual and its
// solution the preconditioned residual z; x / b / r of levels >= 1, the
// level-0 residual temporary r[0] and, for an FP32 preconditioner, the
// rounded right-hand side b[0] live in the session allocation.
constexpr int kMgMaxLevels = 12;
struct MgHierarchy {
  int levels = 0;
  bool fp32 = false;
  int N[kMgMaxLevels] = {0};
  long long G[kMgMaxLevels] = {0};
  double c[kMgMaxLevels] = {0};   // operator scale 4^-l
  void* x[kMgMaxLevels] = {nullptr};
  void* b[kMgMaxLevels] = {nullptr};
  void* r[kMgMaxLevels] = {nullptr};
  void* z = nullptr;              // preconditioned residual (T)
};

// Device buffers of one session. All allocated in maze_init.
struct DeviceState {
  int N = 0;
  long long G = 0;
  int n_ions = 0;
  int order = 2;
  double box = 0, h = 0;
  // grids (FP64): phi history, SHAKE solution, charge, constraint, and the
  // direct-solve vector
  double* phi_cur = nullptr;
  double* phi_prev = nullptr;
  double* y = nullptr;
  double* q = nullptr;
  double* sigma = nullptr;
  double* xsolve = nullptr;
  // CG work vectors, each double-buffered (G elements per buffer): FP64
  // (r, p) and FP32 (r32, p32), plus the FP32 correction e32
  double* r = nullptr;
  double* p = nullptr;
  float* r32 = nullptr;
  float* p32 = nullptr;
  float* e32 = nullptr;
  // reduction partials [SL_COUNT][part_stride] and scalars
  double* part = nullptr;
  int part_stride = 0;
  Scalars* sc = nullptr;
  // ions
  double* Q = nullptr;          // charges (input order)
  // binning: tiles of kTile^3 grid points
  int ntx = 0, ntiles = 0;
  int32_t* tile_count = nullptr;  // ntiles
  int32_t* tile_start = nullptr;  // ntiles + 1
  int32_t* tile_cursor = nullptr; // ntiles
  // ntx * (1 + kMaxCandAxis): for each tile index along an axis, the number
  // of tiles whose ions reach it, then those tiles in ascending order (a
  // function of N and the order only, built once)
  int32_t* cand = nullptr;
  int32_t* ion_cell = nullptr;    // n*3 base cell per axis (input order)
  double* ion_t = nullptr;        // n*3 fractional offsets (input order)
  int32_t* sorted_idx = nullptr;  // n, ion index in tile order
  int32_t* s_cell = nullptr;      // n*3, tile order
  double* s_w = nullptr;          // n*3*order weights, tile order
  double* s_Q = nullptr;          // n, tile order
  // MD driver: per-workgroup short-range energy partials (n_ions + 1)
  double* md_epart = nullptr;
  // residual history of the current CG solve (written by the sweeps)
  double* hist = nullptr;
  int hist_cap = 0;
  // multigrid preconditioner (levels == 0: Jacobi)
  MgHierarchy mg;
  // force estimator: 0 equation "F_nostra", 1 equation "F_Benoit"
  int weight_gradient_force = 0;
};

constexpr int kHistCap = 16384;

// ---- launch wrappers (each queues work on `st`, returns hipError_t) ----
hipError_t launch_bin(const DeviceState& d, const double* pos, hipStream_t st);
hipError_t launch_spread(const DeviceState& d, hipStream_t st);
// Builds d.cand (once per session, before the first spread).
hipError_t launch_cand_table(const DeviceState& d, hipStream_t st);
hipError_t launch_gather(const DeviceState& d, const double* phi, double coulomb_k,
                         double* forces, hipStream_t st);

// finalize modes (single-workgroup reductions of partial slots into Scalars)
enum FinalizeMode : int {
  FIN_QSUM = 0,      // qsum, qbar from SL_QSUM over `count` partials
  FIN_SOLVE_START,   // qnorm, thr, pbar; resets it/done/iters
  FIN_SOLVE_END,     // xbar (from SL_XSUM), true residual
  FIN_ENERGY,        // energy from SL_ENERGY, writes energy_out
  FIN_INNER_START,   // mixed inner solve: thr from `param`, resets counters
  FIN_INNER_FIRST,   // first inner solve of a mixed step: thr from the true
                     // residual (done = 4 if it already meets thr)
  FIN_MG_CHECK0,     // multigrid CG: stopping test of the first residual
  FIN_MG_RHO,        // rho = <r, z>, beta (from SL_MGRZ)
  FIN_MG_MU,         // alpha = rho / <p, A p> (from SL_MU0)
  FIN_MG_CONV,       // ||r|| (SL_RR0 / SL_RMAX0): count, trace, stopping test
};
// imax / norm: iteration cap and norm mode installed by the *_START modes.
hipError_t launch_finalize(const DeviceState& d, int mode, int count, double tol,
                           double param, double coulomb_k, double* energy_out,
                           int imax, int norm, hipStream_t st);

// Right-hand sides (write sigma / s, the first residual, and start partials)
hipError_t launch_rhs_maze(const DeviceState& d, const MarchGeom& g, bool mixed,
                           hipStream_t st);
hipError_t launch_rhs_poisson(const DeviceState& d, const MarchGeom& g, int guess,
                              double* x, bool mixed, hipStream_t st);
// Arguments of the CG sweeps of one session (both parities; the sweep of
// parity par reads r[par], p[par] and writes r[par ^ 1], p[par ^ 1]).
template <typename T>
struct SweepArgs {
  T* r[2];         // residual, double-buffered: sweep of parity par reads r[par]
  T* p[2];         // search direction, double-buffered the same way
  T* x;            // solution (updated in place)
  double* part;    // partial-sum table of the session
  Scalars* sc;
  double* hist;    // residual history: hist[k] = ||r_k||_2 of the current solve
  int pstride;
  int nprev_first; // partials written by the kernel before the first sweep
  int nprev_sweep; // partials written by a sweep (its workgroup count)
  int zero_x;      // first sweep only: write x = 0 (start of an FP32 correction)
  int hist_cap;
  int par_flip;    // batched launches: this session's parity is the launch's
                   // parity XOR par_flip (sessions that joined at different
                   // iterations share one launch)
};

template <typename T>
SweepArgs<T> make_sweep_args(const DeviceState& d, T* x, int nprev_first, int nprev_sweep,
                             bool zero_x);

// One sweep launch: a single session (args -> host SweepArgs<T>, geometry g)
// or a batch (args -> device array of SweepArgs<T>, geoms / wg_begin device
// arrays of count and count + 1 entries, nwg_total workgroups, lds bytes).
struct SweepLaunch {
  bool batch;
  int par;
  int ppt, nh;        // template class shared by every session of the launch
  int zv = 0;         // two-iteration kernels: wavefront-row layout class
  const void* args;
  SweepGeom g;
  const SweepGeom* geoms;
  const int* wg_begin;
  int count;
  int nwg_total;
  size_t lds;
};
// Template class of a halo slot count (1, 2, 4 or 8; 0 if too large).
int sweep_nh_class(int nh);
hipError_t launch_sweep(const SweepLaunch& L, bool fp32, bool first, hipStream_t st);
// Sweep k of a single-session solve (k = 0: p_0 = r_0 / 6, no update).
// nprev_first: partials written by the kernel before sweep 0. x: double* or
// float* by fp32; zero_x: sweep 0 writes x = 0.
hipError_t launch_cg_sweep(const DeviceState& d, const SweepGeom& g, int k, int nprev_first,
                           void* x, bool fp32, bool zero_x, hipStream_t st);
// Outer step o of a two-iteration (s = 2) CG solve: its basis kernel and
// its update kernel (o = 0: p_0 = r_0 / 6; zero_x then writes x from zero).
// Same vectors, partial table and scalars as the sweeps above.
// gb: shape of the basis kernel (256 or 1024 threads per workgroup), gu:
// shape of the update kernel (256 threads).
hipError_t launch_sstep_outer(const DeviceState& d, const SweepGeom& gb, const SweepGeom& gu, int o,
                              void* x, bool fp32, bool zero_x, hipStream_t st);
// One of the two kernels of outer step o (update = false: the basis kernel).
hipError_t launch_sstep_half(const DeviceState& d, const SweepGeom& gb, const SweepGeom& gu, int o,
                             void* x, bool fp32, bool zero_x, bool update, hipStream_t st);
// One batched launch of the basis (update = false) or update kernels of a
// class of sessions (L.batch arrays on the device; L.ppt, L.nh and rows the
// class, nt its threads per workgroup; the update kernel reads one partial
// per basis workgroup of its session, nprev_sweep of its arguments).
hipError_t launch_sstep_batch(const SweepLaunch& L, int nt, bool rows, bool fp32, bool first,
                              bool update, hipStream_t st);
// Whether a two-iteration shape runs in the row-owning layout: its
// workgroup size is a multiple of N, so each thread owns a z column of
// consecutive rows of the segment.
bool sstep_rows(const SweepGeom& g);
// Whether a basis-kernel shape has an instantiation that fits (LDS, halo
// class) and runs without register spills.
bool sstep_basis_shape_ok(const SweepGeom& g, bool fp32);
// The same for an update-kernel shape (256 or 512 threads).
bool sstep_update_shape_ok(const SweepGeom& g, bool fp32);
size_t sstep_lds_bytes(const SweepGeom& g, bool fp32);
// Geometry of a two-iteration kernel with nt threads per workgroup.
SweepGeom make_sstep_geom(int N, int ppt, int cx, int nt);
// Geometry of a two-iteration kernel in the wavefront-row layout (N a
// multiple of 64, at most 256): wv wavefronts per workgroup, each holding
// one z row of N / 64 points per lane; segments of wv - 2 rows.
SweepGeom make_sstep_zv_geom(int N, int cx, int wv);
// Threads per workgroup of a two-iteration shape.
int sstep_threads(const SweepGeom& g);
// Fills x (G elements) with a fixed finite pattern.
hipError_t launch_fill_pattern(void* x, long long G, bool fp32, hipStream_t st);
// Batch helpers: {done, iters, err} of every session into out[3 * count];
// copies of every session's scalars into out[count].
hipError_t launch_batch_poll(Scalars* const* scs, int count, int32_t* out, hipStream_t st);
hipError_t launch_batch_scalars(Scalars* const* scs, int count, Scalars* out, hipStream_t st);

// Multigrid-preconditioned CG: z = V-cycle(r) (fp32: FP32 hierarchy); the
// partials of <r, z>; the direction pass p_new = z + beta p_old with
// <p, A p>; the update pass x += alpha p, r -= alpha A p with ||r||.
hipError_t launch_mg_vcycle(const DeviceState& d, const MgHierarchy& m, const double* r, void* z,
                            bool fp32, hipStream_t st);
hipError_t launch_mg_dot(const DeviceState& d, const double* r, const void* z, bool fp32,
                         hipStream_t st);
int mg_dot_blocks(long long G);
int mg_plan(int N, int* Ns, int max_levels);
hipError_t launch_mg_dir(const DeviceState& d, const MarchGeom& g, const void* z, bool fp32,
                         const double* pold, double* pnew, hipStream_t st);
hipError_t launch_mg_upd(const DeviceState& d, const MarchGeom& g, const double* p, double* x,
                         hipStream_t st);
// Mixed precision: x += e (FP64), FP64 residual M x - s, r32 = float(residual),
// e = 0; partials SL_TRR/SL_TMAX (FP64) and SL_RR0/SL_RMAX0 (of r32).
hipError_t launch_refine(const DeviceState& d, const MarchGeom& g, double* x,
                         bool add_e, hipStream_t st);
// True FP64 residual of x (partials SL_TRR, SL_TMAX).
hipError_t launch_true_residual(const DeviceState& d, const MarchGeom& g,
                                const double* x, hipStream_t st);
// phi^{k+1} = (phi_p - pbar) - (4 pi / h)(y - ybar) into phi_prev; y projected;
// optional field copy; partials SL_ENERGY, SL_PHISUM.
hipError_t launch_update(const DeviceState& d, double* field_out, hipStream_t st);
// Projects a direct-solve vector to mean zero (into field_out if given) and
// writes the energy partials.
hipError_t launch_project(const DeviceState& d, double* x, double* field_out,
                          hipStream_t st);
// Mixed precision: x += e32 (FP64 accumulation of the FP32 correction).
hipError_t launch_add_correction(const DeviceState& d, double* x, hipStream_t st);
// Number of workgroups (= partials) of the elementwise grid kernels.
int update_blocks(long long G);

// MD driver
// Streaming copy of bytes (a multiple of 16; 16-byte aligned device
// buffers) in contiguous chunks, one per workgroup (cus is not used).
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, int cus,
                              hipStream_t st);
hipError_t launch_md_kick_drift(const maze_md_state& md, long long step, hipStream_t st);
hipError_t launch_md_bmh(const maze_md_state& md, const DeviceState& d, hipStream_t st);
hipError_t launch_md_finish(const maze_md_state& md, const DeviceState& d, long long step,
                            hipStream_t st);
hipError_t launch_md_prime(const maze_md_state& md, const DeviceState& d, hipStream_t st);
// Number of short-range energy partials for this cutoff (<= n_ions).
int md_energy_partials(const DeviceState& d, double cutoff);

}  // namespace maze
