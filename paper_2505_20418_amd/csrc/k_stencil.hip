// Stencil passes around the PLCG solve of M y = sigma_p (and of the direct
// Poisson solve M phi = -4 pi q / h): right-hand sides, the FP64 residual of
// the mixed-precision refinement, and the true residual. All of them sweep
// the grid with one marching template. The CG iterations themselves are the
// fused sweeps of k_cg.hip.
//
// Layout: grids are N^3, index (x*N + y)*N + z, z fastest. A workgroup owns
// a segment of S = 256*PPT consecutive points of the flattened (y, z) plane
// and a run of cx consecutive x planes. It walks its planes in x order:
//   - the x neighbours of a point are the same segment in planes x-1 and
//     x+1, kept in registers (prev / cur / next);
//   - the y and z neighbours come from an LDS copy of the plane's segment
//     extended by one full row (N points) on each side, so every y+-1 and
//     periodic z+-1 neighbour of the segment is in LDS;
//   - plane x+2 is loaded while plane x is computed (double-buffered LDS,
//     one barrier per plane).
// All global accesses are z-fastest rows: consecutive lanes touch
// consecutive addresses. Nothing here is a dense contraction, so there is
// no MFMA; the passes are bound by HBM bandwidth.
//
// Reductions: every thread accumulates in FP64 in registers, the workgroup
// reduces with a fixed shuffle/LDS tree, and one partial per workgroup goes
// to a slot of the partial table. The next kernel sums the slot in a fixed
// order (identically in every workgroup). No atomics anywhere, so results
// are bitwise reproducible.
#include <type_traits>

#include "device_util.h"

namespace maze {

MarchGeom make_march_geom(int N, int ppt, int cx) {
  MarchGeom g;
  g.N = N;
  g.P = (long long)N * N;
  g.ppt = ppt;
  g.S = kThreads * ppt;
  g.nseg = (int)((g.P + g.S - 1) / g.S);
  g.cx = cx < 1 ? 1 : (cx > N ? N : cx);
  g.nchunk = (N + g.cx - 1) / g.cx;
  g.nwg = g.nseg * g.nchunk;
  g.nh = (2 * N + kThreads - 1) / kThreads;
  return g;
}

// ---------------------------------------------------------------------------
// The marching template.
// Op supplies: T (LDS element type), K (staged fields), NACC (accumulators),
//   KS (values of its own point that point() reads, 0 to 2), skip(),
//   prepare(sm) -> bool, load(g, T[K]), side(g, double[KS]), point(g, c, xm,
//   xp, ym, yp, zm, zp, sv, acc), acc_is_max(i), acc_slot(i), finish_wg0().
// A plane step loads the side values of its own points first, then the
// plane two ahead (the same loads on every lane: the halo addresses of idle
// lanes are valid points), so that waiting for the side values leaves that
// prefetch in flight while the points are formed.
// ---------------------------------------------------------------------------
template <int PPT, int NH, class Op>
__global__ __launch_bounds__(kThreads) void march_kernel(Op op, MarchGeom g) {
  using T = typename Op::T;
  constexpr int K = Op::K;
  constexpr int NA = Op::NACC;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[8];
  if (op.skip()) return;
  if (!op.prepare(red)) return;

  const int tid = threadIdx.x;
  const int N = g.N;
  const long long P = g.P;
  const int S = g.S;
  const int E = S + 2 * N;
  const int L = xcd_remap(blockIdx.x, g.nwg);
  const int seg = L % g.nseg;
  const int chunk = L / g.nseg;
  const long long s0 = (long long)seg * S;
  const int x0 = chunk * g.cx;
  const int x1 = min(N, x0 + g.cx);
  T* lds = reinterpret_cast<T*>(smem_raw);
#define LDSAT(buf, f, e) lds[((buf) * K + (f)) * E + (e)]

  long long fl[PPT];
  bool valid[PPT];
  int ezm[PPT], ezp[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const long long f = s0 + tid + (long long)j * kThreads;
    valid[j] = f < P;
    const long long fw = valid[j] ? f : (f % P);
    fl[j] = fw;
    const int z = (int)(fw % N);
    const int e = N + tid + j * kThreads;
    ezm[j] = (z == 0) ? e + N - 1 : e - 1;
    ezp[j] = (z == N - 1) ? e - N + 1 : e + 1;
  }
  long long hg[NH];
  int he[NH];
  bool hv[NH];
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int hh = tid + k * kThreads;
    hv[k] = hh < 2 * N;
    const int e = (hh < N) ? hh : (S + hh);
    he[k] = e;
    long long gi = (s0 - N + e) % P;
    if (gi < 0) gi += P;
    hg[k] = gi;
  }

  T prv[PPT][K], cur[PPT][K], nxt[PPT][K];
  double acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = 0.0;

  auto pbase = [&](int x) -> long long {
    x = (x < 0) ? x + N : ((x >= N) ? x - N : x);
    return (long long)x * P;
  };

  // prologue: centre of plane x0-1; plane x0 staged in buffer 0; plane x0+1
  // centre (staged in buffer 1 if it is computed by this workgroup)
  {
    const long long b = pbase(x0 - 1);
#pragma unroll
    for (int j = 0; j < PPT; ++j) op.load(b + fl[j], prv[j]);
  }
  {
    const long long b = pbase(x0);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      op.load(b + fl[j], cur[j]);
#pragma unroll
      for (int f = 0; f < K; ++f) LDSAT(0, f, N + tid + j * kThreads) = cur[j][f];
    }
#pragma unroll
    for (int k = 0; k < NH; ++k)
      if (hv[k]) {
        T v[K];
        op.load(b + hg[k], v);
#pragma unroll
        for (int f = 0; f < K; ++f) LDSAT(0, f, he[k]) = v[f];
      }
  }
  {
    const long long b = pbase(x0 + 1);
#pragma unroll
    for (int j = 0; j < PPT; ++j) op.load(b + fl[j], nxt[j]);
    if (x0 + 1 < x1) {
#pragma unroll
      for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int f = 0; f < K; ++f) LDSAT(1, f, N + tid + j * kThreads) = nxt[j][f];
#pragma unroll
      for (int k = 0; k < NH; ++k)
        if (hv[k]) {
          T v[K];
          op.load(b + hg[k], v);
#pragma unroll
          for (int f = 0; f < K; ++f) LDSAT(1, f, he[k]) = v[f];
        }
    }
  }
  __syncthreads();

  constexpr int KS = Op::KS;
  constexpr int KSA = KS > 0 ? KS : 1;
  // one plane step; PC / PH: the centre / halo of plane x + 2 are loaded
  auto step = [&](auto pc, auto ph, int x, T (&lc)[PPT][K], T (&lh)[NH][K])
                  __attribute__((always_inline)) {
    constexpr bool PC = decltype(pc)::value, PH = decltype(ph)::value;
    const int buf = (x - x0) & 1;
    const long long bx = (long long)x * P;
    double sv[PPT][KSA];
    if constexpr (KS > 0) {
#pragma unroll
      for (int j = 0; j < PPT; ++j) op.side(bx + fl[j], sv[j]);
    }
    if constexpr (PC) {
      const long long b = pbase(x + 2);
#pragma unroll
      for (int j = 0; j < PPT; ++j) op.load(b + fl[j], lc[j]);
      if constexpr (PH) {
#pragma unroll
        for (int k = 0; k < NH; ++k) op.load(b + hg[k], lh[k]);
      }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (valid[j]) {
        const int e = N + tid + j * kThreads;
        T ym[K], yp[K], zm[K], zp[K];
#pragma unroll
        for (int f = 0; f < K; ++f) {
          ym[f] = LDSAT(buf, f, e - N);
          yp[f] = LDSAT(buf, f, e + N);
          zm[f] = LDSAT(buf, f, ezm[j]);
          zp[f] = LDSAT(buf, f, ezp[j]);
        }
        op.point(bx + fl[j], cur[j], prv[j], nxt[j], ym, yp, zm, zp, sv[j], acc);
      }
    }
  };
  using True = std::integral_constant<bool, true>;
  using False = std::integral_constant<bool, false>;

  for (int x = x0; x < x1; ++x) {
    const int buf = (x - x0) & 1;
    const bool need_c = (x + 2 <= x1);
    const bool need_h = (x + 2 < x1);
    T lc[PPT][K];
    T lh[NH][K];
    if (need_h) step(True{}, True{}, x, lc, lh);
    else if (need_c) step(True{}, False{}, x, lc, lh);
    else step(False{}, False{}, x, lc, lh);
    __syncthreads();
    if (need_h) {
#pragma unroll
      for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int f = 0; f < K; ++f) LDSAT(buf, f, N + tid + j * kThreads) = lc[j][f];
#pragma unroll
      for (int k = 0; k < NH; ++k)
        if (hv[k]) {
#pragma unroll
          for (int f = 0; f < K; ++f) LDSAT(buf, f, he[k]) = lh[k][f];
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int f = 0; f < K; ++f) {
        prv[j][f] = cur[j][f];
        cur[j][f] = nxt[j][f];
        if (need_c) nxt[j][f] = lc[j][f];
      }
  }
#undef LDSAT

  // workgroup reduction of each accumulator into its partial slot
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const double v = Op::acc_is_max(i) ? block_max(acc[i], red) : block_sum(acc[i], red);
    if (tid == 0) op.part[(long long)Op::acc_slot(i, op.parity) * op.pstride + L] = v;
  }
  if (blockIdx.x == 0 && tid == 0) op.finish_wg0();
}

// Sum of the six axis neighbours, paired by axis (fixed order).
template <typename T>
__device__ __forceinline__ T nbr_sum(T xm, T xp, T ym, T yp, T zm, T zp) {
  return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// ---------------------------------------------------------------------------
// Right-hand side of the SHAKE system (Section 2, equations "SHAKE" and
// "SHAKEy"): phi_p = 2 phi^k - phi^{k-1}, sigma_p = (h/4pi) M phi_p + (q - qbar),
// first residual r = M y - sigma_p. Staged fields: phi_p and y.
// ---------------------------------------------------------------------------
template <bool MIXED>
struct OpRhsMaze {
  using T = double;
  static constexpr int K = 2;
  static constexpr int NACC = MIXED ? 7 : 5;
  const double* phik;
  const double* phikm1;
  const double* y;
  const double* q;
  double* sigma;
  double* r;
  float* r32;
  double* part;
  int pstride;
  int parity;
  const Scalars* sc;
  double c1;    // h / (4 pi)
  double qbar;

  __device__ bool skip() const { return ctl_ld(&sc->err) != 0; }
  __device__ bool prepare(double*) {
    qbar = ctl_ld(&sc->qbar);
    return true;
  }
  static constexpr int KS = 1;
  __device__ void load(long long g, double v[2]) const {
    v[0] = 2.0 * phik[g] - phikm1[g];
    v[1] = y[g];
  }
  __device__ void side(long long g, double sv[1]) const { sv[0] = q[g]; }
  __device__ void point(long long g, const double* c, const double* xm, const double* xp,
                        const double* ym, const double* yp, const double* zm,
                        const double* zp, const double* sv, double* a) const {
    const double mphi = nbr_sum(xm[0], xp[0], ym[0], yp[0], zm[0], zp[0]) - 6.0 * c[0];
    const double my = nbr_sum(xm[1], xp[1], ym[1], yp[1], zm[1], zp[1]) - 6.0 * c[1];
    const double qv = sv[0] - qbar;
    const double s = c1 * mphi + qv;
    sigma[g] = s;
    const double rv = my - s;
    a[0] += c[0];
    a[1] += qv * qv;
    a[4] += c[1];
    if (MIXED) {
      const float rf = (float)rv;
      r32[g] = rf;
      a[2] += (double)rf * (double)rf;
      a[3] = fmax(a[3], fabs((double)rf));
      a[5] += rv * rv;
      a[6] = fmax(a[6], fabs(rv));
    } else {
      r[g] = rv;
      a[2] += rv * rv;
      a[3] = fmax(a[3], fabs(rv));
    }
  }
  __device__ static bool acc_is_max(int i) { return i == 3 || i == 6; }
  __device__ static int acc_slot(int i, int) {
    const int s[7] = {SL_PHIP, SL_QQ, SL_RR0, SL_RMAX0, SL_XSUM, SL_TRR, SL_TMAX};
    return s[i];
  }
  __device__ void finish_wg0() const {}
};

// ---------------------------------------------------------------------------
// Right-hand side of the direct Poisson solve (equation "linearproblem"):
// s = -(4 pi / h)(q - qbar), start vector x0 = 0, phi^k or 2 phi^k - phi^{k-1}
// (convergence subsection), first residual r = M x0 - s. x0 is written to x.
// ---------------------------------------------------------------------------
template <bool MIXED>
struct OpRhsPoisson {
  using T = double;
  static constexpr int K = 1;
  static constexpr int NACC = MIXED ? 7 : 5;
  const double* phik;
  const double* phikm1;
  const double* q;
  double* sigma;
  double* x;
  double* r;
  float* r32;
  double* part;
  int pstride;
  int parity;
  const Scalars* sc;
  int guess;
  double c4;    // -(4 pi / h)
  double qbar;

  __device__ bool skip() const { return ctl_ld(&sc->err) != 0; }
  __device__ bool prepare(double*) {
    qbar = ctl_ld(&sc->qbar);
    return true;
  }
  static constexpr int KS = 1;
  __device__ void load(long long g, double v[1]) const {
    v[0] = (guess == MAZE_GUESS_ZERO) ? 0.0
         : (guess == MAZE_GUESS_STATIC) ? phik[g] : 2.0 * phik[g] - phikm1[g];
  }
  __device__ void side(long long g, double sv[1]) const { sv[0] = q[g]; }
  __device__ void point(long long g, const double* c, const double* xm, const double* xp,
                        const double* ym, const double* yp, const double* zm,
                        const double* zp, const double* sv, double* a) const {
    const double mx = nbr_sum(xm[0], xp[0], ym[0], yp[0], zm[0], zp[0]) - 6.0 * c[0];
    const double s = c4 * (sv[0] - qbar);
    sigma[g] = s;
    x[g] = c[0];
    const double rv = mx - s;
    a[0] += c[0];
    a[1] += s * s;
    a[4] += c[0];
    if (MIXED) {
      const float rf = (float)rv;
      r32[g] = rf;
      a[2] += (double)rf * (double)rf;
      a[3] = fmax(a[3], fabs((double)rf));
      a[5] += rv * rv;
      a[6] = fmax(a[6], fabs(rv));
    } else {
      r[g] = rv;
      a[2] += rv * rv;
      a[3] = fmax(a[3], fabs(rv));
    }
  }
  __device__ static bool acc_is_max(int i) { return i == 3 || i == 6; }
  __device__ static int acc_slot(int i, int) {
    const int s[7] = {SL_PHIP, SL_QQ, SL_RR0, SL_RMAX0, SL_XSUM, SL_TRR, SL_TMAX};
    return s[i];
  }
  __device__ void finish_wg0() const {}
};

// ---------------------------------------------------------------------------
// Multigrid-preconditioned CG, direction pass: p = z + beta p_old (beta = 0
// on the first iteration) and <p, A p> with A = -M on the fly. z is the
// V-cycle output (FP64 or FP32). Staged field: p.
// ---------------------------------------------------------------------------
template <typename ZT>
struct OpMgDir {
  using T = double;
  static constexpr int K = 1;
  static constexpr int NACC = 1;
  const ZT* z;
  const double* pold;
  double* p;
  double* part;
  int pstride;
  int parity;
  const Scalars* sc;
  double beta;

  __device__ bool skip() const { return ctl_ld(&sc->done) != 0 || ctl_ld(&sc->err) != 0; }
  __device__ bool prepare(double*) {
    beta = ctl_ld(&sc->mg_beta);
    return true;
  }
  static constexpr int KS = 0;
  __device__ void load(long long g, double v[1]) const {
    const double zv = (double)z[g];
    v[0] = (beta == 0.0) ? zv : zv + beta * pold[g];
  }
  __device__ void side(long long, double*) const {}
  __device__ void point(long long g, const double* c, const double* xm, const double* xp,
                        const double* ym, const double* yp, const double* zm, const double* zp,
                        const double*, double* a) const {
    const double ap = 6.0 * c[0] - nbr_sum(xm[0], xp[0], ym[0], yp[0], zm[0], zp[0]);
    p[g] = c[0];
    a[0] += c[0] * ap;
  }
  __device__ static bool acc_is_max(int) { return false; }
  __device__ static int acc_slot(int, int) { return SL_MU0; }
  __device__ void finish_wg0() const {}
};

// Multigrid-preconditioned CG, update pass: x += alpha p, r -= alpha A p
// (A p recomputed from the staged p), ||r||^2 and max |r|.
struct OpMgUpd {
  using T = double;
  static constexpr int K = 1;
  static constexpr int NACC = 2;
  const double* p;
  double* x;
  double* r;
  double* part;
  int pstride;
  int parity;
  const Scalars* sc;
  double alpha;

  __device__ bool skip() const { return ctl_ld(&sc->done) != 0 || ctl_ld(&sc->err) != 0; }
  __device__ bool prepare(double*) {
    alpha = ctl_ld(&sc->mg_alpha);
    return true;
  }
  static constexpr int KS = 2;
  __device__ void load(long long g, double v[1]) const { v[0] = p[g]; }
  __device__ void side(long long g, double sv[2]) const {
    sv[0] = x[g];
    sv[1] = r[g];
  }
  __device__ void point(long long g, const double* c, const double* xm, const double* xp,
                        const double* ym, const double* yp, const double* zm, const double* zp,
                        const double* sv, double* a) const {
    const double ap = 6.0 * c[0] - nbr_sum(xm[0], xp[0], ym[0], yp[0], zm[0], zp[0]);
    x[g] = sv[0] + alpha * c[0];
    const double rv = sv[1] - alpha * ap;
    r[g] = rv;
    a[0] += rv * rv;
    a[1] = fmax(a[1], fabs(rv));
  }
  __device__ static bool acc_is_max(int i) { return i == 1; }
  __device__ static int acc_slot(int i, int) { return i == 0 ? SL_RR0 : SL_RMAX0; }
  __device__ void finish_wg0() const {}
};

// ---------------------------------------------------------------------------
// FP64 residual M x - s of the current solution: the true residual reported
// at exit, and in mixed precision the outer refinement step that restores
// an FP64 residual and hands its FP32 rounding to the next inner solve.
// ---------------------------------------------------------------------------
template <bool WRITE32>
struct OpResidual {
  using T = double;
  static constexpr int K = 1;
  static constexpr int NACC = WRITE32 ? 5 : 3;
  const double* x;
  const double* s;
  float* r32;
  double* part;
  int pstride;
  int parity;
  const Scalars* sc;

  __device__ bool skip() const { return ctl_ld(&sc->err) != 0; }
  __device__ bool prepare(double*) { return true; }
  static constexpr int KS = 1;
  __device__ void load(long long g, double v[1]) const { v[0] = x[g]; }
  __device__ void side(long long g, double sv[1]) const { sv[0] = s[g]; }
  __device__ void point(long long g, const double* c, const double* xm, const double* xp,
                        const double* ym, const double* yp, const double* zm,
                        const double* zp, const double* sv, double* a) const {
    const double rv = (nbr_sum(xm[0], xp[0], ym[0], yp[0], zm[0], zp[0]) - 6.0 * c[0]) - sv[0];
    a[0] += rv * rv;
    a[1] = fmax(a[1], fabs(rv));
    a[2] += c[0];
    if (WRITE32) {
      const float rf = (float)rv;
      r32[g] = rf;
      a[3] += (double)rf * (double)rf;
      a[4] = fmax(a[4], fabs((double)rf));
    }
  }
  __device__ static bool acc_is_max(int i) { return i == 1 || i == 4; }
  __device__ static int acc_slot(int i, int) {
    const int s[5] = {SL_TRR, SL_TMAX, SL_XSUM, SL_RR0, SL_RMAX0};
    return s[i];
  }
  __device__ void finish_wg0() const {}
};

// ---------------------------------------------------------------------------
// Launch plumbing: pick the (PPT, NH) instantiation for the geometry.
// ---------------------------------------------------------------------------
template <int PPT, int NH, class Op>
static hipError_t launch_march_t(const Op& op, const MarchGeom& g, hipStream_t st) {
  const size_t lds = (size_t)2 * Op::K * (g.S + 2 * g.N) * sizeof(typename Op::T);
  if (lds > 65536) {
    // above the default dynamic LDS limit: raise it once for this kernel
    static bool raised = false;
    if (!raised) {
      const hipError_t e = hipFuncSetAttribute((const void*)march_kernel<PPT, NH, Op>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               160 * 1024 - 1024);
      if (e != hipSuccess) return e;
      raised = true;
    }
  }
  hipLaunchKernelGGL((march_kernel<PPT, NH, Op>), dim3(g.nwg), dim3(kThreads), lds, st, op, g);
  return hipGetLastError();
}

template <int PPT, class Op>
static hipError_t launch_march_nh(const Op& op, const MarchGeom& g, hipStream_t st) {
  switch (g.nh) {
    case 1: return launch_march_t<PPT, 1>(op, g, st);
    case 2: return launch_march_t<PPT, 2>(op, g, st);
    case 3:
    case 4: return launch_march_t<PPT, 4>(op, g, st);
    default: return launch_march_t<PPT, 8>(op, g, st);
  }
}

template <class Op>
static hipError_t launch_march(const Op& op, const MarchGeom& g, hipStream_t st) {
  if (g.nh > 8) return hipErrorInvalidValue;
  switch (g.ppt) {
    case 1: return launch_march_nh<1>(op, g, st);
    case 2: return launch_march_nh<2>(op, g, st);
    case 4: return launch_march_nh<4>(op, g, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs_maze(const DeviceState& d, const MarchGeom& g, bool mixed,
                           hipStream_t st) {
  const double c1 = d.h / (4.0 * M_PI);
  if (mixed) {
    OpRhsMaze<true> op{d.phi_cur, d.phi_prev, d.y, d.q, d.sigma, nullptr, d.r32,
                       d.part, d.part_stride, 0, d.sc, c1, 0.0};
    return launch_march(op, g, st);
  }
  OpRhsMaze<false> op{d.phi_cur, d.phi_prev, d.y, d.q, d.sigma, d.r, nullptr,
                      d.part, d.part_stride, 0, d.sc, c1, 0.0};
  return launch_march(op, g, st);
}

hipError_t launch_rhs_poisson(const DeviceState& d, const MarchGeom& g, int guess,
                              double* x, bool mixed, hipStream_t st) {
  const double c4 = -(4.0 * M_PI / d.h);
  if (mixed) {
    OpRhsPoisson<true> op{d.phi_cur, d.phi_prev, d.q, d.sigma, x, nullptr, d.r32,
                          d.part, d.part_stride, 0, d.sc, guess, c4, 0.0};
    return launch_march(op, g, st);
  }
  OpRhsPoisson<false> op{d.phi_cur, d.phi_prev, d.q, d.sigma, x, d.r, nullptr,
                         d.part, d.part_stride, 0, d.sc, guess, c4, 0.0};
  return launch_march(op, g, st);
}

hipError_t launch_mg_dir(const DeviceState& d, const MarchGeom& g, const void* z, bool fp32,
                         const double* pold, double* pnew, hipStream_t st) {
  if (fp32) {
    OpMgDir<float> op{(const float*)z, pold, pnew, d.part, d.part_stride, 0, d.sc, 0.0};
    return launch_march(op, g, st);
  }
  OpMgDir<double> op{(const double*)z, pold, pnew, d.part, d.part_stride, 0, d.sc, 0.0};
  return launch_march(op, g, st);
}

hipError_t launch_mg_upd(const DeviceState& d, const MarchGeom& g, const double* p, double* x,
                         hipStream_t st) {
  OpMgUpd op{p, x, d.r, d.part, d.part_stride, 0, d.sc, 0.0};
  return launch_march(op, g, st);
}

hipError_t launch_refine(const DeviceState& d, const MarchGeom& g, double* x, bool,
                         hipStream_t st) {
  OpResidual<true> op{x, d.sigma, d.r32, d.part, d.part_stride, 0, d.sc};
  return launch_march(op, g, st);
}

hipError_t launch_true_residual(const DeviceState& d, const MarchGeom& g,
                                const double* x, hipStream_t st) {
  OpResidual<false> op{x, d.sigma, nullptr, d.part, d.part_stride, 0, d.sc};
  return launch_march(op, g, st);
}

}  // namespace maze
