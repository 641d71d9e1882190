// Two-iteration (s = 2) form of the Jacobi PLCG solve of M y = sigma_p
// (Appendix B; equation "SHAKEy") and of the direct Poisson solve (equation
// "linearproblem"): the s-step conjugate gradient of Chronopoulos and Gear
// (1989) in the basis form of Hoemmen (2010) and Carson (2015).
//
// With A = -M and the preconditioner diag(A) = 6 I, PCG takes the iterates
// of plain CG on Ahat = A / 6 = I + B, B = -(sum of the six neighbours) / 6,
// with residual rhat = r / 6. Every eigenvalue of Ahat lies in [0, 2], so B
// maps into [-1, 1] and the basis below stays well scaled. Two CG
// iterations starting from (x, r, p) stay in the span of
//
//   Y = [p, B p, B^2 p, rhat, B rhat]
//
// and, writing a vector of that span as Y v, Ahat (Y v) = Y (v + S v) for
// every v with v_2 = v_4 = 0, where S shifts (v0, v1, v3) into (v1, v2, v4).
// One outer step therefore needs the Gram matrix Y^T Y and no other
// grid-wide reduction:
//
//   basis kernel:  Y at every point from r and p (B^2 p needs p two points
//                  away), the Gram sums (as 12 moments) and max |r| per
//                  workgroup;
//   update kernel: the sums, then two CG iterations on 5-vectors (alpha,
//                  beta from v^T G w), then x += Y cx, r = 6 Y cr, p = Y cp
//                  at every point, with Y recomputed from the same r and p.
//
// In exact arithmetic the iterates are those of the one-iteration sweep
// and of Hestenes-Stiefel PCG. Per point the pair reads r and p (basis) and
// x, r, p (update) and writes x, r and p: 32 bytes per two iterations in
// FP32 and 64 in FP64, against 48 and 96 for two single-iteration sweeps.
//
// Stopping: the residual norm at the start of an outer step is the direct
// one (rhat^T rhat and max |r| from the basis kernel); after the first
// inner iteration it is the Gram form v^T G v. A solve that converges, or
// reaches its iteration cap, after one inner iteration applies that one
// and leaves a pending code that the next basis kernel turns into `done`.
// With the max-norm test only the direct values exist, so the test runs
// every two iterations.
//
// Layout and marching follow the fused sweep: a workgroup of NT threads
// (256; the basis kernel also 1024) owns a segment of S = NT*PPT points of
// the (y, z) plane (thread t holding points t + i*NT, or, where N divides
// NT, a z column of PPT consecutive rows) and a run of x planes and walks
// them in x order, upward in even runs and downward in odd ones. Stage U at plane u forms B p on
// the segment plus one row each side from p staged in LDS with two rows
// each side; stage W at the plane before u forms B^2 p and B rhat on the
// segment and either accumulates the Gram sums or writes the updated
// vectors. r and p are double-buffered by outer-step parity; x is updated
// in place.
#include <algorithm>

#include "device_util.h"

namespace maze {

namespace {

// B is symmetric, so <B^a u, B^b v> depends on a + b only: the 15 Gram
// entries of Y come from 12 moments, <p, B^k p> (k = 0..4), <p, B^k rhat>
// (k = 0..3) and <rhat, B^k rhat> (k = 0..2), each summed as the product of
// two basis vectors whose powers add up to k.
constexpr int kNm = 12;       // moments
constexpr int kNs = kNm + 1;  // and max |r|

// Gram index of the pair (a, b), a <= b, of the five basis vectors.
__host__ __device__ constexpr int gidx(int a, int b) {
  return a * 5 - a * (a - 1) / 2 + (b - a);
}

// Moment holding the Gram entry (a, b), a <= b: p-block indices 0..2,
// rhat-block 3..4.
__host__ __device__ constexpr int gmom(int a, int b) {
  return b <= 2 ? a + b : (a <= 2 ? 5 + a + (b - 3) : 9 + (a - 3) + (b - 3));
}

__device__ __forceinline__ int wrap_pl(int u, int N) {
  return u < 0 ? u + N : (u >= N ? u - N : u);
}

// Plane p of a grid as a buffer resource (32-bit per-lane byte offsets,
// reads past the plane return zero); the plane index is made uniform.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pl_rsrc(const T* g, int p, size_t Ps) {
  const T* base = g + (size_t)__builtin_amdgcn_readfirstlane(p) * Ps;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, (int)(Ps * sizeof(T)),
                                           0x00020000);
}
// As pl_rsrc, with no records unless `on` (uniform): loads through it return
// zero without a memory access. A wavefront that issues the same loads on
// every path keeps the compiler's waits for earlier loads from covering
// later ones.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pl_rsrc_if(const T* g, int p, size_t Ps, bool on) {
  const T* base = g + (size_t)__builtin_amdgcn_readfirstlane(p) * Ps;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, on ? (int)(Ps * sizeof(T)) : 0,
                                           0x00020000);
}
// A byte offset past the records of every plane resource: a buffer store
// there is dropped.
constexpr uint32_t kDropOffset = 0x80000000u;
template <typename T>
__device__ __forceinline__ T ld(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}
template <typename T>
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t boff, T v) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, boff, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, v), r, boff, 0, 0);
}

// kNs per-thread values (the last a max) reduced over the NT threads of the
// workgroup in a fixed order; every thread receives the results. Thread i
// of the first kNs combines entry i over the wavefronts, so no thread holds
// more than its own kNs values. sm: kNs * (NT / 64 + 1) doubles.
template <int NT>
__device__ __forceinline__ void block_reduce_ns(double v[kNs], double* sm) {
  constexpr int WV = NT / 64;
#pragma unroll
  for (int i = 0; i < kNs; ++i) v[i] = (i == kNs - 1) ? wave_max(v[i]) : wave_sum(v[i]);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < kNs; ++i) sm[i * WV + w] = v[i];
  }
  __syncthreads();
  double* tot = sm + kNs * WV;
  if (threadIdx.x < kNs) {
    const int i = threadIdx.x;
    double s = sm[i * WV];
    for (int k = 1; k < WV; ++k) s = (i == kNs - 1) ? fmax(s, sm[i * WV + k]) : s + sm[i * WV + k];
    tot[i] = s;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kNs; ++i) v[i] = tot[i];
}

// v^T G w for 5-vectors, G symmetric from its 15 upper entries.
__device__ __forceinline__ double gform(const double* g, const double* v, const double* w) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) s += v[a] * g[a <= b ? gidx(a, b) : gidx(b, a)] * w[b];
  return s;
}

// Ahat v = v + S v for v_2 = v_4 = 0.
__device__ __forceinline__ void ahat(const double* v, double* o) {
  o[0] = v[0];
  o[1] = v[1] + v[0];
  o[2] = v[1];
  o[3] = v[3];
  o[4] = v[3];
}

}  // namespace

// The update kernel's scalar part: the Gram sums of the basis kernel
// (nprev_sweep workgroup partials), then two CG iterations on the
// coordinates of the basis; cx, cr, cp receive the combinations that form
// x, r and p. Returns false where the workgroup has nothing to write (the
// solve stopped; the leader has recorded why).
template <typename T, bool FIRST, int NT>
__device__ __forceinline__ bool sstep_coeffs(const SweepArgs<T>& a, int par, bool leader,
                                             double* red, T (&cx)[5], T (&cr)[5], T (&cp)[5]) {
  Scalars* sc = a.sc;
  const int tid = threadIdx.x;
  double v[kNs];
#pragma unroll
  for (int i = 0; i < kNs; ++i) v[i] = 0.0;
  for (int i = tid; i < a.nprev_sweep; i += NT) {
#pragma unroll
    for (int c = 0; c < kNm; ++c) v[c] += a.part[(size_t)(SL_SG0 + c) * a.pstride + i];
    v[kNm] = fmax(v[kNm], a.part[(size_t)SL_SGMAX * a.pstride + i]);
  }
  block_reduce_ns<NT>(v, red);
  __syncthreads();  // red is reused for the planes below
  double G[15];
#pragma unroll
  for (int aa = 0; aa < 5; ++aa)
#pragma unroll
    for (int b = aa; b < 5; ++b) G[gidx(aa, b)] = v[gmom(aa, b)];
  const int it = ctl_ld(&sc->itp[par]);
  const double thr = ctl_ld(&sc->thr);
  const bool absmax = ctl_ld(&sc->norm) == MAZE_NORM_ABSMAX;
  const int imax = ctl_ld(&sc->max_iter);
  bool finite = true;
#pragma unroll
  for (int c = 0; c < kNs; ++c) finite = finite && isfinite(v[c]);
  const double rr0 = G[gidx(3, 3)];
  const double rn0 = 6.0 * sqrt(fmax(rr0, 0.0));
  if (leader && it < a.hist_cap) a.hist[it] = rn0;
  const bool conv0 = absmax ? (v[kNm] <= thr) : (rn0 <= thr);
  int code = 0;
  if (conv0) code = 1;
  else if (!finite) code = 2;
  else if (it >= imax) code = 3;
  double xv[5] = {0, 0, 0, 0, 0}, rv[5] = {0, 0, 0, 1, 0}, pv[5] = {1, 0, 0, 0, 0};
  double ap[5];
  if (code == 0) {
    ahat(pv, ap);
    const double mu = gform(G, pv, ap);
    if (!(mu > 0.0) || !isfinite(mu)) code = 2;
    else {
      const double al = rr0 / mu;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        xv[c] += al * pv[c];
        rv[c] -= al * ap[c];
      }
    }
  }
  int pend = 0, nsteps = 1;
  if (code != 0) {
    // no update in this outer step. A first step that starts x from zero
    // still has to write x = 0: it runs with zero coefficients for x (r
    // and p copied) and leaves the stop pending, so that no workgroup of
    // this launch skips its points on seeing `done`.
    if (!(FIRST && a.zero_x)) {
      if (leader) {
        ctl_st(&sc->iters, it);
        ctl_st(&sc->done, code);
      }
      return false;
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) xv[c] = rv[c] = pv[c] = 0.0;
    rv[3] = 1.0;
    pv[0] = 1.0;
    pend = code;
    nsteps = 0;
  }
  // first inner iteration done (unless stopped above)
  const double rr1 = fmax(gform(G, rv, rv), 0.0);
  const double rn1 = 6.0 * sqrt(rr1);
  if (pend == 0 && leader && it + 1 < a.hist_cap) a.hist[it + 1] = rn1;
  if (pend == 0) {
    if (!absmax && rn1 <= thr) pend = 1;
    else if (it + 1 >= imax) pend = 3;
  }
  if (nsteps == 1) {
    const double b1 = rr1 / rr0;
#pragma unroll
    for (int c = 0; c < 5; ++c) pv[c] = rv[c] + b1 * pv[c];
  }
  if (pend == 0) {
    ahat(pv, ap);
    const double mu = gform(G, pv, ap);
    if (!(mu > 0.0) || !isfinite(mu)) pend = 2;
    else {
      const double al = rr1 / mu;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        xv[c] += al * pv[c];
        rv[c] -= al * ap[c];
      }
      nsteps = 2;
      const double rr2 = fmax(gform(G, rv, rv), 0.0);
      const double b2 = rr2 / rr1;
#pragma unroll
      for (int c = 0; c < 5; ++c) pv[c] = rv[c] + b2 * pv[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    cx[c] = (T)xv[c];
    cr[c] = (T)(6.0 * rv[c]);
    cp[c] = (T)pv[c];
  }
  if (leader) {
    ctl_st(&sc->itp[par ^ 1], it + nsteps);
    if (pend != 0) ctl_st(&sc->pend, pend);
  }
  return true;
}

// The work of one workgroup (logical index L) of a basis (UPDATE = false)
// or update (UPDATE = true) kernel of outer step parity `par`. FIRST: the
// first outer step of a solve, p = r / 6 (p is not read). ROWS (only where
// N divides NT): each group of N threads owns PPT consecutive rows of the
// segment, a z column per thread, so the y neighbours of a point in an
// inner row are the thread's own values of the rows above and below
// instead of LDS reads.
template <typename T, bool FIRST, bool UPDATE, int PPT, int NH, int NT, bool ROWS>
__device__ __forceinline__ void sstep_wg(const SweepArgs<T>& a, const SweepGeom& g, int par,
                                         int L, unsigned char* smem_raw) {
  // the workgroup reductions use the start of the dynamic LDS (before the
  // march in the update kernel, after it in the basis kernel), so a
  // workgroup needs no LDS beyond its plane buffers
  double* red = reinterpret_cast<double*>(smem_raw);
  Scalars* sc = a.sc;
  if (wg_flags_set(&sc->done, &sc->err, reinterpret_cast<int32_t*>(smem_raw))) return;
  const int tid = threadIdx.x;
  const bool leader = (L == 0) && (tid == 0);
  const T* r_in = par ? a.r[1] : a.r[0];
  T* r_out = par ? a.r[0] : a.r[1];
  const T* p_in = FIRST ? r_in : (par ? a.p[1] : a.p[0]);
  T* p_out = par ? a.p[0] : a.p[1];
  const T sp = FIRST ? (T)(1.0 / 6.0) : (T)1;  // p = sp * (value read)

  // ---- basis kernel: a pending stop left by the update before -------------
  if (!UPDATE && !FIRST) {
    const int pend = ctl_ld(&sc->pend);
    if (pend != 0) {
      if (leader) {
        ctl_st(&sc->iters, ctl_ld(&sc->itp[par]));
        ctl_st(&sc->done, pend);
      }
      return;
    }
  }

  // ---- update kernel: two CG iterations on the coordinates -----------------
  T cx[5], cr[5], cp[5];
  if (UPDATE) {
    if (!sstep_coeffs<T, FIRST, NT>(a, par, leader, red, cx, cr, cp)) return;
  }

  // ---- geometry of this workgroup -------------------------------------------
  // Logical indices run over the chunks of one segment first, so the
  // workgroups that one XCD receives (a contiguous range) hold whole columns
  // of x-neighbouring chunks. Odd chunks march down in x: two neighbouring
  // chunks then start, or end, on the same four planes at the same time.
  // (Measured faster than one direction and segment-major order, by 4% in
  // FP64, although the L2 fetch counters did not fall.)
  const int N = g.N, P = g.P, S = g.S;
  const int chunk = L % g.nchunk, seg = L / g.nchunk;
  const int s0 = seg * S;
  const int x0 = chunk * g.cx, x1 = min(N, x0 + g.cx);
  const int dir = (chunk & 1) ? -1 : 1;
  const int ub = (chunk & 1) ? x1 : x0 - 1;  // plane of stage U at the first step
  const int E1 = S + 4 * N, E2 = S + 2 * N;
  T* P1 = reinterpret_cast<T*>(smem_raw);  // [2][E1] p of plane u (two rows each side)
  // [2][E2] (B p, r) pairs of plane u-1 / u: stage W reads both at each
  // neighbour with one LDS access
  using T2 = T __attribute__((ext_vector_type(2)));
  T2* QR = reinterpret_cast<T2*>(P1 + 2 * E1);
  constexpr int NU = PPT + NH;             // stage-U slots: segment, then inner halo

  int e1[NU], e1zm[NU], e1zp[NU], e2[NU];
  bool uval[NU];
  int e2zm[PPT], e2zp[PPT];
  bool cval[PPT];
  int e1o[NH];
  bool oval[NH];
  uint32_t bo[NU], boo[NH];
  const int grp = ROWS ? tid / N : 0, zcol = tid - grp * N;
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    int f, ee2;
    if (i < PPT) {
      const int loc = ROWS ? (grp * PPT + i) * N + zcol : tid + i * NT;
      f = s0 + loc;
      ee2 = N + loc;
      uval[i] = true;
      cval[i] = f < P;
    } else {
      const int h = tid + (i - PPT) * NT;
      uval[i] = h < 2 * N;
      const int hh = uval[i] ? h : 0;
      ee2 = (hh < N) ? hh : S + hh;
      f = s0 - N + ee2;
    }
    int o = f % P;
    if (o < 0) o += P;
    bo[i] = (uint32_t)o * (uint32_t)sizeof(T);
    e2[i] = ee2;
    e1[i] = ee2 + N;
    const int z = o % N;
    e1zm[i] = (z == 0) ? e1[i] + N - 1 : e1[i] - 1;
    e1zp[i] = (z == N - 1) ? e1[i] - N + 1 : e1[i] + 1;
    if (i < PPT) {
      e2zm[i] = (z == 0) ? ee2 + N - 1 : ee2 - 1;
      e2zp[i] = (z == N - 1) ? ee2 - N + 1 : ee2 + 1;
    }
  }
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int h = tid + k * NT;
    oval[k] = h < 2 * N;
    const int hh = oval[k] ? h : 0;
    e1o[k] = (hh < N) ? hh : S + 2 * N + hh;
    int o = (s0 - 2 * N + e1o[k]) % P;
    if (o < 0) o += P;
    boo[k] = (uint32_t)o * (uint32_t)sizeof(T);
  }

  const T c6 = (T)(1.0 / 6.0);
  const T c36 = (T)(1.0 / 36.0);
  const size_t Ps = (size_t)P;
  // planes named for an upward march (u-1 is the plane before u)
  T pm[NU], pc[NU], pn[NU], pon[NH];  // p: planes u-1, u, u+1; outer halo of u+1
  T rc[NU];                           // r at plane u
  T rm1[PPT], rm2[PPT];               // r at planes u-1, u-2 (segment)
  T bm[PPT], bc[PPT];                 // B p at planes u-2, u-1 (segment)
  T xc[PPT];                          // x at plane u-1 (update)
  // Per-thread moment sums in FP64 for both precisions: the basis values
  // are widened before each product (the product of two floats is exact in
  // FP64), so the Gram matrix of an FP32 inner solve carries only the
  // rounding of the FP32 vectors themselves, and the dot products stay FP64
  // as the precision split of the mixed solver requires.
  double acc[kNs];
#pragma unroll
  for (int i = 0; i < kNs; ++i) acc[i] = 0.0;

  // ---- prologue: planes ub-dir .. ub+dir of p, plane ub of r -----------------
  {
    const auto r0 = pl_rsrc(r_in, wrap_pl(ub, N), Ps);
    const auto pa = pl_rsrc(p_in, wrap_pl(ub - dir, N), Ps);
    const auto pb = pl_rsrc(p_in, wrap_pl(ub, N), Ps);
    const auto pd = pl_rsrc(p_in, wrap_pl(ub + dir, N), Ps);
    T ob[NH];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      rc[i] = ld<T>(r0, bo[i]);
      pm[i] = sp * ld<T>(pa, bo[i]);
      pc[i] = sp * ld<T>(pb, bo[i]);
      pn[i] = sp * ld<T>(pd, bo[i]);
    }
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      ob[k] = sp * ld<T>(pb, boo[k]);
      pon[k] = sp * ld<T>(pd, boo[k]);
    }
#pragma unroll
    for (int i = 0; i < NU; ++i)
      if (uval[i]) P1[e1[i]] = pc[i];
#pragma unroll
    for (int k = 0; k < NH; ++k)
      if (oval[k]) P1[e1o[k]] = ob[k];
#pragma unroll
    for (int j = 0; j < PPT; ++j) rm1[j] = rm2[j] = bm[j] = bc[j] = xc[j] = (T)0;
  }
  __syncthreads();
  __builtin_amdgcn_s_waitcnt(0);

  const int nsteps = x1 - x0 + 2;  // stage U on planes x0-1 .. x1, in march order
  // Uniform memory operations: loads and stores issued alike at every step.
  // Measured per 256^3 launch: the FP32 update kernel 80.8 -> 77.5 us (77.4
  // with stage W skipped on the first two planes); the FP64 update kernel
  // 140.2 -> 142.2 us (148.4 against 147.5 in the second form), so it keeps
  // the conditional form.
  constexpr bool kUniformVm = !UPDATE || sizeof(T) == 4;
  // The compiler does not unroll a loop with a barrier and a run-time trip
  // count, so the plane windows rotate by register moves (about 20 per
  // step); the kernels are not bound by their vector ALU work.
  for (int t = 0; t < nsteps; ++t) {
    const int u = ub + dir * t;
    const bool more = t + 1 < nsteps;
    const bool own_u = (u >= x0) && (u < x1);
    // issue the loads of the next step. With kUniformVm every step issues the
    // same loads (those with nothing to fetch read zeros), so that waiting
    // for them never waits for the stores of stage W issued after them.
    T pf[NU], pof[NH], rf[NU], xf[PPT];
    if (kUniformVm || more) {
      const auto rp = pl_rsrc_if(r_in, wrap_pl(u + dir, N), Ps, more);
      const auto pp = pl_rsrc_if(p_in, wrap_pl(u + 2 * dir, N), Ps, more);
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        rf[i] = ld<T>(rp, bo[i]);
        pf[i] = sp * ld<T>(pp, bo[i]);
      }
#pragma unroll
      for (int k = 0; k < NH; ++k) pof[k] = sp * ld<T>(pp, boo[k]);
      const bool xon = !(FIRST && a.zero_x) && own_u;
      if (UPDATE && (kUniformVm || xon)) {
        const auto xp = pl_rsrc_if((const T*)a.x, wrap_pl(u, N), Ps, more && xon);
#pragma unroll
        for (int j = 0; j < PPT; ++j) xf[j] = ld<T>(xp, bo[j]);
      }
    }

    // stage U at plane u: B p (segment + inner halo), r staged
    const int tb = t & 1;
    T* P1b = P1 + tb * E1;
    T2* QRw = QR + tb * E2;
    T bk[PPT];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      const bool own_m = ROWS && i > 0 && i < PPT, own_p = ROWS && i + 1 < PPT;
      const T ym = own_m ? pc[own_m ? i - 1 : 0] : P1b[e1[i] - N];
      const T yp = own_p ? pc[own_p ? i + 1 : 0] : P1b[e1[i] + N];
      const T bp = -c6 * (((pm[i] + pn[i]) + (ym + yp)) + (P1b[e1zm[i]] + P1b[e1zp[i]]));
      if (uval[i]) {
        T2 w;
        w.x = bp;
        w.y = rc[i];
        QRw[e2[i]] = w;
      }
      if (i < PPT) bk[i] = bp;
    }

    // stage W at plane u-dir: B^2 p and B rhat on the segment, stored from
    // the third step on (plane u-dir then lies in [x0, x1)). With kUniformVm
    // the update kernel enters it at every step and its stores before the
    // third write nothing, so every step issues the same stores.
    if ((UPDATE && kUniformVm) || t >= 2) {
      const T2* QRr = QR + (tb ^ 1) * E2;
      const bool wr = t >= 2;
      const int uo = wrap_pl(u - dir, N);
      const auto xo = pl_rsrc_if((const T*)a.x, uo, Ps, wr);
      const auto ro = pl_rsrc_if((const T*)r_out, uo, Ps, wr);
      const auto po = pl_rsrc_if((const T*)p_out, uo, Ps, wr);
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        // the update kernel's first two steps store zeros that are dropped
        // (nothing to form there)
        T xn = (T)0, rn = (T)0, pnw = (T)0;
        if (!UPDATE || wr) {
        const T y0 = pm[j];
        const T y1 = bc[j];
        T2 ym, yp;
        if (ROWS && j > 0) {
          ym.x = bc[j > 0 ? j - 1 : 0];
          ym.y = rm1[j > 0 ? j - 1 : 0];
        } else {
          ym = QRr[e2[j] - N];
        }
        if (ROWS && j + 1 < PPT) {
          yp.x = bc[j + 1 < PPT ? j + 1 : 0];
          yp.y = rm1[j + 1 < PPT ? j + 1 : 0];
        } else {
          yp = QRr[e2[j] + N];
        }
        const T2 zm = QRr[e2zm[j]], zp = QRr[e2zp[j]];
        const T y2 = -c6 * (((bm[j] + bk[j]) + (ym.x + yp.x)) + (zm.x + zp.x));
        const T y3 = c6 * rm1[j];
        const T y4 = -c36 * (((rm2[j] + rc[j]) + (ym.y + yp.y)) + (zm.y + zp.y));
        if (!UPDATE) {
          if (cval[j]) {
            const double d0 = (double)y0, d1 = (double)y1, d2 = (double)y2, d3 = (double)y3,
                         d4 = (double)y4;
            acc[0] += d0 * d0;
            acc[1] += d0 * d1;
            acc[2] += d1 * d1;
            acc[3] += d1 * d2;
            acc[4] += d2 * d2;
            acc[5] += d0 * d3;
            acc[6] += d0 * d4;
            acc[7] += d1 * d4;
            acc[8] += d2 * d4;
            acc[9] += d3 * d3;
            acc[10] += d3 * d4;
            acc[11] += d4 * d4;
            acc[kNm] = fmax(acc[kNm], fabs((double)rm1[j]));
          }
        } else {
          xn = xc[j] + ((cx[0] * y0 + cx[1] * y1) + (cx[2] * y2 + cx[3] * y3) + cx[4] * y4);
          rn = (cr[0] * y0 + cr[1] * y1) + (cr[2] * y2 + cr[3] * y3) + cr[4] * y4;
          pnw = (cp[0] * y0 + cp[1] * y1) + (cp[2] * y2 + cp[3] * y3) + cp[4] * y4;
        }
        }
        if constexpr (UPDATE) {
          if (kUniformVm || cval[j]) {
            // with kUniformVm a lane past the end of the grid stores out of
            // the buffer's range, which drops it: no branch around the stores
            const uint32_t so = cval[j] ? bo[j] : kDropOffset;
            st<T>(xo, so, xn);
            st<T>(ro, so, rn);
            st<T>(po, so, pnw);
          }
        }
      }
    }

    // stage p of plane u+dir for the next step
    if (more) {
      T* P1n = P1 + (tb ^ 1) * E1;
#pragma unroll
      for (int i = 0; i < NU; ++i)
        if (uval[i]) P1n[e1[i]] = pn[i];
#pragma unroll
      for (int k = 0; k < NH; ++k)
        if (oval[k]) P1n[e1o[k]] = pon[k];
    }
    __syncthreads();

    // rotate
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      bm[j] = bc[j];
      bc[j] = bk[j];
      rm2[j] = rm1[j];
      rm1[j] = rc[j];
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        rc[i] = rf[i];
        pm[i] = pc[i];
        pc[i] = pn[i];
        pn[i] = pf[i];
      }
#pragma unroll
      for (int k = 0; k < NH; ++k) pon[k] = pof[k];
      if (UPDATE) {
#pragma unroll
        for (int j = 0; j < PPT; ++j)
          xc[j] = (kUniformVm || !((FIRST && a.zero_x) || !own_u)) ? xf[j] : (T)0;
      }
    }
  }

  if (!UPDATE) {
    block_reduce_ns<NT>(acc, red);
    if (tid == 0) {
#pragma unroll
      for (int c = 0; c < kNm; ++c) a.part[(size_t)(SL_SG0 + c) * a.pstride + L] = acc[c];
      a.part[(size_t)SL_SGMAX * a.pstride + L] = acc[kNm];
    }
  }
}

template <typename T, bool FIRST, bool UPDATE, int PPT, int NH, int NT, bool ROWS>
__global__ __launch_bounds__(NT) void k_sstep(SweepArgs<T> a, SweepGeom g, int par) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  sstep_wg<T, FIRST, UPDATE, PPT, NH, NT, ROWS>(a, g, par, xcd_remap(blockIdx.x, g.nwg),
                                               smem_raw);
}

// Batched form: the workgroups of `count` sessions in one launch; session i
// owns workgroups [wg_begin[i], wg_begin[i+1]) and runs the same
// per-workgroup code as alone (logical index = block - wg_begin[i]), so a
// session's result does not depend on its batch.
template <typename T, bool FIRST, bool UPDATE, int PPT, int NH, int NT, bool ROWS>
__global__ __launch_bounds__(NT) void k_sstep_batch(const SweepArgs<T>* __restrict__ args,
                                                    const SweepGeom* __restrict__ geoms,
                                                    const int* __restrict__ wg_begin, int count,
                                                    int par) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wg_begin[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const SweepArgs<T> a = args[lo];
  const SweepGeom g = geoms[lo];
  sstep_wg<T, FIRST, UPDATE, PPT, NH, NT, ROWS>(a, g, par ^ a.par_flip, b - wg_begin[lo],
                                               smem_raw);
}

// ---- wavefront-row layout -------------------------------------------------
// Where N = 64 V (V = 1, 2, 4), a wavefront holds whole z rows: lane l the V
// points z = l V .. l V + V - 1 of its row. The z neighbours of a lane's
// points are its own values and, at the two ends, the values of lanes l - 1
// and l + 1, moved by DPP rotations of the whole wavefront by one lane; the
// periodic wrap in z is the rotation's own wrap between lanes 63 and 0. A
// workgroup of WV wavefronts takes the WV consecutive rows y0 - 1 ..
// y0 + WV - 2 of each plane and marches along x as the layouts above: every
// wavefront forms B p on its row (stage U), the inner WV - 2 (the
// workgroup's segment of rows) also B^2 p and B rhat and their Gram sums
// (stage W), and the first and last wavefront also stage p of the rows
// y0 - 2 and y0 + WV - 1. Each lane reads its V points as one 4- to 32-byte
// access, and every LDS offset within a buffer is a compile-time constant
// from the row. The stencil sums are formed in the order of the layouts
// above, so B p, B^2 p and B rhat are the same values; only the grouping
// of the Gram sums into partials differs. The layout serves the basis
// kernel, which only reads: the update kernel, which also writes x, r and
// p, streams at the copy rate in the segment layouts.

template <typename T, int V>
struct VecT {
  using type = T __attribute__((ext_vector_type(V)));
};
template <typename T>
struct VecT<T, 1> {
  using type = T;
};

// lane l receives the value of lane l - 1 (lane 0 that of lane 63)
__device__ __forceinline__ float from_lane_before(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x13C, 0xF, 0xF, false));
}
// lane l receives the value of lane l + 1 (lane 63 that of lane 0)
__device__ __forceinline__ float from_lane_after(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ double from_lane_before(double v) {
  using I2 = int __attribute__((ext_vector_type(2)));
  I2 w = __builtin_bit_cast(I2, v);
  w.x = __builtin_amdgcn_update_dpp(0, w.x, 0x13C, 0xF, 0xF, false);
  w.y = __builtin_amdgcn_update_dpp(0, w.y, 0x13C, 0xF, 0xF, false);
  return __builtin_bit_cast(double, w);
}
__device__ __forceinline__ double from_lane_after(double v) {
  using I2 = int __attribute__((ext_vector_type(2)));
  I2 w = __builtin_bit_cast(I2, v);
  w.x = __builtin_amdgcn_update_dpp(0, w.x, 0x134, 0xF, 0xF, false);
  w.y = __builtin_amdgcn_update_dpp(0, w.y, 0x134, 0xF, 0xF, false);
  return __builtin_bit_cast(double, w);
}

// V consecutive values at byte offset boff of a plane, scaled by s
template <typename T, int V>
__device__ __forceinline__ void ldv(__amdgpu_buffer_rsrc_t r, uint32_t boff, T s, T (&o)[V]) {
  using U4 = unsigned int __attribute__((ext_vector_type(4)));
  constexpr int B = V * (int)sizeof(T);
  struct Arr {
    T v[V];
  } w;
  if constexpr (B == 4) {
    w = __builtin_bit_cast(Arr, __builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0));
  } else if constexpr (B == 8) {
    w = __builtin_bit_cast(Arr, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
  } else if constexpr (B == 16) {
    w = __builtin_bit_cast(Arr, __builtin_amdgcn_raw_buffer_load_b128(r, boff, 0, 0));
  } else {
    static_assert(B == 32, "4 to 32 bytes per lane");
    struct Two {
      U4 a, b;
    } t{__builtin_amdgcn_raw_buffer_load_b128(r, boff, 0, 0),
        __builtin_amdgcn_raw_buffer_load_b128(r, boff + 16, 0, 0)};
    w = __builtin_bit_cast(Arr, t);
  }
#pragma unroll
  for (int i = 0; i < V; ++i) o[i] = s * w.v[i];
}

// LDS: V consecutive values at p (aligned to V * sizeof(T))
template <typename T, int V>
__device__ __forceinline__ void lds_ld(const T* p, T (&o)[V]) {
  using TV = typename VecT<T, V>::type;
  const TV w = *reinterpret_cast<const TV*>(p);
  if constexpr (V == 1) {
    o[0] = w;
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) o[i] = w[i];
  }
}
template <typename T, int V>
__device__ __forceinline__ void lds_st(T* p, const T (&v)[V]) {
  using TV = typename VecT<T, V>::type;
  TV w;
  if constexpr (V == 1) {
    w = v[0];
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) w[i] = v[i];
  }
  *reinterpret_cast<TV*>(p) = w;
}

// Plane buffers of the wavefront-row layout, in elements of T: p rows
// y0 - 2 .. y0 + WV - 1, then B p and r rows y0 - 1 .. y0 + WV - 2, each
// double-buffered.
__host__ __device__ constexpr int zv_lds_elems(int N, int wv) { return 2 * (wv + 2) * N + 4 * wv * N; }

template <typename T, bool FIRST, int V, int WV>
__device__ __forceinline__ void sstep_zv_wg(const SweepArgs<T>& a, const SweepGeom& g, int par,
                                            int L, unsigned char* smem_raw) {
  constexpr int N = 64 * V, NT = 64 * WV, WO = WV - 2;
  double* red = reinterpret_cast<double*>(smem_raw);
  Scalars* sc = a.sc;
  if (wg_flags_set(&sc->done, &sc->err, reinterpret_cast<int32_t*>(smem_raw))) return;
  const int tid = threadIdx.x;
  const bool leader = (L == 0) && (tid == 0);
  const T* r_in = par ? a.r[1] : a.r[0];
  const T* p_in = FIRST ? r_in : (par ? a.p[1] : a.p[0]);
  const T sp = FIRST ? (T)(1.0 / 6.0) : (T)1;  // p = sp * (value read)

  // a stop left pending by the update kernel before ends the solve here
  if (!FIRST) {
    const int pend = ctl_ld(&sc->pend);
    if (pend != 0) {
      if (leader) {
        ctl_st(&sc->iters, ctl_ld(&sc->itp[par]));
        ctl_st(&sc->done, pend);
      }
      return;
    }
  }

  // ---- geometry: chunks of one segment first, odd chunks march down --------
  const int chunk = L % g.nchunk, seg = L / g.nchunk;
  const int y0 = seg * WO;
  const int x0 = chunk * g.cx, x1 = min(N, x0 + g.cx);
  const int dir = (chunk & 1) ? -1 : 1;
  const int ub = (chunk & 1) ? x1 : x0 - 1;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lo = (tid & 63) * V;
  const int yr = (y0 - 1 + w) & (N - 1);
  const bool outw = (w >= 1) && (w <= WO) && (y0 + w - 1 < N);  // row of the segment
  const bool has_o = (w == 0) || (w == WV - 1);                  // stages an outer p row
  const int yo = (w == 0 ? y0 - 2 : y0 - 1 + WV) & (N - 1);
  const int orow = (w == 0) ? 0 : WV + 1;
  const uint32_t bo = (uint32_t)((yr * N + lo) * (int)sizeof(T));
  const uint32_t boo = (uint32_t)((yo * N + lo) * (int)sizeof(T));
  T* P1 = reinterpret_cast<T*>(smem_raw);  // [2][WV + 2][N]
  T* QB = P1 + 2 * (WV + 2) * N;           // [2][WV][N] B p
  T* QS = QB + 2 * WV * N;                 // [2][WV][N] r

  const T c6 = (T)(1.0 / 6.0);
  const T c36 = (T)(1.0 / 36.0);
  const size_t Ps = (size_t)N * N;
  // Plane windows of the row, as rings indexed by the step's phase F =
  // t mod 4 (the march is unrolled four steps deep, so a step renames its
  // windows instead of moving registers). At phase F, plane u:
  //   p:    PW[F] plane u-1, PW[F+1] u, PW[F+2] u+1; loads of u+2 to PW[F+3]
  //   r:    RW[F] plane u-2, RW[F+1] u-1, RW[F+2] u; loads of u+1 to RW[F+3]
  //   B p:  BW[F] plane u-2, BW[F+1] u-1; stage U writes BW[F+2] (plane u)
  //   outer p row: OW[F & 1] plane u+1; loads of u+2 to OW[(F+1) & 1]
  T PW[4][V], RW[4][V], BW[4][V], OW[2][V];
  double acc[kNm];
#pragma unroll
  for (int i = 0; i < kNm; ++i) acc[i] = 0.0;
  T rmax = (T)0;

  {
    const auto r0 = pl_rsrc(r_in, wrap_pl(ub, N), Ps);
    const auto pa = pl_rsrc(p_in, wrap_pl(ub - dir, N), Ps);
    const auto pb = pl_rsrc(p_in, wrap_pl(ub, N), Ps);
    const auto pd = pl_rsrc(p_in, wrap_pl(ub + dir, N), Ps);
    // the outer rows of a wavefront that stages none fetch nothing
    const auto qb = pl_rsrc_if(p_in, wrap_pl(ub, N), Ps, has_o);
    const auto qd = pl_rsrc_if(p_in, wrap_pl(ub + dir, N), Ps, has_o);
    T ob[V];
    ldv<T, V>(r0, bo, (T)1, RW[2]);
    ldv<T, V>(pa, bo, sp, PW[0]);
    ldv<T, V>(pb, bo, sp, PW[1]);
    ldv<T, V>(pd, bo, sp, PW[2]);
    ldv<T, V>(qb, boo, sp, ob);
    ldv<T, V>(qd, boo, sp, OW[0]);
    lds_st<T, V>(P1 + (w + 1) * N + lo, PW[1]);
    if (has_o) lds_st<T, V>(P1 + orow * N + lo, ob);
#pragma unroll
    for (int j = 0; j < V; ++j) RW[0][j] = RW[1][j] = BW[0][j] = BW[1][j] = (T)0;
  }
  __syncthreads();

  const int nsteps = x1 - x0 + 2;  // stage U on planes x0-1 .. x1, in march order
  auto step = [&](auto phase, const int t) __attribute__((always_inline)) {
    constexpr int F = decltype(phase)::value;
    constexpr int F1 = (F + 1) & 3, F2 = (F + 2) & 3, F3 = (F + 3) & 3, tb = F & 1;
    T(&pm)[V] = PW[F];
    T(&pc)[V] = PW[F1];
    T(&pn)[V] = PW[F2];
    T(&pf)[V] = PW[F3];
    T(&rm2)[V] = RW[F];
    T(&rm1)[V] = RW[F1];
    T(&rc)[V] = RW[F2];
    T(&rf)[V] = RW[F3];
    T(&bm)[V] = BW[F];
    T(&bc)[V] = BW[F1];
    T(&bk)[V] = BW[F2];
    T(&po)[V] = OW[tb];
    T(&pof)[V] = OW[tb ^ 1];
    const int u = ub + dir * t;
    const bool more = t + 1 < nsteps;
    {
      // the same three loads on every path: the last step's, and the outer
      // row's of a wavefront that stages none, fetch nothing
      const auto rp = pl_rsrc_if(r_in, wrap_pl(u + dir, N), Ps, more);
      const auto pp = pl_rsrc_if(p_in, wrap_pl(u + 2 * dir, N), Ps, more);
      const auto pq = pl_rsrc_if(p_in, wrap_pl(u + 2 * dir, N), Ps, more && has_o);
      ldv<T, V>(rp, bo, (T)1, rf);
      ldv<T, V>(pp, bo, sp, pf);
      ldv<T, V>(pq, boo, sp, pof);
    }

    // LDS reads of both stages, issued together so that the reads of
    // stage W are in flight while stage U computes (a wavefront outside the
    // segment reads the rows of its nearest segment row and ignores them)
    T ym[V], yp[V], bym[V], byp[V], sym[V], syp[V];
    {
      const T* pr = P1 + (tb * (WV + 2) + w) * N + lo;  // row y - 1; y + 1 is 2N further
      lds_ld<T, V>(pr, ym);
      lds_ld<T, V>(pr + 2 * N, yp);
      const int wc = min(max(w, 1), WO);
      const int q = ((tb ^ 1) * WV + wc - 1) * N + lo;  // row y - 1; y + 1 is 2N further
      lds_ld<T, V>(QB + q, bym);
      lds_ld<T, V>(QB + q + 2 * N, byp);
      lds_ld<T, V>(QS + q, sym);
      lds_ld<T, V>(QS + q + 2 * N, syp);
    }

    // stage U at plane u: B p of the row; (B p, r) staged
    {
      const T zl = from_lane_before(pc[V - 1]), zr = from_lane_after(pc[0]);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const T zm = (i == 0) ? zl : pc[i > 0 ? i - 1 : 0];
        const T zp = (i == V - 1) ? zr : pc[i + 1 < V ? i + 1 : 0];
        bk[i] = -c6 * (((pm[i] + pn[i]) + (ym[i] + yp[i])) + (zm + zp));
      }
      lds_st<T, V>(QB + (tb * WV + w) * N + lo, bk);
      lds_st<T, V>(QS + (tb * WV + w) * N + lo, rc);
    }

    // stage W at plane u-dir: B^2 p, B rhat and the Gram sums on the rows of
    // the segment
    if (t >= 2 && outw) {
      const T bl = from_lane_before(bc[V - 1]), br = from_lane_after(bc[0]);
      const T sl = from_lane_before(rm1[V - 1]), sr = from_lane_after(rm1[0]);
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const T zmb = (j == 0) ? bl : bc[j > 0 ? j - 1 : 0];
        const T zpb = (j == V - 1) ? br : bc[j + 1 < V ? j + 1 : 0];
        const T zms = (j == 0) ? sl : rm1[j > 0 ? j - 1 : 0];
        const T zps = (j == V - 1) ? sr : rm1[j + 1 < V ? j + 1 : 0];
        const T y0v = pm[j];
        const T y1 = bc[j];
        const T y2 = -c6 * (((bm[j] + bk[j]) + (bym[j] + byp[j])) + (zmb + zpb));
        const T y3 = c6 * rm1[j];
        const T y4 = -c36 * (((rm2[j] + rc[j]) + (sym[j] + syp[j])) + (zms + zps));
        const double d0 = (double)y0v, d1 = (double)y1, d2 = (double)y2, d3 = (double)y3,
                     d4 = (double)y4;
        acc[0] += d0 * d0;
        acc[1] += d0 * d1;
        acc[2] += d1 * d1;
        acc[3] += d1 * d2;
        acc[4] += d2 * d2;
        acc[5] += d0 * d3;
        acc[6] += d0 * d4;
        acc[7] += d1 * d4;
        acc[8] += d2 * d4;
        acc[9] += d3 * d3;
        acc[10] += d3 * d4;
        acc[11] += d4 * d4;
        rmax = fmax(rmax, fabs(rm1[j]));
      }
    }

    // stage p of plane u+dir for the next step
    if (more) {
      T* pw = P1 + (tb ^ 1) * (WV + 2) * N + lo;
      lds_st<T, V>(pw + (w + 1) * N, pn);
      if (has_o) lds_st<T, V>(pw + orow * N, po);
    }
    __syncthreads();
    // keep the scheduler from interleaving consecutive steps, which would
    // hold two steps' temporaries at once
    __builtin_amdgcn_sched_barrier(0);
  };
  using Ph0 = std::integral_constant<int, 0>;
  using Ph1 = std::integral_constant<int, 1>;
  using Ph2 = std::integral_constant<int, 2>;
  using Ph3 = std::integral_constant<int, 3>;
  int t = 0;
  for (; t + 4 <= nsteps; t += 4) {
    step(Ph0{}, t);
    step(Ph1{}, t + 1);
    step(Ph2{}, t + 2);
    step(Ph3{}, t + 3);
  }
  if (t < nsteps) step(Ph0{}, t);
  if (t + 1 < nsteps) step(Ph1{}, t + 1);
  if (t + 2 < nsteps) step(Ph2{}, t + 2);

  double sums[kNs];
#pragma unroll
  for (int c = 0; c < kNm; ++c) sums[c] = acc[c];
  sums[kNm] = (double)rmax;
  block_reduce_ns<NT>(sums, red);
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < kNm; ++c) a.part[(size_t)(SL_SG0 + c) * a.pstride + L] = sums[c];
    a.part[(size_t)SL_SGMAX * a.pstride + L] = sums[kNm];
  }
}

template <typename T, bool FIRST, int V, int WV>
__global__ __launch_bounds__(64 * WV) void k_sstep_zv(SweepArgs<T> a, SweepGeom g, int par) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  sstep_zv_wg<T, FIRST, V, WV>(a, g, par, xcd_remap(blockIdx.x, g.nwg), smem_raw);
}

template <typename T, bool FIRST, int V, int WV>
__global__ __launch_bounds__(64 * WV) void k_sstep_zv_batch(const SweepArgs<T>* __restrict__ args,
                                                            const SweepGeom* __restrict__ geoms,
                                                            const int* __restrict__ wg_begin,
                                                            int count, int par) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wg_begin[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const SweepArgs<T> a = args[lo];
  const SweepGeom g = geoms[lo];
  sstep_zv_wg<T, FIRST, V, WV>(a, g, par ^ a.par_flip, b - wg_begin[lo], smem_raw);
}

// Geometry of a two-iteration kernel with nt threads per workgroup
// (segments of nt * ppt points, nh halo slots per thread for one row).
SweepGeom make_sstep_geom(int N, int ppt, int cx, int nt) {
  SweepGeom g;
  g.N = N;
  g.P = N * N;
  g.ppt = ppt;
  g.S = nt * ppt;
  g.nseg = (g.P + g.S - 1) / g.S;
  g.cx = cx < 1 ? 1 : (cx > N ? N : cx);
  g.nchunk = (N + g.cx - 1) / g.cx;
  g.nwg = g.nseg * g.nchunk;
  g.nh = (2 * N + nt - 1) / nt;
  return g;
}

SweepGeom make_sstep_zv_geom(int N, int cx, int wv) {
  SweepGeom g;
  const int wo = wv - 2;
  g.N = N;
  g.P = N * N;
  g.ppt = N / 64;
  g.S = wo * N;
  g.nseg = (N + wo - 1) / wo;
  g.cx = cx < 1 ? 1 : (cx > N ? N : cx);
  g.nchunk = (N + g.cx - 1) / g.cx;
  g.nwg = g.nseg * g.nchunk;
  g.nh = 1;  // no halo slots; a valid class for the checks that read it
  g.zv = wv;
  return g;
}

int sstep_threads(const SweepGeom& g) { return g.zv ? 64 * g.zv : g.S / g.ppt; }

bool sstep_rows(const SweepGeom& g) { return !g.zv && (g.S / g.ppt) % g.N == 0; }

size_t sstep_lds_bytes(const SweepGeom& g, bool fp32) {
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  if (g.zv) {
    const size_t red = sizeof(double) * kNs * (size_t)(g.zv + 1);
    return std::max(es * (size_t)zv_lds_elems(g.N, g.zv), red);
  }
  const size_t e1 = (size_t)g.S + 4 * (size_t)g.N, e2 = (size_t)g.S + 2 * (size_t)g.N;
  const size_t red = sizeof(double) * kNs * (size_t)(g.S / g.ppt / 64 + 1);
  return std::max(es * 2 * (e1 + 2 * e2), red);
}

namespace {

// Dynamic LDS the kernel fn accepts, raised once where it is below lds (the
// runtime refuses the request for some workgroup sizes whose limit is
// already the whole LDS, so the limit is queried first).
hipError_t ensure_lds(const void* fn, size_t lds, size_t* allowed) {
  if (lds > 160 * 1024 - 2048) return hipErrorInvalidValue;
  if (lds <= 65536 || lds <= *allowed) return hipSuccess;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, fn) == hipSuccess && (size_t)fa.maxDynamicSharedSizeBytes >= lds) {
    *allowed = (size_t)fa.maxDynamicSharedSizeBytes;
    return hipSuccess;
  }
  const hipError_t e =
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
  if (e == hipSuccess) *allowed = 160 * 1024 - 2048;
  return e;
}

// Wavefront-row classes with an instantiation: basis kernels only (the
// update kernels stream at the copy rate in the segment layouts), N = 64,
// 128 or 256 (V = 1, 2, 4 points per lane), workgroups of 8 wavefronts;
// at N = 256 in FP32 also of 16 (14 rows per segment, one workgroup per CU:
// fewer halo rows per row than two workgroups of 8; in FP64 its LDS does
// not fit).
constexpr bool zv_class_ok(int v, int wv, bool fp32) {
  return ((v == 1 || v == 2 || v == 4) && wv == 8) || (fp32 && v == 4 && wv == 16);
}

// One session: args and geometry on the host.
template <typename T, bool FIRST, bool UPDATE>
struct SingleLaunch {
  const SweepArgs<T>& a;
  const SweepGeom& g;
  int par;
  hipStream_t st;
  template <int PPT, int NH, int NT, bool ROWS>
  hipError_t run() const {
    static size_t allowed = 0;
    const size_t lds = sstep_lds_bytes(g, sizeof(T) == 4);
    const hipError_t e = ensure_lds(
        (const void*)k_sstep<T, FIRST, UPDATE, PPT, NH, NT, ROWS>, lds, &allowed);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sstep<T, FIRST, UPDATE, PPT, NH, NT, ROWS>), dim3(g.nwg), dim3(NT),
                       lds, st, a, g, par);
    return hipGetLastError();
  }
  template <int V, int WV>
  hipError_t run_zv() const {
    if constexpr (!zv_class_ok(V, WV, sizeof(T) == 4)) {
      return hipErrorInvalidValue;
    } else {
      static size_t allowed = 0;
      const size_t lds = sstep_lds_bytes(g, sizeof(T) == 4);
      const hipError_t e =
          ensure_lds((const void*)k_sstep_zv<T, FIRST, V, WV>, lds, &allowed);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_sstep_zv<T, FIRST, V, WV>), dim3(g.nwg), dim3(64 * WV), lds, st,
                         a, g, par);
      return hipGetLastError();
    }
  }
};

// A batch of sessions of one template class (device arrays in L).
template <typename T, bool FIRST, bool UPDATE>
struct BatchLaunch {
  const SweepLaunch& L;
  hipStream_t st;
  template <int PPT, int NH, int NT, bool ROWS>
  hipError_t run() const {
    static size_t allowed = 0;
    const hipError_t e = ensure_lds(
        (const void*)k_sstep_batch<T, FIRST, UPDATE, PPT, NH, NT, ROWS>, L.lds, &allowed);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sstep_batch<T, FIRST, UPDATE, PPT, NH, NT, ROWS>), dim3(L.nwg_total),
                       dim3(NT), L.lds, st, static_cast<const SweepArgs<T>*>(L.args), L.geoms,
                       L.wg_begin, L.count, L.par);
    return hipGetLastError();
  }
  template <int V, int WV>
  hipError_t run_zv() const {
    if constexpr (!zv_class_ok(V, WV, sizeof(T) == 4)) {
      return hipErrorInvalidValue;
    } else {
      static size_t allowed = 0;
      const hipError_t e =
          ensure_lds((const void*)k_sstep_zv_batch<T, FIRST, V, WV>, L.lds, &allowed);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_sstep_zv_batch<T, FIRST, V, WV>), dim3(L.nwg_total),
                         dim3(64 * WV), L.lds, st, static_cast<const SweepArgs<T>*>(L.args),
                         L.geoms, L.wg_begin, L.count, L.par);
      return hipGetLastError();
    }
  }
};


template <bool UPDATE, class F>
hipError_t sstep_zv_dispatch(int v, int wv, const F& f) {
  if constexpr (UPDATE) {
    return hipErrorInvalidValue;
  } else {
    switch (v * 100 + wv) {
      case 108: return f.template run_zv<1, 8>();
      case 208: return f.template run_zv<2, 8>();
      case 408: return f.template run_zv<4, 8>();
      case 416: return f.template run_zv<4, 16>();
      default: return hipErrorInvalidValue;
    }
  }
}

// rows: the row-owning layout (N divides NT, so at most two halo slots)
template <bool UPDATE, int PPT, int NT, class F>
hipError_t sstep_nh(int nh, bool rows, const F& f) {
  switch (nh) {
    case 1:
      return rows ? f.template run<PPT, 1, NT, true>() : f.template run<PPT, 1, NT, false>();
    case 2:
      return rows ? f.template run<PPT, 2, NT, true>() : f.template run<PPT, 2, NT, false>();
    case 4:
      if constexpr (NT == kThreads)
        if (!rows) return f.template run<PPT, 4, NT, false>();
      return hipErrorInvalidValue;
    case 8:
      if constexpr (NT == kThreads)
        if (!rows) return f.template run<PPT, 8, NT, false>();
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// Workgroups of kThreads for every kernel; both also come in 512-thread and
// the basis kernel in 1024-thread workgroups (longer segments, less halo
// work per point).
template <bool UPDATE, class F>
hipError_t sstep_dispatch(int nt, int ppt, int nh, bool rows, const F& f) {
  if (nt == kThreads) {
    switch (ppt) {
      case 1: return sstep_nh<UPDATE, 1, kThreads>(nh, rows, f);
      case 2: return sstep_nh<UPDATE, 2, kThreads>(nh, rows, f);
      case 4: return sstep_nh<UPDATE, 4, kThreads>(nh, rows, f);
      default: return hipErrorInvalidValue;
    }
  }
  if (nt == 512) {
    switch (ppt) {
      case 2: return sstep_nh<UPDATE, 2, 512>(nh, rows, f);
      case 4: return sstep_nh<UPDATE, 4, 512>(nh, rows, f);
      default: return hipErrorInvalidValue;
    }
  }
  if constexpr (!UPDATE) {
    if (nt == 1024) {
      switch (ppt) {
        case 1: return sstep_nh<UPDATE, 1, 1024>(nh, rows, f);
        case 2: return sstep_nh<UPDATE, 2, 1024>(nh, rows, f);
        case 4: return sstep_nh<UPDATE, 4, 1024>(nh, rows, f);
        default: return hipErrorInvalidValue;
      }
    }
  }
  return hipErrorInvalidValue;
}

template <typename T, bool FIRST, bool UPDATE>
hipError_t sstep_ppt(const SweepArgs<T>& a, const SweepGeom& g, int par, hipStream_t st) {
  const SingleLaunch<T, FIRST, UPDATE> f{a, g, par, st};
  if (g.zv) return sstep_zv_dispatch<UPDATE>(g.ppt, g.zv, f);
  return sstep_dispatch<UPDATE>(g.S / g.ppt, g.ppt, sweep_nh_class(g.nh), sstep_rows(g), f);
}

template <typename T, bool FIRST, bool UPDATE>
hipError_t sstep_batch_ppt(const SweepLaunch& L, int nt, bool rows, hipStream_t st) {
  const BatchLaunch<T, FIRST, UPDATE> f{L, st};
  if (L.zv) return sstep_zv_dispatch<UPDATE>(L.ppt, L.zv, f);
  return sstep_dispatch<UPDATE>(nt, L.ppt, L.nh, rows, f);
}

template <typename T>
hipError_t sstep_half(const SweepArgs<T>& a, const SweepGeom& g, int o, bool update,
                      hipStream_t st) {
  const int par = o & 1;
  if (o == 0)
    return update ? sstep_ppt<T, true, true>(a, g, par, st) : sstep_ppt<T, true, false>(a, g, par, st);
  return update ? sstep_ppt<T, false, true>(a, g, par, st) : sstep_ppt<T, false, false>(a, g, par, st);
}

}  // namespace

hipError_t launch_sstep_half(const DeviceState& d, const SweepGeom& gb, const SweepGeom& gu, int o,
                             void* x, bool fp32, bool zero_x, bool update, hipStream_t st) {
  // one partial per workgroup and slot: the basis shape must fit the
  // buffer's rows (the update reads one row per basis workgroup)
  if (gb.nwg < 1 || gb.nwg > d.part_stride || gu.nwg < 1 || o < 0) return hipErrorInvalidValue;
  const bool zx = zero_x && o == 0;
  const SweepGeom& g = update ? gu : gb;
  if (fp32) return sstep_half<float>(make_sweep_args<float>(d, (float*)x, 0, gb.nwg, zx), g, o,
                                     update, st);
  return sstep_half<double>(make_sweep_args<double>(d, (double*)x, 0, gb.nwg, zx), g, o, update,
                            st);
}

hipError_t launch_sstep_outer(const DeviceState& d, const SweepGeom& gb, const SweepGeom& gu, int o,
                              void* x, bool fp32, bool zero_x, hipStream_t st) {
  const hipError_t e = launch_sstep_half(d, gb, gu, o, x, fp32, zero_x, false, st);
  if (e != hipSuccess) return e;
  return launch_sstep_half(d, gb, gu, o, x, fp32, zero_x, true, st);
}

hipError_t launch_sstep_batch(const SweepLaunch& L, int nt, bool rows, bool fp32, bool first,
                              bool update, hipStream_t st) {
  if (L.count < 1 || L.nwg_total < 1) return hipErrorInvalidValue;
  if (fp32) {
    if (first) return update ? sstep_batch_ppt<float, true, true>(L, nt, rows, st)
                             : sstep_batch_ppt<float, true, false>(L, nt, rows, st);
    return update ? sstep_batch_ppt<float, false, true>(L, nt, rows, st)
                  : sstep_batch_ppt<float, false, false>(L, nt, rows, st);
  }
  if (first) return update ? sstep_batch_ppt<double, true, true>(L, nt, rows, st)
                           : sstep_batch_ppt<double, true, false>(L, nt, rows, st);
  return update ? sstep_batch_ppt<double, false, true>(L, nt, rows, st)
                : sstep_batch_ppt<double, false, false>(L, nt, rows, st);
}

// Wavefront-row shapes with an instantiation whose LDS fits.
static bool sstep_zv_shape_ok(const SweepGeom& g, bool fp32) {
  return g.N == 64 * g.ppt && zv_class_ok(g.ppt, g.zv, fp32) && g.zv - 2 <= g.N &&
         sstep_lds_bytes(g, fp32) <= 160 * 1024 - 2048;
}

// Update-kernel shapes with an instantiation: 256 threads in every class;
// 512 threads with 2 or 4 points per thread and at most two halo slots.
bool sstep_update_shape_ok(const SweepGeom& g, bool fp32) {
  if (g.zv) return false;
  const int nt = g.S / g.ppt;
  const int nh = sweep_nh_class(g.nh);
  if (nh == 0 || sstep_lds_bytes(g, fp32) > 160 * 1024 - 2048) return false;
  if (nt == kThreads) return g.ppt == 1 || g.ppt == 2 || g.ppt == 4;
  return nt == 512 && nh <= 2 && (g.ppt == 2 || g.ppt == 4);
}

// Basis-kernel shapes that compile without register spills: 256 threads in
// every class; 512 threads with 2 or 4 points per thread (FP32) or 2 (FP64)
// and at most two halo slots; 1024 threads for FP32 up to 4 points per
// thread with one halo slot (2 points with two), and for FP64 up to 2
// points with one halo slot (1 point with two).
bool sstep_basis_shape_ok(const SweepGeom& g, bool fp32) {
  if (g.zv) return sstep_zv_shape_ok(g, fp32);
  const int nt = g.S / g.ppt;
  const int nh = sweep_nh_class(g.nh);
  if (nh == 0 || sstep_lds_bytes(g, fp32) > 160 * 1024 - 2048) return false;
  if (nt == kThreads) return g.ppt == 1 || g.ppt == 2 || g.ppt == 4;
  if (nt == 512) return nh <= 2 && (g.ppt == 2 || (fp32 && g.ppt == 4));
  if (nt != 1024 || nh > 2) return false;
  if (fp32) return g.ppt == 1 || g.ppt == 2 || (g.ppt == 4 && nh == 1);
  return g.ppt == 1 || (g.ppt == 2 && nh == 1);
}

}  // namespace maze
