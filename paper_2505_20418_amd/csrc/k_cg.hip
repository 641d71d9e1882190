// One fused sweep per iteration of the Jacobi PLCG solve of M y = sigma_p
// (Appendix B; equation "SHAKEy"), and of the direct Poisson solve
// (equation "linearproblem"), on FP64 or FP32 vectors.
//
// The solve is written for A = -M (symmetric positive definite on mean-zero
// vectors) with residual r = b - A x and the Jacobi preconditioner
// diag(A) = 6 I, i.e. z = r / 6. Hestenes-Stiefel PCG needs two global
// reductions per iteration: <p, A p> before the update of x and r, and
// <r, z> before the next search direction. This kernel uses the
// single-reduction rearrangement of D'Azevedo, Eijkhout and Romine (1992):
// with w = A p, the squared norm of the next residual is predicted from
// dots that are all available in the same sweep,
//
//   ||r - alpha w||^2 = ||r||^2 - 2 alpha <r, w> + alpha^2 <w, w>,
//
// so one sweep k (k >= 1) performs, per grid point,
//
//   w_{k-1} = A p_{k-1}                      (stencil of p_{k-1})
//   x_k     = x_{k-1} + alpha_{k-1} p_{k-1}
//   r_k     = r_{k-1} - alpha_{k-1} w_{k-1}
//   p_k     = r_k / 6 + beta_k p_{k-1}
//   w_k     = A p_k                          (stencil of p_k)
//
// and accumulates ||r_k||^2, max|r_k|, <p_k, w_k>, <r_k, w_k>, <w_k, w_k>.
// The next sweep turns those five sums into alpha_k = (||r_k||^2/6)/<p_k,w_k>
// and beta_{k+1} = ||r_{k+1}||^2_predicted / ||r_k||^2. In exact arithmetic
// the iterates are those of Hestenes-Stiefel PCG; the norm used by the
// stopping test is the directly computed ||r_k||, not the prediction.
//
// Neither w vector is stored: w_{k-1} is recomputed from p_{k-1}, which
// needs p_{k-1} two points away from the points whose p_k enters the stencil
// of w_k. Per point a sweep reads x, r, p and writes x, r, p once: 48 bytes
// in FP64 and 24 in FP32, against 64 / 32 for the two-pass form.
//
// Layout and marching: grids are N^3 with index (x*N + y)*N + z. A
// workgroup owns a segment of S = 256*PPT consecutive points of the
// flattened (y, z) plane and a run of consecutive x planes. It walks the
// planes in x order. Stage U at plane u produces r_k and p_k on the segment
// extended by N points (one row) on each side; stage W at plane u-1 forms
// w_k on the segment. The x neighbours live in registers; the y and z
// neighbours come from LDS copies of p_{k-1}(u) (segment plus two rows on
// each side) and p_k(u-1) (segment plus one row), both double-buffered so
// one barrier per plane suffices. Loads of the next plane are issued at the
// start of a step and consumed in the next one. r and p are double-buffered
// in HBM: neighbouring workgroups still read r_{k-1} and p_{k-1} at this
// workgroup's points while it writes r_k and p_k; x is updated in place
// (only its owner reads it).
//
// Reductions are atomic-free and deterministic: one partial per workgroup
// per sum, summed in a fixed order by every workgroup of the next sweep.
#include "device_util.h"

namespace maze {

SweepGeom make_sweep_geom(int N, int ppt, int cx) {
  SweepGeom g;
  g.N = N;
  g.P = N * N;
  g.ppt = ppt;
  g.S = kThreads * ppt;
  g.nseg = (g.P + g.S - 1) / g.S;
  g.cx = cx < 1 ? 1 : (cx > N ? N : cx);
  g.nchunk = (N + g.cx - 1) / g.cx;
  g.nwg = g.nseg * g.nchunk;
  g.nh = (2 * N + kThreads - 1) / kThreads;
  return g;
}

size_t sweep_lds_bytes(const SweepGeom& g, bool fp32, bool first) {
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  const size_t e1 = (size_t)g.S + 4 * (size_t)g.N, e2 = (size_t)g.S + 2 * (size_t)g.N;
  return es * (2 * e2 + (first ? 0 : 2 * e1));
}

// Five per-thread sums (index 1 is a max) reduced over the workgroup in a
// fixed order; every thread receives the results.
__device__ __forceinline__ void block_reduce5(double v[5], double* sm) {
#pragma unroll
  for (int i = 0; i < 5; ++i) v[i] = (i == 1) ? wave_max(v[i]) : wave_sum(v[i]);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < 5; ++i) sm[i * (kThreads / 64) + w] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double s = sm[i * (kThreads / 64)];
#pragma unroll
    for (int k = 1; k < kThreads / 64; ++k)
      s = (i == 1) ? fmax(s, sm[i * (kThreads / 64) + k]) : s + sm[i * (kThreads / 64) + k];
    v[i] = s;
  }
}

// Sums the partials of the previous kernel: ||r||^2, max|r| and (not FIRST)
// <p, w>, <r, w>, <w, w> of parity set `par`.
template <bool FIRST>
__device__ __forceinline__ void read_sweep_partials(const double* part, int ps, int par,
                                                    int nprev, double v[5], double* sm) {
  for (int i = 0; i < 5; ++i) v[i] = 0.0;
  const double* rr = part + (size_t)(SL_RR0 + par) * ps;
  const double* rm = part + (size_t)(SL_RMAX0 + par) * ps;
  const double* mu = part + (size_t)(SL_MU0 + par) * ps;
  const double* rw = part + (size_t)(SL_RW0 + par) * ps;
  const double* ww = part + (size_t)(SL_WW0 + par) * ps;
  for (int i = threadIdx.x; i < nprev; i += kThreads) {
    v[0] += rr[i];
    v[1] = fmax(v[1], rm[i]);
    if (!FIRST) {
      v[2] += mu[i];
      v[3] += rw[i];
      v[4] += ww[i];
    }
  }
  block_reduce5(v, sm);
}



__device__ __forceinline__ int wrap_plane(int u, int N) {
  return u < 0 ? u + N : (u >= N ? u - N : u);
}

// Plane p of a grid as a buffer resource: a scalar descriptor (base of the
// plane, its size in bytes) that loads and stores address with a 32-bit
// per-lane byte offset. Every address then takes one VGPR and no per-lane
// 64-bit arithmetic, and an offset past the plane reads zero instead of
// touching other memory. The plane index passes through readfirstlane so
// the base stays scalar.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T* g, int p, size_t Ps) {
  const T* base = g + (size_t)__builtin_amdgcn_readfirstlane(p) * Ps;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, (int)(Ps * sizeof(T)),
                                           0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}
template <typename T>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t boff, T v) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, boff, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, v), r, boff, 0, 0);
}

// The work of one workgroup of a sweep: logical index L of the session's
// grid (L = 0 also writes the session's control scalars). Shared by the
// single-session and the batched kernels, so a session gets bitwise the same
// result alone and in a batch.
template <typename T, bool FIRST, int PPT, int NH>
__device__ __forceinline__ void sweep_wg(const SweepArgs<T>& a, const SweepGeom& g, int par,
                                         int L, unsigned char* smem_raw, double* red) {
  Scalars* sc = a.sc;
  if (wg_flags_set(&sc->done, &sc->err, reinterpret_cast<int32_t*>(red))) return;
  const int tid = threadIdx.x;
  const bool leader = (L == 0) && (tid == 0);
  // buffers by parity, selected rather than indexed (an indexed copy of the
  // batched arguments would live in scratch)
  const T* r_in = par ? a.r[1] : a.r[0];
  T* r_out = par ? a.r[0] : a.r[1];
  const T* p_in = par ? a.p[1] : a.p[0];
  T* p_out = par ? a.p[0] : a.p[1];
  // number of updates done so far in this solve; a per-parity counter, so
  // the leader's write for the next sweep never races with this sweep's reads
  const int it = ctl_ld(&sc->itp[par]);

  // ---- step scalars from the previous kernel's partials -------------------
  T alpha = (T)0, beta = (T)0;
  {
    double v[5];
    read_sweep_partials<FIRST>(a.part, a.pstride, par, FIRST ? a.nprev_first : a.nprev_sweep, v,
                               red);
    const double gam = v[0];
    const double thr = ctl_ld(&sc->thr);
    const bool conv = (ctl_ld(&sc->norm) == MAZE_NORM_ABSMAX) ? (v[1] <= thr) : (sqrt(gam) <= thr);
    if (leader && it < a.hist_cap) a.hist[it] = sqrt(gam);
    bool stop = conv || !isfinite(gam);
    int code = conv ? 1 : 2;
    // iteration cap: this sweep would perform update it + 1
    if (!FIRST && !stop && it >= ctl_ld(&sc->max_iter)) {
      stop = true;
      code = 3;
    }
    if (!FIRST && !stop) {
      const double mu = v[2];
      if (!(mu > 0.0) || !isfinite(mu)) {
        stop = true;
        code = 2;
      } else {
        const double al = gam / (6.0 * mu);
        const double gnext = gam - 2.0 * al * v[3] + al * al * v[4];
        alpha = (T)al;
        beta = (T)((gnext > 0.0) ? gnext / gam : 0.0);
      }
    }
    if (stop) {
      if (leader) {
        ctl_st(&sc->gamma[par], gam);
        ctl_st(&sc->iters, it);
        ctl_st(&sc->done, code);
      }
      return;
    }
  }

  // ---- geometry of this workgroup -----------------------------------------
  const int N = g.N, P = g.P, S = g.S;
  const int seg = L % g.nseg, chunk = L / g.nseg;
  const int s0 = seg * S;
  const int x0 = chunk * g.cx, x1 = min(N, x0 + g.cx);
  const int E1 = S + 4 * N, E2 = S + 2 * N;
  T* P2 = reinterpret_cast<T*>(smem_raw);  // [2][E2] p_k of plane u-1 / u
  T* P1 = P2 + 2 * E2;                     // [2][E1] p_{k-1} of plane u (not FIRST)
  constexpr int NU = PPT + NH;             // stage-U slots: segment, then inner halo

  int off[NU], e1[NU], e1zm[NU], e1zp[NU], e2[NU];
  bool uval[NU];
  int e2zm[PPT], e2zp[PPT];
  bool cval[PPT];
  int offo[NH], e1o[NH];
  bool oval[NH];
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    int f, ee2;
    if (i < PPT) {
      const int loc = tid + i * kThreads;
      f = s0 + loc;
      ee2 = N + loc;
      uval[i] = true;
      cval[i] = f < P;
    } else {
      const int h = tid + (i - PPT) * kThreads;
      uval[i] = h < 2 * N;
      const int hh = uval[i] ? h : 0;
      ee2 = (hh < N) ? hh : S + hh;
      f = s0 - N + ee2;
    }
    int o = f % P;
    if (o < 0) o += P;
    off[i] = o;
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
    const int h = tid + k * kThreads;
    oval[k] = h < 2 * N;
    const int hh = oval[k] ? h : 0;
    e1o[k] = (hh < N) ? hh : S + 2 * N + hh;
    int o = (s0 - 2 * N + e1o[k]) % P;
    if (o < 0) o += P;
    offo[k] = o;
  }
  // byte offsets within a plane (below P * sizeof(T) <= 2^23)
  uint32_t bo[NU], boo[NH];
#pragma unroll
  for (int i = 0; i < NU; ++i) bo[i] = (uint32_t)off[i] * (uint32_t)sizeof(T);
#pragma unroll
  for (int k = 0; k < NH; ++k) boo[k] = (uint32_t)offo[k] * (uint32_t)sizeof(T);

  const T c6 = (T)(1.0 / 6.0);
  const size_t Ps = (size_t)P;
  T pm[NU], pc[NU], pn[NU], pon[NH];  // p_{k-1}: planes u-1, u, u+1; outer halo u+1
  T rc[NU], xc[PPT];                  // r_{k-1}, x_{k-1} at plane u
  T qm[PPT], qc[PPT], qn[PPT], sv[PPT];  // p_k at planes u-2, u-1, u; r_k at u-1
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

  // ---- prologue: planes x0-2 .. x0 of p_{k-1}, plane x0-1 of r_{k-1} ------
  {
    const auto r0 = plane_rsrc(r_in, wrap_plane(x0 - 1, N), Ps);
#pragma unroll
    for (int i = 0; i < NU; ++i) rc[i] = buf_ld<T>(r0, bo[i]);
    if (!FIRST) {
      const auto pa = plane_rsrc(p_in, wrap_plane(x0 - 2, N), Ps);
      const auto pb = plane_rsrc(p_in, wrap_plane(x0 - 1, N), Ps);
      const auto pd = plane_rsrc(p_in, wrap_plane(x0, N), Ps);
      T ob[NH];
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        pm[i] = buf_ld<T>(pa, bo[i]);
        pc[i] = buf_ld<T>(pb, bo[i]);
        pn[i] = buf_ld<T>(pd, bo[i]);
      }
#pragma unroll
      for (int k = 0; k < NH; ++k) {
        ob[k] = buf_ld<T>(pb, boo[k]);
        pon[k] = buf_ld<T>(pd, boo[k]);
      }
#pragma unroll
      for (int i = 0; i < NU; ++i)
        if (uval[i]) P1[e1[i]] = pc[i];
#pragma unroll
      for (int k = 0; k < NH; ++k)
        if (oval[k]) P1[e1o[k]] = ob[k];
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      xc[j] = (T)0;
      qm[j] = qc[j] = qn[j] = sv[j] = (T)0;
    }
  }
  __syncthreads();
  // Complete the prologue loads here: every value entering the loop is then
  // known to be resident, and the waits inside the loop only cover the loads
  // issued for the next step (which stay in flight across its compute).
  __builtin_amdgcn_s_waitcnt(0);

  const int nsteps = x1 - x0 + 2;  // stage U on planes x0-1 .. x1
  for (int t = 0; t < nsteps; ++t) {
    const int u = x0 - 1 + t;
    const bool more = t + 1 < nsteps;
    const bool own_u = (u >= x0) && (u < x1);
    const bool own_n = (u + 1 >= x0) && (u + 1 < x1);
    // issue the loads of the next step
    T pf[NU], pof[NH], rf[NU], xf[PPT];
    if (more) {
      const auto rp = plane_rsrc(r_in, wrap_plane(u + 1, N), Ps);
#pragma unroll
      for (int i = 0; i < NU; ++i) rf[i] = buf_ld<T>(rp, bo[i]);
      if (!FIRST) {
        const auto pp = plane_rsrc(p_in, wrap_plane(u + 2, N), Ps);
#pragma unroll
        for (int i = 0; i < NU; ++i) pf[i] = buf_ld<T>(pp, bo[i]);
#pragma unroll
        for (int k = 0; k < NH; ++k) pof[k] = buf_ld<T>(pp, boo[k]);
        if (own_n) {
          const auto xp = plane_rsrc((const T*)a.x, u + 1, Ps);
#pragma unroll
          for (int j = 0; j < PPT; ++j) xf[j] = buf_ld<T>(xp, bo[j]);
        }
      }
    }

    // stage U at plane u: r_k, p_k (segment + inner halo), x_k (segment)
    const int tb = t & 1;
    T* P1b = P1 + tb * E1;
    T* P2w = P2 + tb * E2;
    T rk[PPT], pk[PPT];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      T r_new, p_new;
      if (FIRST) {
        r_new = rc[i];
        p_new = c6 * r_new;
      } else {
        const T w = (T)6 * pc[i] - (((pm[i] + pn[i]) + (P1b[e1[i] - N] + P1b[e1[i] + N])) +
                                    (P1b[e1zm[i]] + P1b[e1zp[i]]));
        r_new = rc[i] - alpha * w;
        p_new = c6 * r_new + beta * pc[i];
      }
      if (uval[i]) P2w[e2[i]] = p_new;
      if (i < PPT) {
        rk[i] = r_new;
        pk[i] = p_new;
      }
    }
    if (own_u) {
      const auto ro = plane_rsrc((const T*)r_out, u, Ps);
      const auto po = plane_rsrc((const T*)p_out, u, Ps);
      const auto xo = plane_rsrc((const T*)a.x, u, Ps);
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        if (cval[j]) {
          buf_st<T>(ro, bo[j], rk[j]);
          buf_st<T>(po, bo[j], pk[j]);
          if (!FIRST) buf_st<T>(xo, bo[j], xc[j] + alpha * pc[j]);
          else if (a.zero_x) buf_st<T>(xo, bo[j], (T)0);
          const double rd = (double)rk[j];
          acc[0] += rd * rd;
          acc[1] = fmax(acc[1], fabs(rd));
        }
      }
    }

    // stage W at plane u-1: w_k = A p_k on the segment, dots
    if (t >= 2) {
      const T* P2r = P2 + (tb ^ 1) * E2;
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const T w = (T)6 * qc[j] - (((qm[j] + pk[j]) + (P2r[e2[j] - N] + P2r[e2[j] + N])) +
                                    (P2r[e2zm[j]] + P2r[e2zp[j]]));
        if (cval[j]) {
          const double wd = (double)w;
          acc[2] += (double)qc[j] * wd;
          acc[3] += (double)sv[j] * wd;
          acc[4] += wd * wd;
        }
      }
    }

    // stage p_{k-1} of plane u+1 for the next step
    if (!FIRST && more) {
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
      qm[j] = qc[j];
      qc[j] = pk[j];
      sv[j] = rk[j];
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        rc[i] = rf[i];
        if (!FIRST) {
          pm[i] = pc[i];
          pc[i] = pn[i];
          pn[i] = pf[i];
        }
      }
      if (!FIRST) {
#pragma unroll
        for (int k = 0; k < NH; ++k) pon[k] = pof[k];
        if (own_n) {
#pragma unroll
          for (int j = 0; j < PPT; ++j) xc[j] = xf[j];
        }
      }
    }
  }

  block_reduce5(acc, red);
  if (tid == 0) {
    const int po = par ^ 1;
    a.part[(size_t)(SL_RR0 + po) * a.pstride + L] = acc[0];
    a.part[(size_t)(SL_RMAX0 + po) * a.pstride + L] = acc[1];
    a.part[(size_t)(SL_MU0 + po) * a.pstride + L] = acc[2];
    a.part[(size_t)(SL_RW0 + po) * a.pstride + L] = acc[3];
    a.part[(size_t)(SL_WW0 + po) * a.pstride + L] = acc[4];
    if (L == 0) ctl_st(&sc->itp[par ^ 1], FIRST ? 0 : it + 1);
  }
}

template <typename T, bool FIRST, int PPT, int NH>
__global__ __launch_bounds__(kThreads) void k_cg_sweep(SweepArgs<T> a, SweepGeom g, int par) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[5 * (kThreads / 64)];
  sweep_wg<T, FIRST, PPT, NH>(a, g, par, xcd_remap(blockIdx.x, g.nwg), smem_raw, red);
}

// Batched sweep: the workgroups of `count` sessions in one launch. Session i
// owns workgroups [wg_begin[i], wg_begin[i+1]); sessions that have converged
// return at once. All sessions of a launch share T, PPT and NH.
template <typename T, bool FIRST, int PPT, int NH>
__global__ __launch_bounds__(kThreads) void k_cg_sweep_batch(const SweepArgs<T>* __restrict__ args,
                                                             const SweepGeom* __restrict__ geoms,
                                                             const int* __restrict__ wg_begin,
                                                             int count, int par) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[5 * (kThreads / 64)];
  const int b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wg_begin[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const SweepArgs<T> a = args[lo];
  const SweepGeom g = geoms[lo];
  sweep_wg<T, FIRST, PPT, NH>(a, g, par ^ a.par_flip, b - wg_begin[lo], smem_raw, red);
}

// Status of every session of a batch in one compact array: done, iters, err.
__global__ __launch_bounds__(kThreads) void k_batch_poll(Scalars* const* scs, int count,
                                                         int32_t* out) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= count) return;
  const Scalars* sc = scs[i];
  out[3 * i] = ctl_ld(&sc->done);
  out[3 * i + 1] = ctl_ld(&sc->iters);
  out[3 * i + 2] = ctl_ld(&sc->err);
}

// Copies the scalars of every session of a batch into one array.
__global__ __launch_bounds__(kThreads) void k_batch_scalars(Scalars* const* scs, int count,
                                                            Scalars* out) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const int32_t* src = reinterpret_cast<const int32_t*>(scs[i]);
  int32_t* dst = reinterpret_cast<int32_t*>(out + i);
  constexpr int nw = (int)(sizeof(Scalars) / sizeof(int32_t));
  for (int w = threadIdx.x; w < nw; w += kThreads) dst[w] = ctl_ld(src + w);
}

// ---- launch plumbing ---------------------------------------------------------
// Raises the dynamic LDS limit of a kernel once per process when a launch
// needs more than the default 64 KiB.
static hipError_t raise_lds(const void* fn, size_t lds, bool* raised) {
  if (lds <= 65536 || *raised) return hipSuccess;
  const hipError_t e =
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
  if (e == hipSuccess) *raised = true;
  return e;
}

template <typename T, bool FIRST, int PPT, int NH>
static hipError_t launch_t(const SweepLaunch& L, hipStream_t st) {
  if (!L.batch) {
    static bool raised = false;
    const size_t lds = sweep_lds_bytes(L.g, sizeof(T) == 4, FIRST);
    const hipError_t e = raise_lds((const void*)k_cg_sweep<T, FIRST, PPT, NH>, lds, &raised);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cg_sweep<T, FIRST, PPT, NH>), dim3(L.g.nwg), dim3(kThreads), lds, st,
                       *static_cast<const SweepArgs<T>*>(L.args), L.g, L.par);
  } else {
    static bool raised = false;
    const hipError_t e =
        raise_lds((const void*)k_cg_sweep_batch<T, FIRST, PPT, NH>, L.lds, &raised);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cg_sweep_batch<T, FIRST, PPT, NH>), dim3(L.nwg_total), dim3(kThreads),
                       L.lds, st, static_cast<const SweepArgs<T>*>(L.args), L.geoms, L.wg_begin,
                       L.count, L.par);
  }
  return hipGetLastError();
}

template <typename T, bool FIRST, int PPT>
static hipError_t launch_nh(const SweepLaunch& L, hipStream_t st) {
  switch (L.nh) {
    case 1: return launch_t<T, FIRST, PPT, 1>(L, st);
    case 2: return launch_t<T, FIRST, PPT, 2>(L, st);
    case 4: return launch_t<T, FIRST, PPT, 4>(L, st);
    case 8: return launch_t<T, FIRST, PPT, 8>(L, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, bool FIRST>
static hipError_t launch_ppt(const SweepLaunch& L, hipStream_t st) {
  switch (L.ppt) {
    case 1: return launch_nh<T, FIRST, 1>(L, st);
    case 2: return launch_nh<T, FIRST, 2>(L, st);
    case 4: return launch_nh<T, FIRST, 4>(L, st);
    default: return hipErrorInvalidValue;
  }
}

int sweep_nh_class(int nh) { return nh <= 1 ? 1 : nh <= 2 ? 2 : nh <= 4 ? 4 : nh <= 8 ? 8 : 0; }

hipError_t launch_sweep(const SweepLaunch& L, bool fp32, bool first, hipStream_t st) {
  if (fp32) return first ? launch_ppt<float, true>(L, st) : launch_ppt<float, false>(L, st);
  return first ? launch_ppt<double, true>(L, st) : launch_ppt<double, false>(L, st);
}

template <typename T>
SweepArgs<T> make_sweep_args(const DeviceState& d, T* x, int nprev_first, int nprev_sweep,
                             bool zero_x) {
  const size_t G = (size_t)d.G;
  SweepArgs<T> a{};
  if constexpr (sizeof(T) == 4) {
    a.r[0] = d.r32;
    a.r[1] = d.r32 + G;
    a.p[0] = d.p32;
    a.p[1] = d.p32 + G;
  } else {
    a.r[0] = d.r;
    a.r[1] = d.r + G;
    a.p[0] = d.p;
    a.p[1] = d.p + G;
  }
  a.x = x;
  a.part = d.part;
  a.sc = d.sc;
  a.hist = d.hist;
  a.pstride = d.part_stride;
  a.nprev_first = nprev_first;
  a.nprev_sweep = nprev_sweep;
  a.zero_x = zero_x ? 1 : 0;
  a.hist_cap = d.hist_cap;
  return a;
}
template SweepArgs<float> make_sweep_args<float>(const DeviceState&, float*, int, int, bool);
template SweepArgs<double> make_sweep_args<double>(const DeviceState&, double*, int, int, bool);

hipError_t launch_cg_sweep(const DeviceState& d, const SweepGeom& g, int k, int nprev_first,
                           void* x, bool fp32, bool zero_x, hipStream_t st) {
  // one partial per workgroup and slot: the shape must fit the buffer's rows
  if (g.nwg < 1 || g.nwg > d.part_stride) return hipErrorInvalidValue;
  SweepLaunch L{};
  L.batch = false;
  L.g = g;
  L.par = k & 1;
  L.ppt = g.ppt;
  L.nh = sweep_nh_class(g.nh);
  if (fp32) {
    const SweepArgs<float> a = make_sweep_args<float>(d, (float*)x, nprev_first, g.nwg, zero_x);
    L.args = &a;
    return launch_sweep(L, true, k == 0, st);
  }
  const SweepArgs<double> a = make_sweep_args<double>(d, (double*)x, nprev_first, g.nwg, zero_x);
  L.args = &a;
  return launch_sweep(L, false, k == 0, st);
}

// Deterministic, finite, non-smooth fill (used to time sweeps on real work
// before a session's buffers are cleared for its first solve).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_pattern(T* x, long long G) {
  const long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (g >= G) return;
  uint32_t h = (uint32_t)(g * 2654435761ull) ^ (uint32_t)(g >> 32);
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  x[g] = (T)((double)(h & 0xffffff) / 16777216.0 - 0.5);
}

hipError_t launch_fill_pattern(void* x, long long G, bool fp32, hipStream_t st) {
  const unsigned nb = (unsigned)((G + kThreads - 1) / kThreads);
  if (fp32) hipLaunchKernelGGL(k_fill_pattern<float>, dim3(nb), dim3(kThreads), 0, st, (float*)x, G);
  else hipLaunchKernelGGL(k_fill_pattern<double>, dim3(nb), dim3(kThreads), 0, st, (double*)x, G);
  return hipGetLastError();
}

hipError_t launch_batch_poll(Scalars* const* scs, int count, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_poll, dim3((count + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     scs, count, out);
  return hipGetLastError();
}

hipError_t launch_batch_scalars(Scalars* const* scs, int count, Scalars* out, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_scalars, dim3(count), dim3(64), 0, st, scs, count, out);
  return hipGetLastError();
}

}  // namespace maze
