// Particle <-> grid kernels: binning of ions into grid tiles, atomic-free
// charge assignment, force interpolation, the field update of the MaZe
// step, and the single-workgroup finalisation of reductions.
//
// Charge assignment (Section 2.1, text after equation "F_nostra"):
// q_n = sum_a Q_a W(r_a - r_n), W the tensor product of 1-D weights of order
// 2 (linear, 8 points) or 4 (centred cubic B-spline, 64 points).
//
// Instead of scattering ion contributions with floating-point atomics, ions
// are counting-sorted into tiles of 8^3 grid points and each workgroup owns
// one tile of the grid: it walks the ions of the tiles whose support can
// reach it, in a fixed order, and every thread sums the contributions to its
// own grid points. Each grid value is written exactly once, and the sum
// order (tile order, then ion index) does not depend on scheduling, so the
// result is bitwise reproducible. Integer atomics only count and place ions;
// a per-tile sort by ion index makes the order canonical.
#include "device_util.h"

namespace maze {

// Periodic wrap of one coordinate and its split into a base cell and an
// offset, computed without FMA contraction so the cell decision is the same
// FP64 rounding sequence as a plain C implementation: xw = x - L floor(x/L),
// u = xw / h, i0 = floor(u), t = u - i0.
__device__ __forceinline__ void cell_of(double x, double box, double h, int N, int* cell,
                                        double* t) {
#pragma clang fp contract(off)
  const double xw = x - box * floor(x / box);
  const double u = xw / h;
  const double fl = floor(u);
  *t = u - fl;
  long long i0 = (long long)fl % N;
  if (i0 < 0) i0 += N;
  *cell = (int)i0;
}

__device__ __forceinline__ double bspline3(double s) {
#pragma clang fp contract(off)
  const double a = fabs(s);
  if (a < 1.0) return 2.0 / 3.0 - a * a + a * a * a / 2.0;
  if (a < 2.0) {
    const double t = 2.0 - a;
    return t * t * t / 6.0;
  }
  return 0.0;
}

// 1-D weights for the order-p support starting at cell (order 2) or cell-1
// (order 4).
__device__ __forceinline__ void axis_weights(int order, double t, double* w) {
#pragma clang fp contract(off)
  if (order == 2) {
    w[0] = 1.0 - t;
    w[1] = t;
  } else {
    w[0] = bspline3(1.0 + t);
    w[1] = bspline3(t);
    w[2] = bspline3(1.0 - t);
    w[3] = bspline3(2.0 - t);
  }
}

__device__ __forceinline__ int tile_of(const int* c, int ntx) {
  return ((c[0] / kTile) * ntx + c[1] / kTile) * ntx + c[2] / kTile;
}

// ---- binning ----------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_bin_ions(const double* __restrict__ pos, int n,
                                                       double box, double h, int N, int ntx,
                                                       int32_t* ion_cell, double* ion_t,
                                                       int32_t* tile_count, Scalars* sc) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  if (!isfinite(x[0]) || !isfinite(x[1]) || !isfinite(x[2])) {
    ctl_st(&sc->err, 1);
    return;
  }
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double t;
    cell_of(x[d], box, h, N, &c[d], &t);
    ion_cell[3 * i + d] = c[d];
    ion_t[3 * i + d] = t;
  }
  atomicAdd(&tile_count[tile_of(c, ntx)], 1);
}

// Exclusive scan of the tile counts (one workgroup; each thread scans a
// contiguous chunk), cursor = start, counts reset to zero for the next step.
// Exclusive scan of the tile counts into tile starts (and cursors), which
// also clears the counts for the next binning. One workgroup of 1024
// threads walks the tiles in chunks of 4096: each thread takes four
// consecutive counts, a wavefront scan and the 16 wavefront totals give its
// offset, and a carry runs across chunks. Integer sums, so any order gives
// the same starts.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void k_bin_scan(int32_t* tile_count,
                                                           int32_t* tile_start,
                                                           int32_t* tile_cursor, int ntiles,
                                                           const Scalars* sc) {
  constexpr int W = kScanThreads / 64;
  __shared__ int32_t wsum[W];
  if (ctl_ld(&sc->err)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int32_t carry = 0;
  for (int c0 = 0; c0 < ntiles; c0 += 4 * kScanThreads) {
    int32_t v[4];
    int32_t own = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = c0 + 4 * tid + k;
      v[k] = (i < ntiles) ? tile_count[i] : 0;
      own += v[k];
    }
    int32_t x = own;  // inclusive scan over the wavefront
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      before += (k < w) ? wsum[k] : 0;
      total += wsum[k];
    }
    int32_t run = carry + before + (x - own);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = c0 + 4 * tid + k;
      if (i < ntiles) {
        tile_start[i] = run;
        tile_cursor[i] = run;
        tile_count[i] = 0;
      }
      run += v[k];
    }
    carry += total;
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (tid == 0) tile_start[ntiles] = carry;
}

__global__ __launch_bounds__(kThreads) void k_bin_scatter(int n, int ntx, const int32_t* ion_cell,
                                                          int32_t* tile_cursor, int32_t* sorted_idx,
                                                          const Scalars* sc) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n || ctl_ld(&sc->err)) return;
  const int c[3] = {ion_cell[3 * i], ion_cell[3 * i + 1], ion_cell[3 * i + 2]};
  const int slot = atomicAdd(&tile_cursor[tile_of(c, ntx)], 1);
  sorted_idx[slot] = i;
}

// One thread per tile: insertion sort of the tile's ions by index, then the
// tile-ordered copies of cell, weights and charge used by spread and gather.
__global__ __launch_bounds__(kThreads) void k_bin_sort(int ntiles, int order,
                                                       const int32_t* tile_start,
                                                       int32_t* sorted_idx,
                                                       const int32_t* ion_cell,
                                                       const double* ion_t, const double* Q,
                                                       int32_t* s_cell, double* s_w, double* s_Q,
                                                       const Scalars* sc) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= ntiles || ctl_ld(&sc->err)) return;
  const int b = tile_start[t], e = tile_start[t + 1];
  for (int i = b + 1; i < e; ++i) {
    const int32_t v = sorted_idx[i];
    int j = i - 1;
    while (j >= b && sorted_idx[j] > v) {
      sorted_idx[j + 1] = sorted_idx[j];
      --j;
    }
    sorted_idx[j + 1] = v;
  }
  for (int s = b; s < e; ++s) {
    const int ion = sorted_idx[s];
    s_Q[s] = Q[ion];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      s_cell[3 * s + d] = ion_cell[3 * ion + d];
      double w[kMaxOrder];
      axis_weights(order, ion_t[3 * ion + d], w);
      for (int m = 0; m < order; ++m) s_w[(3 * s + d) * order + m] = w[m];
    }
  }
}

hipError_t launch_bin(const DeviceState& d, const double* pos, hipStream_t st) {
  const int nb = (d.n_ions + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_bin_ions, dim3(nb), dim3(kThreads), 0, st, pos, d.n_ions, d.box, d.h,
                     d.N, d.ntx, d.ion_cell, d.ion_t, d.tile_count, d.sc);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kScanThreads), 0, st, d.tile_count, d.tile_start,
                     d.tile_cursor, d.ntiles, (const Scalars*)d.sc);
  hipLaunchKernelGGL(k_bin_scatter, dim3(nb), dim3(kThreads), 0, st, d.n_ions, d.ntx,
                     d.ion_cell, d.tile_cursor, d.sorted_idx, (const Scalars*)d.sc);
  const int nt = (d.ntiles + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_bin_sort, dim3(nt), dim3(kThreads), 0, st, d.ntiles, d.order,
                     d.tile_start, d.sorted_idx, d.ion_cell, d.ion_t, d.Q, d.s_cell, d.s_w,
                     d.s_Q, (const Scalars*)d.sc);
  return hipGetLastError();
}

// ---- charge assignment -------------------------------------------------------
// Candidate tiles along one axis whose ions can reach grid tile T. An ion with
// base cell c touches points c .. c+1 (order 2) or c-1 .. c+2 (order 4), mod
// N, so the points p of tile T receive from the cells p-1 .. p (order 2) or
// p-2 .. p+1 (order 4). Those cells are the tile's own, the one (order 2)
// or two (order 4) below its first point and, for order 4, the one above
// its last, each taken mod N: the candidates are the tiles holding these at
// most four cells. Where N leaves a last tile of a single plane, the two
// cells below point 0 lie in two different tiles, so neighbouring tile
// indices alone would miss one of them. The set is returned in ascending
// order, so the summation order is canonical. It depends on N and the order
// only: a session builds the table of it once (k_cand_table), since each
// workgroup of the assignment forming it anew, on the scalar unit of every
// wavefront, cost more than the assignment itself.
__device__ __forceinline__ int candidate_tiles(int T, int N, int order, int* out) {
  auto tile_of = [N](int c) {
    c = (c < 0) ? c + N : (c >= N ? c - N : c);
    return c / kTile;
  };
  const int first = T * kTile, last = min(first + kTile - 1, N - 1);
  int v0 = T, v1 = tile_of(first - 1), v2 = v1, v3 = v1;  // repeats are dropped below
  if (order != 2) {
    v2 = tile_of(first - 2);
    v3 = tile_of(last + 1);
  }
  auto order2 = [](int& a, int& b) {
    const int lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
  };
  order2(v0, v1);
  order2(v2, v3);
  order2(v0, v2);
  order2(v1, v3);
  order2(v1, v2);
  int n = 1;
  out[0] = v0;
  if (v1 != v0) out[n++] = v1;
  if (v2 != v1) out[n++] = v2;
  if (v3 != v2) out[n++] = v3;
  return n;
}

__global__ __launch_bounds__(kThreads) void k_cand_table(int ntx, int N, int order,
                                                         int32_t* __restrict__ tab) {
  const int T = blockIdx.x * kThreads + threadIdx.x;
  if (T >= ntx) return;
  int out[kMaxCandAxis];
  const int n = candidate_tiles(T, N, order, out);
  int32_t* row = tab + (size_t)T * (1 + kMaxCandAxis);
  row[0] = n;
#pragma unroll
  for (int k = 0; k < kMaxCandAxis; ++k) row[1 + k] = (k < n) ? out[k] : 0;
}

hipError_t launch_cand_table(const DeviceState& d, hipStream_t st) {
  if (!d.cand || d.ntx < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cand_table, dim3((d.ntx + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     d.ntx, d.N, d.order, d.cand);
  return hipGetLastError();
}

// One workgroup per tile of kTile^3 grid points. The ions of the candidate
// tiles are read cooperatively into LDS in batches, in the canonical order
// (candidate tiles in (x, y, z) order, ions in tile order). The first
// wavefront then takes them one at a time, a lane for each of the ion's
// order^3 support points, and adds the weights that land in this tile to an
// LDS copy of it: every point sums its contributions in that order, so the
// result is independent of scheduling (a wavefront's LDS accesses complete
// in order, and one ion's points are distinct since N >= 4 >= order). Each
// (ion, point) pair costs one lane, not one test per point per ion.
constexpr int kSpreadBatch = 128;
__global__ __launch_bounds__(kThreads) void k_spread(int N, int ntx, int order,
                                                     const int32_t* __restrict__ cand,
                                                     const int32_t* __restrict__ tile_start,
                                                     const int32_t* __restrict__ s_cell,
                                                     const double* __restrict__ s_w,
                                                     const double* __restrict__ s_Q,
                                                     double* __restrict__ q, double* part,
                                                     const Scalars* sc) {
#pragma clang fp contract(off)
  __shared__ double red[8];
  constexpr int kMaxCand = kMaxCandAxis * kMaxCandAxis * kMaxCandAxis;
  constexpr int kTilePts = kTile * kTile * kTile;
  __shared__ int32_t cstart[kMaxCand], cpre[kMaxCand + 1];
  __shared__ double lQ[kSpreadBatch];
  __shared__ int32_t lcell[kSpreadBatch * 3];
  __shared__ double lw[kSpreadBatch * 3 * kMaxOrder];
  __shared__ double lq[kTilePts];
  if (ctl_ld(&sc->err)) return;
  const int T = blockIdx.x;
  const int TX = T / (ntx * ntx), TY = (T / ntx) % ntx, TZ = T % ntx;
  const int32_t* cx = cand + (size_t)TX * (1 + kMaxCandAxis) + 1;
  const int32_t* cy = cand + (size_t)TY * (1 + kMaxCandAxis) + 1;
  const int32_t* cz = cand + (size_t)TZ * (1 + kMaxCandAxis) + 1;
  const int nx = cx[-1], ny = cy[-1], nz = cz[-1];
  const int ncand = nx * ny * nz;
  const int off = (order == 2) ? 0 : 1;
  const int tid = threadIdx.x;
  if (tid < ncand) {
    const int a = tid / (ny * nz), b = (tid / nz) % ny, c = tid % nz;
    const int ct = (cx[a] * ntx + cy[b]) * ntx + cz[c];
    cstart[tid] = tile_start[ct];
    cpre[tid + 1] = tile_start[ct + 1] - tile_start[ct];
  }
#pragma unroll
  for (int j = 0; j < kTilePts / kThreads; ++j) lq[tid + j * kThreads] = 0.0;
  __syncthreads();
  if (tid == 0) {
    cpre[0] = 0;
    for (int t = 0; t < ncand; ++t) cpre[t + 1] += cpre[t];
  }
  __syncthreads();
  const int total = cpre[ncand];

  // lane l of the first wavefront: support offset (dx, dy, dz) of an ion
  const int o2 = order * order;
  const bool lane_on = tid < o2 * order;
  const int dx = tid / o2, dy = (tid / order) % order, dz = tid % order;
  const int t0x = TX * kTile, t0y = TY * kTile, t0z = TZ * kTile;
  for (int base = 0; base < total; base += kSpreadBatch) {
    const int m = min(kSpreadBatch, total - base);
    if (tid < m) {
      const int k = base + tid;
      int t = 0;
      while (cpre[t + 1] <= k) ++t;
      const int s = cstart[t] + (k - cpre[t]);
      lQ[tid] = s_Q[s];
#pragma unroll
      for (int d = 0; d < 3; ++d) lcell[3 * tid + d] = s_cell[3 * s + d];
      for (int e = 0; e < 3 * order; ++e) lw[tid * 3 * kMaxOrder + e] = s_w[(size_t)3 * s * order + e];
    }
    __syncthreads();
    if (lane_on) {
      for (int i = 0; i < m; ++i) {
        int px = lcell[3 * i] - off + dx, py = lcell[3 * i + 1] - off + dy,
            pz = lcell[3 * i + 2] - off + dz;
        px = (px < 0) ? px + N : (px >= N ? px - N : px);
        py = (py < 0) ? py + N : (py >= N ? py - N : py);
        pz = (pz < 0) ? pz + N : (pz >= N ? pz - N : pz);
        const int lx = px - t0x, ly = py - t0y, lz = pz - t0z;
        if ((unsigned)lx < (unsigned)kTile && (unsigned)ly < (unsigned)kTile &&
            (unsigned)lz < (unsigned)kTile) {
          const double* w = lw + i * 3 * kMaxOrder;
          double v = lQ[i] * w[dx];
          v = v * w[order + dy];
          v = v * w[2 * order + dz];
          const int li = (lx * kTile + ly) * kTile + lz;
          lq[li] = lq[li] + v;
        }
      }
    }
    __syncthreads();  // the batch buffers are refilled next; the tile is complete
  }
  double local = 0.0;
#pragma unroll
  for (int j = 0; j < kTilePts / kThreads; ++j) {
    const int pt = tid + j * kThreads;
    const int gx = t0x + (pt >> 6), gy = t0y + ((pt >> 3) & 7), gz = t0z + (pt & 7);
    if (gx < N && gy < N && gz < N) {
      const double v = lq[pt];
      q[((long long)gx * N + gy) * N + gz] = v;
      local += v;
    }
  }
  const double tot = block_sum(local, red);
  if (tid == 0) part[T] = tot;
}

hipError_t launch_spread(const DeviceState& d, hipStream_t st) {
  hipLaunchKernelGGL(k_spread, dim3(d.ntiles), dim3(kThreads), 0, st, d.N, d.ntx, d.order,
                     d.cand, d.tile_start, d.s_cell, d.s_w, d.s_Q, d.q,
                     d.part + (size_t)SL_QSUM * d.part_stride, (const Scalars*)d.sc);
  return hipGetLastError();
}

// ---- force interpolation (equation "F_nostra") --------------------------------
// One thread per ion in tile order (neighbouring threads read neighbouring
// grid points); F_a = -k Q_a sum_n W(r_a - r_n) (phi_{n+e} - phi_{n-e}) / 2h.
__global__ __launch_bounds__(kThreads) void k_gather(int n, int N, int order, double h,
                                                     double coulomb_k,
                                                     const int32_t* __restrict__ sorted_idx,
                                                     const int32_t* __restrict__ s_cell,
                                                     const double* __restrict__ s_w,
                                                     const double* __restrict__ s_Q,
                                                     const double* __restrict__ phi,
                                                     double* __restrict__ forces,
                                                     const Scalars* sc) {
#pragma clang fp contract(off)
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= n || ctl_ld(&sc->err)) return;
  const int off = (order == 2) ? 0 : 1;
  int ix[kMaxOrder], iy[kMaxOrder], iz[kMaxOrder];
  int ixm[kMaxOrder], ixp[kMaxOrder], iym[kMaxOrder], iyp[kMaxOrder], izm[kMaxOrder],
      izp[kMaxOrder];
  const double* w = s_w + (size_t)3 * s * order;
  for (int m = 0; m < order; ++m) {
    auto wrap = [N](int v) { return v < 0 ? v + N : (v >= N ? v - N : v); };
    ix[m] = wrap(s_cell[3 * s] - off + m);
    iy[m] = wrap(s_cell[3 * s + 1] - off + m);
    iz[m] = wrap(s_cell[3 * s + 2] - off + m);
    ixm[m] = wrap(ix[m] - 1);
    ixp[m] = wrap(ix[m] + 1);
    iym[m] = wrap(iy[m] - 1);
    iyp[m] = wrap(iy[m] + 1);
    izm[m] = wrap(iz[m] - 1);
    izp[m] = wrap(iz[m] + 1);
  }
  const long long NN = (long long)N * N;
  const double two_h = 2.0 * h;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < order; ++a)
    for (int b = 0; b < order; ++b)
      for (int c = 0; c < order; ++c) {
        double W = w[a] * w[order + b];
        W = W * w[2 * order + c];
        const long long I = ix[a] * NN, J = (long long)iy[b] * N;
        const double dx = (phi[ixp[a] * NN + J + iz[c]] - phi[ixm[a] * NN + J + iz[c]]) / two_h;
        const double dy = (phi[I + (long long)iyp[b] * N + iz[c]] -
                           phi[I + (long long)iym[b] * N + iz[c]]) / two_h;
        const double dz = (phi[I + J + izp[c]] - phi[I + J + izm[c]]) / two_h;
        acc[0] += W * dx;
        acc[1] += W * dy;
        acc[2] += W * dz;
      }
  const int ion = sorted_idx[s];
  const double kq = -coulomb_k * s_Q[s];
  forces[3 * ion + 0] = kq * acc[0];
  forces[3 * ion + 1] = kq * acc[1];
  forces[3 * ion + 2] = kq * acc[2];
}

// ---- alternative force (equation "F_Benoit") --------------------------------
// F_a = -k Q_a sum_n grad W(r_a - r_n) phi_n: the derivative falls on the
// assignment weights instead of the potential. It is minus the gradient of
// the discrete energy of equation "energy_discr" (for the exact field) but
// does not conserve momentum; kept for the comparison of force estimators.
__device__ __forceinline__ double bspline3_deriv(double s) {
#pragma clang fp contract(off)
  const double a = fabs(s);
  const double sg = (s < 0.0) ? -1.0 : 1.0;
  if (a < 1.0) return sg * (-2.0 * a + 1.5 * a * a);
  if (a < 2.0) {
    const double t = 2.0 - a;
    return sg * (-0.5 * t * t);
  }
  return 0.0;
}

__global__ __launch_bounds__(kThreads) void k_gather_wg(int n, int N, int order, double h,
                                                        double coulomb_k,
                                                        const int32_t* __restrict__ sorted_idx,
                                                        const int32_t* __restrict__ s_cell,
                                                        const double* __restrict__ s_w,
                                                        const double* __restrict__ s_Q,
                                                        const double* __restrict__ ion_t,
                                                        const double* __restrict__ phi,
                                                        double* __restrict__ forces,
                                                        const Scalars* sc) {
#pragma clang fp contract(off)
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= n || ctl_ld(&sc->err)) return;
  const int ion = sorted_idx[s];
  const int off = (order == 2) ? 0 : 1;
  const double* w = s_w + (size_t)3 * s * order;
  double dw[3][kMaxOrder];
  int idx[3][kMaxOrder];
  for (int d = 0; d < 3; ++d) {
    const double t = ion_t[3 * ion + d];
    if (order == 2) {
      dw[d][0] = -1.0 / h;
      dw[d][1] = 1.0 / h;
    } else {
      dw[d][0] = bspline3_deriv(t + 1.0) / h;
      dw[d][1] = bspline3_deriv(t) / h;
      dw[d][2] = bspline3_deriv(t - 1.0) / h;
      dw[d][3] = bspline3_deriv(t - 2.0) / h;
    }
    for (int m = 0; m < order; ++m) {
      int v = s_cell[3 * s + d] - off + m;
      idx[d][m] = v < 0 ? v + N : (v >= N ? v - N : v);
    }
  }
  const long long NN = (long long)N * N;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < order; ++a)
    for (int b = 0; b < order; ++b)
      for (int c = 0; c < order; ++c) {
        const double v = phi[idx[0][a] * NN + (long long)idx[1][b] * N + idx[2][c]];
        acc[0] += dw[0][a] * w[order + b] * w[2 * order + c] * v;
        acc[1] += w[a] * dw[1][b] * w[2 * order + c] * v;
        acc[2] += w[a] * w[order + b] * dw[2][c] * v;
      }
  const double kq = -coulomb_k * s_Q[s];
  forces[3 * ion + 0] = kq * acc[0];
  forces[3 * ion + 1] = kq * acc[1];
  forces[3 * ion + 2] = kq * acc[2];
}

hipError_t launch_gather(const DeviceState& d, const double* phi, double coulomb_k,
                         double* forces, hipStream_t st) {
  const int nb = (d.n_ions + kThreads - 1) / kThreads;
  if (d.weight_gradient_force) {
    hipLaunchKernelGGL(k_gather_wg, dim3(nb), dim3(kThreads), 0, st, d.n_ions, d.N, d.order, d.h,
                       coulomb_k, d.sorted_idx, d.s_cell, d.s_w, d.s_Q, (const double*)d.ion_t,
                       phi, forces, (const Scalars*)d.sc);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_gather, dim3(nb), dim3(kThreads), 0, st, d.n_ions, d.N, d.order, d.h,
                     coulomb_k, d.sorted_idx, d.s_cell, d.s_w, d.s_Q, phi, forces,
                     (const Scalars*)d.sc);
  return hipGetLastError();
}

// ---- field update (equation "SHAKEPhiFinal") --------------------------------
// phi^{k+1} = (phi_p - mean phi_p) - (4 pi / h)(y - mean y), written over
// phi^{k-1}; y stored projected (warm start of the next step); partials of
// phi^{k+1} . (q - qbar) for the energy of equation "energy_discr".
constexpr int kElemPerThread = 4;

__global__ __launch_bounds__(kThreads) void k_update(long long G, const double* __restrict__ phik,
                                                     double* phikm1, double* y,
                                                     const double* __restrict__ q,
                                                     double* field_out, double c4,
                                                     double* part_e, double* part_s,
                                                     const Scalars* sc) {
  __shared__ double red[8];
  if (ctl_ld(&sc->err)) return;
  const double pbar = ctl_ld(&sc->pbar), ybar = ctl_ld(&sc->xbar), qbar = ctl_ld(&sc->qbar);
  double e = 0.0, s = 0.0;
  const long long base = (long long)blockIdx.x * kThreads * kElemPerThread + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kElemPerThread; ++j) {
    const long long g = base + (long long)j * kThreads;
    if (g < G) {
      const double php = 2.0 * phik[g] - phikm1[g];
      const double yv = y[g] - ybar;
      const double phn = (php - pbar) - c4 * yv;
      phikm1[g] = phn;
      y[g] = yv;
      if (field_out) field_out[g] = phn;
      e += phn * (q[g] - qbar);
      s += phn;
    }
  }
  const double te = block_sum(e, red);
  const double ts = block_sum(s, red);
  if (threadIdx.x == 0) {
    part_e[blockIdx.x] = te;
    part_s[blockIdx.x] = ts;
  }
}

int update_blocks(long long G) {
  return (int)((G + (long long)kThreads * kElemPerThread - 1) / ((long long)kThreads * kElemPerThread));
}

hipError_t launch_update(const DeviceState& d, double* field_out, hipStream_t st) {
  hipLaunchKernelGGL(k_update, dim3(update_blocks(d.G)), dim3(kThreads), 0, st, d.G,
                     (const double*)d.phi_cur, d.phi_prev, d.y, (const double*)d.q, field_out,
                     4.0 * M_PI / d.h, d.part + (size_t)SL_ENERGY * d.part_stride,
                     d.part + (size_t)SL_PHISUM * d.part_stride, (const Scalars*)d.sc);
  return hipGetLastError();
}

// Direct solve: x -= mean(x); optional field copy; energy partials.
__global__ __launch_bounds__(kThreads) void k_project(long long G, double* x,
                                                      const double* __restrict__ q,
                                                      double* field_out, double* part_e,
                                                      double* part_s, const Scalars* sc) {
  __shared__ double red[8];
  if (ctl_ld(&sc->err)) return;
  const double xbar = ctl_ld(&sc->xbar), qbar = ctl_ld(&sc->qbar);
  double e = 0.0, s = 0.0;
  const long long base = (long long)blockIdx.x * kThreads * kElemPerThread + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kElemPerThread; ++j) {
    const long long g = base + (long long)j * kThreads;
    if (g < G) {
      const double v = x[g] - xbar;
      x[g] = v;
      if (field_out) field_out[g] = v;
      e += v * (q[g] - qbar);
      s += v;
    }
  }
  const double te = block_sum(e, red);
  const double ts = block_sum(s, red);
  if (threadIdx.x == 0) {
    part_e[blockIdx.x] = te;
    part_s[blockIdx.x] = ts;
  }
}

hipError_t launch_project(const DeviceState& d, double* x, double* field_out, hipStream_t st) {
  hipLaunchKernelGGL(k_project, dim3(update_blocks(d.G)), dim3(kThreads), 0, st, d.G, x,
                     (const double*)d.q, field_out, d.part + (size_t)SL_ENERGY * d.part_stride,
                     d.part + (size_t)SL_PHISUM * d.part_stride, (const Scalars*)d.sc);
  return hipGetLastError();
}

// ---- finalisation of reductions (one workgroup) ------------------------------
__global__ __launch_bounds__(kThreads) void k_finalize(int mode, int count, long long G,
                                                       double tol, double param,
                                                       double coulomb_k, const double* part,
                                                       int pstride, Scalars* sc,
                                                       double* energy_out, int imax, int norm,
                                                       double* hist, int hist_cap) {
  __shared__ double red[8];
  auto slot = [&](int s) { return part + (size_t)s * pstride; };
  if (mode == FIN_QSUM) {
    const double s = sum_partials(slot(SL_QSUM), count, red);
    if (threadIdx.x == 0) {
      ctl_st(&sc->qsum, s);
      ctl_st(&sc->qbar, s / (double)G);
    }
  } else if (mode == FIN_SOLVE_START) {
    const double qq = sum_partials(slot(SL_QQ), count, red);
    const double pp = sum_partials(slot(SL_PHIP), count, red);
    const double trr = sum_partials(slot(SL_TRR), count, red);
    const double tmx = max_partials(slot(SL_TMAX), count, red);
    if (threadIdx.x == 0) {
      ctl_st(&sc->norm, norm);
      ctl_st(&sc->max_iter, imax);
      ctl_st(&sc->qnorm, sqrt(qq));
      ctl_st(&sc->thr, (norm == MAZE_NORM_ABSMAX) ? tol : tol * sqrt(qq));
      ctl_st(&sc->pbar, pp / (double)G);
      ctl_st(&sc->true_rr, trr);
      ctl_st(&sc->true_max, tmx);
      ctl_st(&sc->itp[0], 0);
      ctl_st(&sc->itp[1], 0);
      ctl_st(&sc->pend, 0);
      ctl_st(&sc->done, 0);
      ctl_st(&sc->iters, 0);
    }
  } else if (mode == FIN_SOLVE_END) {
    const double xs = sum_partials(slot(SL_XSUM), count, red);
    const double trr = sum_partials(slot(SL_TRR), count, red);
    const double tmx = max_partials(slot(SL_TMAX), count, red);
    if (threadIdx.x == 0) {
      ctl_st(&sc->xbar, xs / (double)G);
      ctl_st(&sc->true_rr, trr);
      ctl_st(&sc->true_max, tmx);
    }
  } else if (mode == FIN_ENERGY) {
    if (ctl_ld(&sc->err)) return;
    const double e = sum_partials(slot(SL_ENERGY), count, red);
    if (threadIdx.x == 0) {
      ctl_st(&sc->energy, 0.5 * coulomb_k * e);
      if (energy_out) *energy_out = 0.5 * coulomb_k * e;
    }
  } else if (mode == FIN_INNER_FIRST) {
    // The step's first inner solve decided on the device, as the host decides
    // the later ones: converged already if the true residual of the
    // right-hand side meets thr, else an inner tolerance of
    // max(tol * residual, param * thr) (tol, param: the reduction and margin
    // of the mixed refinement).
    if (threadIdx.x == 0) {
      const double thr = ctl_ld(&sc->thr);
      const double res = (ctl_ld(&sc->norm) == MAZE_NORM_ABSMAX) ? ctl_ld(&sc->true_max)
                                                                 : sqrt(ctl_ld(&sc->true_rr));
      ctl_st(&sc->thr_outer, thr);
      ctl_st(&sc->max_iter, imax);
      ctl_st(&sc->itp[0], 0);
      ctl_st(&sc->itp[1], 0);
      ctl_st(&sc->pend, 0);
      ctl_st(&sc->iters, 0);
      if (res <= thr) {
        ctl_st(&sc->done, 4);
      } else {
        const double a = tol * res, b = param * thr;
        ctl_st(&sc->thr, (a < b) ? b : a);
        ctl_st(&sc->done, 0);
      }
    }
  } else if (mode == FIN_INNER_START) {
    if (threadIdx.x == 0) {
      ctl_st(&sc->thr, param);
      ctl_st(&sc->max_iter, imax);
      ctl_st(&sc->itp[0], 0);
      ctl_st(&sc->itp[1], 0);
      ctl_st(&sc->pend, 0);
      ctl_st(&sc->done, 0);
      ctl_st(&sc->iters, 0);
    }
  } else if (mode >= FIN_MG_CHECK0) {
    // multigrid-preconditioned CG; itp[0] counts its iterations
    if (ctl_ld(&sc->done) != 0 || ctl_ld(&sc->err) != 0) return;
    if (mode == FIN_MG_RHO) {
      const double rho = sum_partials(slot(SL_MGRZ), count, red);
      if (threadIdx.x == 0) {
        const int it = ctl_ld(&sc->itp[0]);
        if (!(rho > 0.0) || !isfinite(rho)) {
          ctl_st(&sc->iters, it);
          ctl_st(&sc->done, 2);
          return;
        }
        ctl_st(&sc->mg_beta, it == 0 ? 0.0 : rho / ctl_ld(&sc->mg_rho));
        ctl_st(&sc->mg_rho, rho);
      }
    } else if (mode == FIN_MG_MU) {
      const double mu = sum_partials(slot(SL_MU0), count, red);
      if (threadIdx.x == 0) {
        if (!(mu > 0.0) || !isfinite(mu)) {
          ctl_st(&sc->iters, ctl_ld(&sc->itp[0]));
          ctl_st(&sc->done, 2);
          return;
        }
        ctl_st(&sc->mg_alpha, ctl_ld(&sc->mg_rho) / mu);
      }
    } else {
      const double gam = sum_partials(slot(SL_RR0), count, red);
      const double rmax = max_partials(slot(SL_RMAX0), count, red);
      if (threadIdx.x == 0) {
        const int it = ctl_ld(&sc->itp[0]) + (mode == FIN_MG_CONV ? 1 : 0);
        ctl_st(&sc->itp[0], it);
        if (it < hist_cap) hist[it] = sqrt(gam);
        const double thr = ctl_ld(&sc->thr);
        const bool conv = (ctl_ld(&sc->norm) == MAZE_NORM_ABSMAX) ? (rmax <= thr)
                                                                   : (sqrt(gam) <= thr);
        if (mode == FIN_MG_CHECK0) ctl_st(&sc->mg_beta, 0.0);
        if (conv || !isfinite(gam)) {
          ctl_st(&sc->iters, it);
          ctl_st(&sc->done, conv ? 1 : 2);
        } else if (it >= ctl_ld(&sc->max_iter)) {
          ctl_st(&sc->iters, it);
          ctl_st(&sc->done, 3);
        }
      }
    }
  }
}

hipError_t launch_finalize(const DeviceState& d, int mode, int count, double tol,
                           double param, double coulomb_k, double* energy_out, int imax,
                           int norm, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, st, mode, count, d.G, tol, param,
                     coulomb_k, (const double*)d.part, d.part_stride, d.sc, energy_out, imax,
                     norm, d.hist, d.hist_cap);
  return hipGetLastError();
}

// Mixed precision: x += e (FP64 accumulation of the FP32 correction).
__global__ __launch_bounds__(kThreads) void k_add_correction(long long G, double* x,
                                                             const float* __restrict__ e,
                                                             const Scalars* sc) {
  if (ctl_ld(&sc->err)) return;
  const long long base = (long long)blockIdx.x * kThreads * kElemPerThread + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kElemPerThread; ++j) {
    const long long g = base + (long long)j * kThreads;
    if (g < G) x[g] += (double)e[g];
  }
}

hipError_t launch_add_correction(const DeviceState& d, double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_add_correction, dim3(update_blocks(d.G)), dim3(kThreads), 0, st, d.G, x,
                     (const float*)d.e32, (const Scalars*)d.sc);
  return hipGetLastError();
}

}  // namespace maze
