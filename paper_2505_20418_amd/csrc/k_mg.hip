// Geometric multigrid V-cycle used as the preconditioner of the PLCG solve
// of M y = sigma_p (the multigrid of the Results section, "Performance and
// scaling": red-black Gauss-Seidel smoothing, 27-point full-weighting
// restriction, trilinear prolongation, and a conjugate-gradient solve on the
// coarsest grid).
//
// Level l has N_l = N / 2^l points per side and solves A_l x = b with
// A_l = c_l (6 I - sum of the six neighbours), c_l = 4^-l: the fine operator
// A = -M rediscretised at spacing 2^l h, in fine-grid units. One V-cycle
// maps a residual r to z = B r:
//
//   for each level going down: x = 0; red then black half-sweep (pre);
//                              residual; full-weighting restriction
//   coarsest level: CG to round-off, mean-zero projection
//   for each level going up:   trilinear prolongation of the coarse
//                              correction; black then red half-sweep (post)
//
// The post-smoother visits the colours in the reverse order of the
// pre-smoother and the restriction is 1/8 of the transpose of the
// prolongation, so B is symmetric and the outer CG stays a CG. Grids are
// N^3 with index (x*N + y)*N + z, z fastest; consecutive threads take
// consecutive z. The vector type T is double, or float for the FP32
// preconditioner of the mixed-precision path.
#include "device_util.h"

namespace maze {

__device__ __forceinline__ int wrapi(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

template <typename T> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };

// Red-black Gauss-Seidel half-sweep: points with (i + j + k) % 2 == color
// get x = (b / c + sum of neighbours) / 6. zero: x starts at zero, so the
// red points take b / (6 c) and the black points are cleared.
// Each thread takes two z-neighbours (k even, k + 1; N is even on every
// smoothed level), one of each colour: it updates the one of `color` and
// stores the pair whole, the other point with the value it read. Every
// thread does one update and every store covers whole cache lines; the
// point of the other colour is not changed by this half-sweep, so writing
// it back is harmless to the threads that read it as a neighbour.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mg_smooth(T* __restrict__ x,
                                                        const T* __restrict__ b, int N,
                                                        T inv_c, int color, int zero,
                                                        const Scalars* sc) {
  using T2 = typename Pair<T>::type;
  if (ctl_ld(&sc->done) != 0) return;
  const long long G2 = (long long)N * N * N / 2;
  const long long m = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (m >= G2) return;
  const long long g0 = 2 * m;
  const int k0 = (int)(g0 % N);
  const int j = (int)((g0 / N) % N);
  const int i = (int)(g0 / ((long long)N * N));
  const int d = (((i + j + k0) & 1) == color) ? 0 : 1;  // the point of `color`
  const T s6 = (T)(1.0 / 6.0);
  const T2 bp = *reinterpret_cast<const T2*>(b + g0);
  if (zero) {
    T2 o;
    o.x = (d == 0) ? bp.x * inv_c * s6 : (T)0;
    o.y = (d == 1) ? bp.y * inv_c * s6 : (T)0;
    *reinterpret_cast<T2*>(x + g0) = o;
    return;
  }
  T2 xp = *reinterpret_cast<const T2*>(x + g0);
  const int k = k0 + d;
  const long long NN = (long long)N * N;
  const long long bi = (long long)i * NN, bj = (long long)j * N;
  const T zm = (d == 0) ? x[bi + bj + wrapi(k0 - 1, N)] : xp.x;
  const T zp = (d == 0) ? xp.y : x[bi + bj + wrapi(k0 + 2, N)];
  const T nb = (x[(long long)wrapi(i - 1, N) * NN + bj + k] +
                x[(long long)wrapi(i + 1, N) * NN + bj + k]) +
               (x[bi + (long long)wrapi(j - 1, N) * N + k] +
                x[bi + (long long)wrapi(j + 1, N) * N + k]) +
               (zm + zp);
  const T bk = (d == 0) ? bp.x : bp.y;
  const T v = (bk * inv_c + nb) * s6;
  if (d == 0) xp.x = v;
  else xp.y = v;
  *reinterpret_cast<T2*>(x + g0) = xp;
}

// r = b - c (6 x - sum of neighbours)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mg_residual(const T* __restrict__ x,
                                                          const T* __restrict__ b,
                                                          T* __restrict__ r, int N, T c,
                                                          const Scalars* sc) {
  if (ctl_ld(&sc->done) != 0) return;
  const long long G = (long long)N * N * N;
  const long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (g >= G) return;
  const int k = (int)(g % N);
  const int j = (int)((g / N) % N);
  const int i = (int)(g / ((long long)N * N));
  const long long NN = (long long)N * N;
  const long long bi = (long long)i * NN, bj = (long long)j * N;
  const T nb = (x[(long long)wrapi(i - 1, N) * NN + bj + k] +
                x[(long long)wrapi(i + 1, N) * NN + bj + k]) +
               (x[bi + (long long)wrapi(j - 1, N) * N + k] +
                x[bi + (long long)wrapi(j + 1, N) * N + k]) +
               (x[bi + bj + wrapi(k - 1, N)] + x[bi + bj + wrapi(k + 1, N)]);
  r[g] = b[g] - c * ((T)6 * x[g] - nb);
}

// Full weighting: bc[I] = sum over d in {-1,0,1}^3 of w(d) r[2I + d],
// w = product of 1/2 (d = 0) and 1/4 (d = +-1) per axis (weights sum to 1).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mg_restrict(const T* __restrict__ r,
                                                          T* __restrict__ bc, int Nc,
                                                          const Scalars* sc) {
  if (ctl_ld(&sc->done) != 0) return;
  const long long Gc = (long long)Nc * Nc * Nc;
  const long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (g >= Gc) return;
  const int Nf = 2 * Nc;
  const int K = (int)(g % Nc);
  const int J = (int)((g / Nc) % Nc);
  const int I = (int)(g / ((long long)Nc * Nc));
  const long long NN = (long long)Nf * Nf;
  T acc = (T)0;
#pragma unroll
  for (int a = -1; a <= 1; ++a) {
    const T wa = a == 0 ? (T)0.5 : (T)0.25;
    const long long ba = (long long)wrapi(2 * I + a, Nf) * NN;
    T sb = (T)0;
#pragma unroll
    for (int bb = -1; bb <= 1; ++bb) {
      const T wb = bb == 0 ? (T)0.5 : (T)0.25;
      const long long bbase = ba + (long long)wrapi(2 * J + bb, Nf) * Nf;
      const T v = (T)0.25 * r[bbase + wrapi(2 * K - 1, Nf)] + (T)0.5 * r[bbase + 2 * K] +
                  (T)0.25 * r[bbase + wrapi(2 * K + 1, Nf)];
      sb += wb * v;
    }
    acc += wa * sb;
  }
  bc[g] = acc;
}

// Trilinear prolongation of the coarse correction, added to x.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mg_prolong(T* __restrict__ x,
                                                         const T* __restrict__ ec, int Nf,
                                                         const Scalars* sc) {
  if (ctl_ld(&sc->done) != 0) return;
  const long long G = (long long)Nf * Nf * Nf;
  const long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (g >= G) return;
  const int Nc = Nf / 2;
  const int k = (int)(g % Nf);
  const int j = (int)((g / Nf) % Nf);
  const int i = (int)(g / ((long long)Nf * Nf));
  int ia[2], ja[2], ka[2];
  T wi[2], wj[2], wk[2];
  ia[0] = i >> 1; ia[1] = wrapi((i >> 1) + 1, Nc);
  ja[0] = j >> 1; ja[1] = wrapi((j >> 1) + 1, Nc);
  ka[0] = k >> 1; ka[1] = wrapi((k >> 1) + 1, Nc);
  wi[0] = (i & 1) ? (T)0.5 : (T)1; wi[1] = (i & 1) ? (T)0.5 : (T)0;
  wj[0] = (j & 1) ? (T)0.5 : (T)1; wj[1] = (j & 1) ? (T)0.5 : (T)0;
  wk[0] = (k & 1) ? (T)0.5 : (T)1; wk[1] = (k & 1) ? (T)0.5 : (T)0;
  const long long NN = (long long)Nc * Nc;
  T acc = (T)0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const long long base = (long long)ia[a] * NN + (long long)ja[b] * Nc;
      acc += (wi[a] * wj[b]) * (wk[0] * ec[base + ka[0]] + wk[1] * ec[base + ka[1]]);
    }
  x[g] += acc;
}

// Coarsest level: one workgroup solves c (6 x - sum of neighbours) = b - mean(b)
// by CG in LDS (FP64) to round-off, then stores x - mean(x).
constexpr int kCoarseMax = 1728;  // 12^3

template <typename T>
__global__ __launch_bounds__(kThreads) void k_mg_coarse(T* __restrict__ xo,
                                                        const T* __restrict__ bi, int N,
                                                        double c, const Scalars* sc) {
  __shared__ double x[kCoarseMax], r[kCoarseMax], p[kCoarseMax], w[kCoarseMax];
  __shared__ double red[kThreads / 64];
  if (ctl_ld(&sc->done) != 0) return;
  const int G = N * N * N;
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int g = tid; g < G; g += kThreads) s += (double)bi[g];
  const double mean = block_sum(s, red) / (double)G;
  double rr = 0.0;
  for (int g = tid; g < G; g += kThreads) {
    const double v = (double)bi[g] - mean;
    x[g] = 0.0;
    r[g] = v;
    p[g] = v;
    rr += v * v;
  }
  rr = block_sum(rr, red);
  const double stop = rr * 1e-28;
  for (int it = 0; it < 4 * G && rr > stop && rr > 0.0; ++it) {
    __syncthreads();
    double pw = 0.0;
    for (int g = tid; g < G; g += kThreads) {
      const int k = g % N, j = (g / N) % N, i = g / (N * N);
      const double nb = p[wrapi(i - 1, N) * N * N + j * N + k] + p[wrapi(i + 1, N) * N * N + j * N + k] +
                        p[i * N * N + wrapi(j - 1, N) * N + k] + p[i * N * N + wrapi(j + 1, N) * N + k] +
                        p[i * N * N + j * N + wrapi(k - 1, N)] + p[i * N * N + j * N + wrapi(k + 1, N)];
      const double wv = c * (6.0 * p[g] - nb);
      w[g] = wv;
      pw += p[g] * wv;
    }
    pw = block_sum(pw, red);
    if (!(pw > 0.0)) break;
    const double al = rr / pw;
    double rn = 0.0;
    for (int g = tid; g < G; g += kThreads) {
      x[g] += al * p[g];
      r[g] -= al * w[g];
      rn += r[g] * r[g];
    }
    rn = block_sum(rn, red);
    const double be = rn / rr;
    rr = rn;
    for (int g = tid; g < G; g += kThreads) p[g] = r[g] + be * p[g];
  }
  __syncthreads();
  double xs = 0.0;
  for (int g = tid; g < G; g += kThreads) xs += x[g];
  const double xm = block_sum(xs, red) / (double)G;
  for (int g = tid; g < G; g += kThreads) xo[g] = (T)(x[g] - xm);
}

// FP64 residual rounded to the preconditioner's precision (level-0 input of
// an FP32 V-cycle).
__global__ __launch_bounds__(kThreads) void k_mg_round(const double* __restrict__ r,
                                                       float* __restrict__ b, long long G,
                                                       const Scalars* sc) {
  if (ctl_ld(&sc->done) != 0) return;
  const long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (g < G) b[g] = (float)r[g];
}

// Level 0 of an FP32 V-cycle: the FP64 residual rounded into b, and the
// first (zero-start, red) half-sweep of the pre-smoother in the same pass:
// x = b / (6 c) on red points, 0 on black, with the float arithmetic of
// k_mg_smooth, so the result is bitwise that of the two passes. One z-pair
// (k even, k + 1) per thread, as in k_mg_smooth; N is even.
__global__ __launch_bounds__(kThreads) void k_mg_round_zero(const double* __restrict__ r,
                                                            float* __restrict__ b,
                                                            float* __restrict__ x, int N,
                                                            float inv_c, const Scalars* sc) {
  if (ctl_ld(&sc->done) != 0) return;
  const long long G2 = (long long)N * N * N / 2;
  const long long m = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (m >= G2) return;
  const long long g0 = 2 * m;
  const int k0 = (int)(g0 % N);
  const int j = (int)((g0 / N) % N);
  const int i = (int)(g0 / ((long long)N * N));
  const int d = ((i + j + k0) & 1) == 0 ? 0 : 1;  // the red point of the pair
  const double2 rp = *reinterpret_cast<const double2*>(r + g0);
  float2 bp;
  bp.x = (float)rp.x;
  bp.y = (float)rp.y;
  *reinterpret_cast<float2*>(b + g0) = bp;
  const float s6 = (float)(1.0 / 6.0);
  float2 o;
  o.x = (d == 0) ? bp.x * inv_c * s6 : 0.0f;
  o.y = (d == 1) ? bp.y * inv_c * s6 : 0.0f;
  *reinterpret_cast<float2*>(x + g0) = o;
}

// <r, z> per workgroup into the partial slot SL_MGRZ.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mg_dot(const double* __restrict__ r,
                                                     const T* __restrict__ z, long long G,
                                                     double* part, const Scalars* sc) {
  __shared__ double red[kThreads / 64];
  if (ctl_ld(&sc->done) != 0) return;
  double s = 0.0;
  const long long base = (long long)blockIdx.x * kThreads * 4 + threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long long g = base + (long long)q * kThreads;
    if (g < G) s += r[g] * (double)z[g];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

static inline unsigned nblk(long long G) { return (unsigned)((G + kThreads - 1) / kThreads); }

template <typename T>
static hipError_t vcycle_t(const DeviceState& d, const MgHierarchy& m, const double* r,
                           void* z, hipStream_t st) {
  const int L = m.levels;
  T* const* X = reinterpret_cast<T* const*>(m.x);
  T* const* B = reinterpret_cast<T* const*>(m.b);
  T* const* R = reinterpret_cast<T* const*>(m.r);
  const T* b0;
  T* x0 = reinterpret_cast<T*>(z);
  // an FP32 hierarchy rounds the level-0 residual in the pass that starts
  // its pre-smoother (when level 0 is smoothed at all)
  const bool fused0 = sizeof(T) == sizeof(float) && L > 1;
  if (sizeof(T) == sizeof(double)) {
    b0 = reinterpret_cast<const T*>(r);
  } else if (fused0) {
    hipLaunchKernelGGL(k_mg_round_zero, dim3(nblk(m.G[0] / 2)), dim3(kThreads), 0, st, r,
                       reinterpret_cast<float*>(B[0]), reinterpret_cast<float*>(x0), m.N[0],
                       (float)(1.0 / m.c[0]), (const Scalars*)d.sc);
    b0 = B[0];
  } else {
    hipLaunchKernelGGL(k_mg_round, dim3(nblk(m.G[0])), dim3(kThreads), 0, st, r,
                       reinterpret_cast<float*>(B[0]), m.G[0], (const Scalars*)d.sc);
    b0 = B[0];
  }
  auto xl = [&](int l) { return l == 0 ? x0 : X[l]; };
  auto bl = [&](int l) { return l == 0 ? b0 : (const T*)B[l]; };
  const Scalars* sc = d.sc;
  for (int l = 0; l + 1 < L; ++l) {
    const int N = m.N[l];
    const double c = m.c[l];
    if (!(l == 0 && fused0))
      hipLaunchKernelGGL(k_mg_smooth<T>, dim3(nblk(m.G[l] / 2)), dim3(kThreads), 0, st, xl(l),
                         bl(l), N, (T)(1.0 / c), 0, 1, sc);
    hipLaunchKernelGGL(k_mg_smooth<T>, dim3(nblk(m.G[l] / 2)), dim3(kThreads), 0, st, xl(l), bl(l),
                       N, (T)(1.0 / c), 1, 0, sc);
    hipLaunchKernelGGL(k_mg_residual<T>, dim3(nblk(m.G[l])), dim3(kThreads), 0, st,
                       (const T*)xl(l), bl(l), R[l], N, (T)c, sc);
    hipLaunchKernelGGL(k_mg_restrict<T>, dim3(nblk(m.G[l + 1])), dim3(kThreads), 0, st,
                       (const T*)R[l], B[l + 1], m.N[l + 1], sc);
  }
  const int lc = L - 1;
  hipLaunchKernelGGL(k_mg_coarse<T>, dim3(1), dim3(kThreads), 0, st, xl(lc), bl(lc), m.N[lc],
                     m.c[lc], sc);
  for (int l = L - 2; l >= 0; --l) {
    const int N = m.N[l];
    const double c = m.c[l];
    hipLaunchKernelGGL(k_mg_prolong<T>, dim3(nblk(m.G[l])), dim3(kThreads), 0, st, xl(l),
                       (const T*)xl(l + 1), N, sc);
    hipLaunchKernelGGL(k_mg_smooth<T>, dim3(nblk(m.G[l] / 2)), dim3(kThreads), 0, st, xl(l), bl(l),
                       N, (T)(1.0 / c), 1, 0, sc);
    hipLaunchKernelGGL(k_mg_smooth<T>, dim3(nblk(m.G[l] / 2)), dim3(kThreads), 0, st, xl(l), bl(l),
                       N, (T)(1.0 / c), 0, 0, sc);
  }
  return hipGetLastError();
}

hipError_t launch_mg_vcycle(const DeviceState& d, const MgHierarchy& m, const double* r, void* z,
                            bool fp32, hipStream_t st) {
  return fp32 ? vcycle_t<float>(d, m, r, z, st) : vcycle_t<double>(d, m, r, z, st);
}

int mg_dot_blocks(long long G) { return (int)((G + kThreads * 4 - 1) / (kThreads * 4)); }

hipError_t launch_mg_dot(const DeviceState& d, const double* r, const void* z, bool fp32,
                         hipStream_t st) {
  double* part = d.part + (size_t)SL_MGRZ * d.part_stride;
  if (fp32)
    hipLaunchKernelGGL(k_mg_dot<float>, dim3(mg_dot_blocks(d.G)), dim3(kThreads), 0, st, r,
                       (const float*)z, d.G, part, (const Scalars*)d.sc);
  else
    hipLaunchKernelGGL(k_mg_dot<double>, dim3(mg_dot_blocks(d.G)), dim3(kThreads), 0, st, r,
                       (const double*)z, d.G, part, (const Scalars*)d.sc);
  return hipGetLastError();
}

// Levels: halve while the grid stays even and the next grid has at least 4
// points per side; the coarsest grid must fit the one-workgroup solve.
int mg_plan(int N, int* Ns, int max_levels) {
  int L = 0;
  int n = N;
  Ns[L++] = n;
  while (L < max_levels && n % 2 == 0 && n / 2 >= 4) {
    n /= 2;
    Ns[L++] = n;
  }
  if ((long long)n * n * n > kCoarseMax) return 0;
  return L;
}

}  // namespace maze
