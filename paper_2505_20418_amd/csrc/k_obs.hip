// Structural and transport observables of the Results section, and the
// Langevin noise as an entry point of its own.
//
// * maze_langevin_noise: the normal deviates one OVRVO half step draws.
// * maze_rdf_accumulate: pair-distance histograms for g_IJ(r). Tiles of
//   256 x 256 ion pairs; each workgroup histograms its tile in LDS (integer
//   atomics, so counts are exact and order-free) and adds the tile's counts
//   to the global histogram.
// * maze_tcf_*: velocity autocorrelation and mean squared displacement per
//   species over a ring of time origins; one workgroup per live origin and
//   sample, reduced in a fixed order.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "device_util.h"
#include "philox.h"

namespace maze {

namespace {

constexpr int kRdfMaxBins = 4096;

__global__ __launch_bounds__(kThreads) void k_langevin_noise(uint64_t seed, long long step,
                                                             int half, int n, double* out) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double z[3];
  langevin_normals(seed, step, half, i, z);
  out[3 * i] = z[0];
  out[3 * i + 1] = z[1];
  out[3 * i + 2] = z[2];
}

// Squared minimum-image distance, rounded as written: each product and sum
// on its own, no fused multiply-add (the bin of a pair is decided on it).
__device__ __forceinline__ double min_image_r2(const double* a, const double* b, double box) {
#pragma clang fp contract(off)
  double r2 = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double dx = b[d] - a[d];
    dx = dx - box * rint(dx / box);
    r2 = (d == 0) ? dx * dx : r2 + dx * dx;
  }
  return r2;
}

// Tile (bi, bj), bj >= bi, of 256 x 256 ion pairs. LDS: the squared edges,
// the tile's histogram (3 rows of nbins counters) and the j ions.
__global__ __launch_bounds__(kThreads) void k_rdf_tile(const double* __restrict__ pos,
                                                       const int32_t* __restrict__ species, int n,
                                                       double box, const double* __restrict__ edges2,
                                                       int nbins, unsigned long long* hist) {
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bj < bi) return;
  extern __shared__ __align__(16) unsigned char smem[];
  double* E = reinterpret_cast<double*>(smem);                 // nbins + 1
  double* pj = E + (nbins + 1);                                // 3 * kThreads
  int* sj = reinterpret_cast<int*>(pj + 3 * kThreads);         // kThreads
  unsigned* H = reinterpret_cast<unsigned*>(sj + kThreads);    // 3 * nbins
  const int tid = threadIdx.x;
  for (int b = tid; b <= nbins; b += kThreads) E[b] = edges2[b];
  for (int b = tid; b < 3 * nbins; b += kThreads) H[b] = 0u;
  const int j0 = bj * kThreads, j = j0 + tid;
  if (j < n) {
    pj[3 * tid] = pos[3 * j];
    pj[3 * tid + 1] = pos[3 * j + 1];
    pj[3 * tid + 2] = pos[3 * j + 2];
    sj[tid] = species[j] ? 1 : 0;  // any nonzero value counts as Cl
  }
  __syncthreads();
  const int i = bi * kThreads + tid;
  if (i < n) {
    const double pi[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    const int si = species[i] ? 1 : 0;
    const int jn = min(kThreads, n - j0);
    const double lo_e = E[0], hi_e = E[nbins];
    for (int t = 0; t < jn; ++t) {
      if (j0 + t <= i) continue;  // each pair once, i < j
      const double r2 = min_image_r2(pi, pj + 3 * t, box);
      if (!(r2 >= lo_e) || !(r2 < hi_e)) continue;
      int lo = 0, hi = nbins;  // E[lo] <= r2 < E[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (E[mid] <= r2) lo = mid;
        else hi = mid;
      }
      atomicAdd(&H[(si + sj[t]) * nbins + lo], 1u);
    }
  }
  __syncthreads();
  for (int b = tid; b < 3 * nbins; b += kThreads)
    if (H[b] != 0u) atomicAdd(&hist[b], (unsigned long long)H[b]);
}

// One workgroup per origin slot: the slot holds origin q (sample q*every),
// the latest origin with q mod slots == slot; lag = k - q*every. Adds the
// per-species sums of v(origin).v(k) and |r(k) - r(origin)|^2 to lag's row.
__global__ __launch_bounds__(kThreads) void k_tcf_accumulate(
    const double* __restrict__ pos, const double* __restrict__ vel,
    const double* __restrict__ opos, const double* __restrict__ ovel,
    const int32_t* __restrict__ species, int n, long long k, int every, int max_lag, int slots,
    double* sums) {
  __shared__ double red[8];
  const int s = blockIdx.x;
  const long long Q = k / every;
  if (Q < s) return;
  const long long q = Q - ((Q - s) % slots);
  const long long lag = k - q * every;
  if (lag > max_lag) return;
  const double* p0 = opos + (size_t)s * 3 * n;
  const double* v0 = ovel + (size_t)s * 3 * n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // VACF Na, VACF Cl, MSD Na, MSD Cl
  for (int i = threadIdx.x; i < n; i += kThreads) {
    double vv = 0.0, rr = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      vv += v0[3 * i + d] * vel[3 * i + d];
      const double dr = pos[3 * i + d] - p0[3 * i + d];
      rr += dr * dr;
    }
    const int c = species[i] ? 1 : 0;
    acc[c] += vv;
    acc[2 + c] += rr;
  }
  const int L = max_lag + 1;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double t = block_sum(acc[r], red);
    if (threadIdx.x == 0) sums[(size_t)r * L + lag] += t;
  }
}

__global__ __launch_bounds__(kThreads) void k_fill_zero(double* x, long long m) {
  const long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (g < m) x[g] = 0.0;
}

}  // namespace
}  // namespace maze

using namespace maze;

struct maze_tcf {
  int n = 0, max_lag = 0, every = 1, slots = 0, device = 0;
  long long k = 0;
  hipStream_t stream = nullptr;
  int32_t* species = nullptr;
  double* opos = nullptr;
  double* ovel = nullptr;
  double* sums = nullptr;
  std::vector<int64_t> counts;
};

#define OBS_TRY(x)                    \
  do {                                \
    if ((x) != hipSuccess) {          \
      (void)hipGetLastError();        \
      return MAZE_E_DEVICE;           \
    }                                 \
  } while (0)

extern "C" {

int maze_langevin_noise(uint64_t seed, int64_t step, int32_t half, int32_t n, double* out_dev,
                        void* stream) {
  if (n < 0 || (half != 0 && half != 1) || step < 0 || (n > 0 && !out_dev)) return MAZE_E_INVALID;
  if (n == 0) return MAZE_OK;
  hipLaunchKernelGGL(k_langevin_noise, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     (hipStream_t)stream, seed, (long long)step, (int)half, (int)n, out_dev);
  OBS_TRY(hipGetLastError());
  return MAZE_OK;
}

int maze_rdf_accumulate(const double* pos_dev, const int32_t* species_dev, int32_t n, double box,
                        const double* edges2_dev, int32_t nbins, uint64_t* hist_dev,
                        void* stream) {
  if (n < 0 || nbins < 1 || nbins > kRdfMaxBins || !(box > 0) || !std::isfinite(box) ||
      !edges2_dev || !hist_dev || (n > 0 && (!pos_dev || !species_dev)))
    return MAZE_E_INVALID;
  if (n < 2) return MAZE_OK;
  const int nb = (n + kThreads - 1) / kThreads;
  const size_t lds = sizeof(double) * ((size_t)nbins + 1 + 3 * kThreads) +
                     sizeof(int) * kThreads + sizeof(unsigned) * 3 * (size_t)nbins;
  if (lds > 64 * 1024) {
    static bool raised = false;
    if (!raised) {
      OBS_TRY(hipFuncSetAttribute((const void*)k_rdf_tile,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024));
      raised = true;
    }
  }
  hipLaunchKernelGGL(k_rdf_tile, dim3(nb, nb), dim3(kThreads), lds, (hipStream_t)stream, pos_dev,
                     species_dev, (int)n, box, edges2_dev, (int)nbins,
                     reinterpret_cast<unsigned long long*>(hist_dev));
  OBS_TRY(hipGetLastError());
  return MAZE_OK;
}

int maze_tcf_create(int32_t n, const int32_t* species_dev, int32_t max_lag, int32_t origin_every,
                    void* stream, maze_tcf** out) {
  if (!out) return MAZE_E_INVALID;
  *out = nullptr;
  if (n < 1 || !species_dev || max_lag < 0 || origin_every < 1) return MAZE_E_INVALID;
  maze_tcf* t = new (std::nothrow) maze_tcf;
  if (!t) return MAZE_E_OOM;
  t->n = n;
  t->max_lag = max_lag;
  t->every = origin_every;
  t->slots = max_lag / origin_every + 1;
  t->stream = (hipStream_t)stream;
  t->counts.assign((size_t)max_lag + 1, 0);
  if (hipGetDevice(&t->device) != hipSuccess) {
    (void)hipGetLastError();
    delete t;
    return MAZE_E_DEVICE;
  }
  const size_t per = sizeof(double) * 3 * (size_t)n * (size_t)t->slots;
  const size_t nsum = 4 * ((size_t)max_lag + 1);
  if (hipMalloc(&t->species, sizeof(int32_t) * (size_t)n) != hipSuccess ||
      hipMalloc(&t->opos, per) != hipSuccess || hipMalloc(&t->ovel, per) != hipSuccess ||
      hipMalloc(&t->sums, sizeof(double) * nsum) != hipSuccess) {
    (void)hipGetLastError();
    maze_tcf_destroy(t);
    return MAZE_E_OOM;
  }
  if (hipMemcpyAsync(t->species, species_dev, sizeof(int32_t) * (size_t)n,
                     hipMemcpyDeviceToDevice, t->stream) != hipSuccess) {
    (void)hipGetLastError();
    maze_tcf_destroy(t);
    return MAZE_E_DEVICE;
  }
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((nsum + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, t->stream, t->sums, (long long)nsum);
  if (hipGetLastError() != hipSuccess) {
    maze_tcf_destroy(t);
    return MAZE_E_DEVICE;
  }
  *out = t;
  return MAZE_OK;
}

int maze_tcf_sample(maze_tcf* t, const double* pos_dev, const double* vel_dev) {
  if (!t || !pos_dev || !vel_dev) return MAZE_E_INVALID;
  OBS_TRY(hipSetDevice(t->device));
  const long long k = t->k;
  const size_t bytes = sizeof(double) * 3 * (size_t)t->n;
  if (k % t->every == 0) {
    const long long slot = (k / t->every) % t->slots;
    OBS_TRY(hipMemcpyAsync(t->opos + (size_t)slot * 3 * t->n, pos_dev, bytes,
                           hipMemcpyDeviceToDevice, t->stream));
    OBS_TRY(hipMemcpyAsync(t->ovel + (size_t)slot * 3 * t->n, vel_dev, bytes,
                           hipMemcpyDeviceToDevice, t->stream));
  }
  hipLaunchKernelGGL(k_tcf_accumulate, dim3(t->slots), dim3(kThreads), 0, t->stream, pos_dev,
                     vel_dev, (const double*)t->opos, (const double*)t->ovel,
                     (const int32_t*)t->species, t->n, k, t->every, t->max_lag, t->slots, t->sums);
  OBS_TRY(hipGetLastError());
  // the same live-origin rule on the host, for the counts
  const long long Q = k / t->every;
  for (long long s = 0; s < t->slots && s <= Q; ++s) {
    const long long q = Q - ((Q - s) % t->slots);
    const long long lag = k - q * t->every;
    if (lag <= t->max_lag) t->counts[(size_t)lag] += 1;
  }
  t->k = k + 1;
  return MAZE_OK;
}

int maze_tcf_read(const maze_tcf* t, double* sums_host, int64_t* counts_host) {
  if (!t) return MAZE_E_INVALID;
  OBS_TRY(hipSetDevice(t->device));
  const size_t L = (size_t)t->max_lag + 1;
  if (sums_host) {
    OBS_TRY(hipMemcpyAsync(sums_host, t->sums, sizeof(double) * 4 * L, hipMemcpyDeviceToHost,
                           t->stream));
  }
  OBS_TRY(hipStreamSynchronize(t->stream));
  if (counts_host) std::memcpy(counts_host, t->counts.data(), sizeof(int64_t) * L);
  return MAZE_OK;
}

void maze_tcf_destroy(maze_tcf* t) {
  if (!t) return;
  (void)hipSetDevice(t->device);
  if (t->stream) (void)hipStreamSynchronize(t->stream);
  else (void)hipDeviceSynchronize();
  if (t->species) (void)hipFree(t->species);
  if (t->opos) (void)hipFree(t->opos);
  if (t->ovel) (void)hipFree(t->ovel);
  if (t->sums) (void)hipFree(t->sums);
  delete t;
}

}  // extern "C"
