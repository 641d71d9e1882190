// Molecular-dynamics driver kernels around the MaZe step: velocity Verlet
// for the ions (Section 2) and the Born-Huggins-Mayer short-range term with
// the electrostatic part removed (Results section). Not part of the
// electrostatic hot path; they make a full device-resident MD step.
//
// Scratch layout (md.scratch_dev): [0, 3n) positions before the drift,
// [3n, 6n) electrostatic forces before the drift, then per-workgroup
// partials: 5 slots of `nb` doubles (short-range energy, kinetic energy,
// work increment, unused, unused) followed by 3*nb momentum partials.
#include "device_util.h"

namespace maze {

struct MdParams {
  int n;
  double dt, accel, cutoff, box, inv_box;
  double tab[15];
};

static MdParams md_params(const maze_md_state& md, double box) {
  MdParams p;
  p.n = md.n_ions;
  p.dt = md.dt;
  p.accel = md.accel;
  p.cutoff = md.cutoff;
  p.box = box;
  p.inv_box = 1.0 / box;
  for (int i = 0; i < 15; ++i) p.tab[i] = md.bmh_table[i];
  return p;
}

static int md_blocks(int n) { return (n + kThreads - 1) / kThreads; }

__device__ __forceinline__ double bmh_v(const double* row, double r) {
  const double r2 = r * r, r6 = r2 * r2 * r2, r8 = r6 * r2;
  return row[0] * exp(row[1] * (row[2] - r)) - row[3] / r6 - row[4] / r8;
}

__device__ __forceinline__ double bmh_dvdr(const double* row, double r) {
  const double r2 = r * r, r7 = r2 * r2 * r2 * r, r9 = r7 * r2;
  return -row[0] * row[1] * exp(row[1] * (row[2] - r)) + 6.0 * row[3] / r7 + 8.0 * row[4] / r9;
}

// Short range: one thread per ion i, all j streamed through LDS in tiles.
// Minimum image, cutoff, energy shifted to zero at the cutoff. Each pair is
// evaluated from both sides (force on i only), so no atomics are needed;
// the energy counts each pair once (j > i).
__global__ __launch_bounds__(kThreads) void k_md_bmh(MdParams p, const double* __restrict__ pos,
                                                     const int32_t* __restrict__ species,
                                                     double* __restrict__ f_sr, double* part_e) {
  __shared__ double sx[kThreads], sy[kThreads], sz[kThreads];
  __shared__ int ss[kThreads];
  __shared__ double red[8];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const bool act = i < p.n;
  double xi = 0, yi = 0, zi = 0;
  int si = 0;
  if (act) {
    xi = pos[3 * i];
    yi = pos[3 * i + 1];
    zi = pos[3 * i + 2];
    si = species[i];
  }
  double vshift[3];
  for (int t = 0; t < 3; ++t) vshift[t] = bmh_v(p.tab + 5 * t, p.cutoff);
  const double rc2 = p.cutoff * p.cutoff;
  double fx = 0, fy = 0, fz = 0, e = 0;
  for (int base = 0; base < p.n; base += kThreads) {
    const int j = base + threadIdx.x;
    __syncthreads();
    if (j < p.n) {
      sx[threadIdx.x] = pos[3 * j];
      sy[threadIdx.x] = pos[3 * j + 1];
      sz[threadIdx.x] = pos[3 * j + 2];
      ss[threadIdx.x] = species[j];
    }
    __syncthreads();
    const int m = min(kThreads, p.n - base);
    if (act) {
      for (int k = 0; k < m; ++k) {
        const int jj = base + k;
        if (jj == i) continue;
        double dx = xi - sx[k], dy = yi - sy[k], dz = zi - sz[k];
        dx -= p.box * rint(dx * p.inv_box);
        dy -= p.box * rint(dy * p.inv_box);
        dz -= p.box * rint(dz * p.inv_box);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= rc2) continue;
        const double r = sqrt(r2);
        const int t = si + ss[k];
        const double* row = p.tab + 5 * t;
        const double f = -bmh_dvdr(row, r) / r;
        fx += f * dx;
        fy += f * dy;
        fz += f * dz;
        if (jj > i) e += bmh_v(row, r) - vshift[t];
      }
    }
  }
  if (act) {
    f_sr[3 * i] = fx;
    f_sr[3 * i + 1] = fy;
    f_sr[3 * i + 2] = fz;
  }
  const double te = block_sum(e, red);
  if (threadIdx.x == 0) part_e[blockIdx.x] = te;
}

// First half kick and drift; remembers the positions and electrostatic
// forces before the drift for the work integral.
__global__ __launch_bounds__(kThreads) void k_md_kick_drift(MdParams p, double* pos, double* vel,
                                                            const double* __restrict__ mass,
                                                            const double* __restrict__ f_es,
                                                            const double* __restrict__ f_sr,
                                                            double* x_old, double* f_old) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= p.n) return;
  const double c = 0.5 * p.dt * p.accel / mass[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int k = 3 * i + d;
    const double v = vel[k] + c * (f_es[k] + f_sr[k]);
    vel[k] = v;
    x_old[k] = pos[k];
    f_old[k] = f_es[k];
    pos[k] = pos[k] + p.dt * v;
  }
}

// Second half kick, kinetic energy, momentum and the trapezoid work of the
// electrostatic force (equation "E_nostra").
__global__ __launch_bounds__(kThreads) void k_md_kick2(MdParams p, const double* pos, double* vel,
                                                       const double* __restrict__ mass,
                                                       const double* __restrict__ f_es,
                                                       const double* __restrict__ f_sr,
                                                       const double* x_old, const double* f_old,
                                                       int do_kick, double* part, int nb) {
  __shared__ double red[8];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  double ke = 0, w = 0, px = 0, py = 0, pz = 0;
  if (i < p.n) {
    const double m = mass[i];
    const double c = 0.5 * p.dt * p.accel / m;
    double v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int k = 3 * i + d;
      v[d] = vel[k];
      if (do_kick) {
        v[d] += c * (f_es[k] + f_sr[k]);
        vel[k] = v[d];
        w += 0.5 * (f_old[k] + f_es[k]) * (pos[k] - x_old[k]);
      }
    }
    ke = 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / p.accel;
    px = m * v[0];
    py = m * v[1];
    pz = m * v[2];
  }
  const double t0 = block_sum(ke, red);
  const double t1 = block_sum(w, red);
  const double t2 = block_sum(px, red);
  const double t3 = block_sum(py, red);
  const double t4 = block_sum(pz, red);
  if (threadIdx.x == 0) {
    part[1 * nb + blockIdx.x] = t0;
    part[2 * nb + blockIdx.x] = t1;
    part[5 * nb + blockIdx.x] = t2;
    part[6 * nb + blockIdx.x] = t3;
    part[7 * nb + blockIdx.x] = t4;
  }
}

__global__ __launch_bounds__(kThreads) void k_md_finish(const double* part, int nb, int prime,
                                                        double* scalars) {
  __shared__ double red[8];
  const double e_sr = sum_partials(part + 0 * nb, nb, red);
  const double ke = sum_partials(part + 1 * nb, nb, red);
  const double w = sum_partials(part + 2 * nb, nb, red);
  const double px = sum_partials(part + 5 * nb, nb, red);
  const double py = sum_partials(part + 6 * nb, nb, red);
  const double pz = sum_partials(part + 7 * nb, nb, red);
  if (threadIdx.x == 0) {
    scalars[0] = prime ? 0.0 : scalars[0] - w;
    scalars[1] = e_sr;
    scalars[2] = ke;
    scalars[3] = px;
    scalars[4] = py;
    scalars[5] = pz;
  }
}

hipError_t launch_md_kick_drift(const maze_md_state& md, hipStream_t st) {
  MdParams p = md_params(md, 1.0);
  const int n = md.n_ions;
  hipLaunchKernelGGL(k_md_kick_drift, dim3(md_blocks(n)), dim3(kThreads), 0, st, p, md.pos_dev,
                     md.vel_dev, md.mass_dev, (const double*)md.f_es_dev,
                     (const double*)md.f_sr_dev, md.scratch_dev, md.scratch_dev + 3 * (size_t)n);
  return hipGetLastError();
}

hipError_t launch_md_bmh(const maze_md_state& md, double box, hipStream_t st) {
  MdParams p = md_params(md, box);
  const int n = md.n_ions;
  hipLaunchKernelGGL(k_md_bmh, dim3(md_blocks(n)), dim3(kThreads), 0, st, p,
                     (const double*)md.pos_dev, md.species_dev, md.f_sr_dev,
                     md.scratch_dev + 6 * (size_t)n);
  return hipGetLastError();
}

static hipError_t md_finish(const maze_md_state& md, int do_kick, hipStream_t st) {
  MdParams p = md_params(md, 1.0);
  const int n = md.n_ions, nb = md_blocks(n);
  double* part = md.scratch_dev + 6 * (size_t)n;
  hipLaunchKernelGGL(k_md_kick2, dim3(nb), dim3(kThreads), 0, st, p, (const double*)md.pos_dev,
                     md.vel_dev, md.mass_dev, (const double*)md.f_es_dev,
                     (const double*)md.f_sr_dev, (const double*)md.scratch_dev,
                     (const double*)(md.scratch_dev + 3 * (size_t)n), do_kick, part, nb);
  hipLaunchKernelGGL(k_md_finish, dim3(1), dim3(kThreads), 0, st, (const double*)part, nb,
                     do_kick ? 0 : 1, md.scalars_dev);
  return hipGetLastError();
}

hipError_t launch_md_finish(const maze_md_state& md, hipStream_t st) { return md_finish(md, 1, st); }
hipError_t launch_md_prime(const maze_md_state& md, hipStream_t st) { return md_finish(md, 0, st); }

}  // namespace maze
