// Molecular-dynamics driver kernels around the MaZe step: velocity Verlet
// for the ions (Section 2), its Langevin extension OVRVO for canonical runs
// (Results section), and the Born-Huggins-Mayer short-range term with the
// electrostatic part removed (Results section). Not part of the
// electrostatic hot path; they make a full device-resident MD step.
//
// Scratch layout (md.scratch_dev): [0, 3n) positions before the drift,
// [3n, 6n) electrostatic forces before the drift, then per-workgroup
// partials: 5 slots of `nb` doubles (unused, kinetic energy, work increment,
// unused, unused) followed by 3*nb momentum partials. The short-range
// energy partials go to the session's own buffer (DeviceState::md_epart).
#include <cmath>

#include "device_util.h"
#include "philox.h"

namespace maze {

struct MdParams {
  int n;
  int lgv;             // Langevin half steps on (gamma > 0)
  double dt, accel, cutoff, box, inv_box;
  double tab[15];
  double ou_a, ou_b2;  // v <- a v + sqrt(b2 / m) xi
  uint64_t seed;
  long long step;      // noise counter of this step
};

// The Ornstein-Uhlenbeck half step over dt/2: a = exp(-gamma dt / 2) and
// b2 = (1 - a^2) kT accel, so that sqrt(b2 / m) is the velocity spread
// [A/fs] that the half step adds for an ion of mass m [amu].
static MdParams md_params(const maze_md_state& md, double box, long long step = 0) {
  MdParams p;
  p.n = md.n_ions;
  p.dt = md.dt;
  p.accel = md.accel;
  p.cutoff = md.cutoff;
  p.box = box;
  p.inv_box = 1.0 / box;
  for (int i = 0; i < 15; ++i) p.tab[i] = md.bmh_table[i];
  p.lgv = md.gamma > 0.0 ? 1 : 0;
  p.ou_a = p.lgv ? std::exp(-md.gamma * md.dt / 2.0) : 1.0;
  p.ou_b2 = p.lgv ? (1.0 - p.ou_a * p.ou_a) * md.kT * md.accel : 0.0;
  p.seed = md.seed;
  p.step = step;
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

// Short range over the tiles of the MaZe binning (tiles of kTile^3 grid
// points, filled by the assignment of the step at the same positions): each
// ion visits the (2R+1)^3 tiles around its own, R tiles covering the cutoff.
// Eight lanes share one ion, each taking every eighth tile of the block in a
// fixed order, and the lanes' sums are combined by a fixed butterfly, so the
// result is deterministic. Energy counts each pair once (j > i) and is
// reduced per workgroup into e_part.
constexpr int kBmhLanes = 8;

struct BmhTiles {
  const int32_t* tile_start;
  const int32_t* sorted_idx;
  const int32_t* s_cell;
  int ntx;
  int R;
};

__global__ __launch_bounds__(kThreads) void k_md_bmh_tiles(MdParams p, BmhTiles t,
                                                           const double* __restrict__ pos,
                                                           const int32_t* __restrict__ species,
                                                           double* __restrict__ f_sr,
                                                           double* e_part) {
  __shared__ double red[8];
  const int gt = blockIdx.x * kThreads + threadIdx.x;
  const int s = gt / kBmhLanes, lane = gt % kBmhLanes;
  const bool act = s < p.n;
  double fx = 0, fy = 0, fz = 0, e = 0;
  int i = 0;
  if (act) {
    i = t.sorted_idx[s];
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    const int si = species[i];
    const int tx = t.s_cell[3 * s] / kTile, ty = t.s_cell[3 * s + 1] / kTile,
              tz = t.s_cell[3 * s + 2] / kTile;
    double vshift[3];
    for (int q = 0; q < 3; ++q) vshift[q] = bmh_v(p.tab + 5 * q, p.cutoff);
    const double rc2 = p.cutoff * p.cutoff;
    const int W = 2 * t.R + 1, ntot = W * W * W;
    for (int c = lane; c < ntot; c += kBmhLanes) {
      int ax = tx + c / (W * W) - t.R, ay = ty + (c / W) % W - t.R, az = tz + c % W - t.R;
      ax = (ax < 0) ? ax + t.ntx : (ax >= t.ntx ? ax - t.ntx : ax);
      ay = (ay < 0) ? ay + t.ntx : (ay >= t.ntx ? ay - t.ntx : ay);
      az = (az < 0) ? az + t.ntx : (az >= t.ntx ? az - t.ntx : az);
      const int ct = (ax * t.ntx + ay) * t.ntx + az;
      const int b = t.tile_start[ct], en = t.tile_start[ct + 1];
      for (int s2 = b; s2 < en; ++s2) {
        const int j = t.sorted_idx[s2];
        if (j == i) continue;
        double dx = xi - pos[3 * j], dy = yi - pos[3 * j + 1], dz = zi - pos[3 * j + 2];
        dx -= p.box * rint(dx * p.inv_box);
        dy -= p.box * rint(dy * p.inv_box);
        dz -= p.box * rint(dz * p.inv_box);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= rc2) continue;
        const double r = sqrt(r2);
        const int q = si + species[j];
        const double* row = p.tab + 5 * q;
        const double f = -bmh_dvdr(row, r) / r;
        fx += f * dx;
        fy += f * dy;
        fz += f * dz;
        if (j > i) e += bmh_v(row, r) - vshift[q];
      }
    }
  }
#pragma unroll
  for (int m = kBmhLanes / 2; m > 0; m >>= 1) {
    fx += __shfl_xor(fx, m, 64);
    fy += __shfl_xor(fy, m, 64);
    fz += __shfl_xor(fz, m, 64);
    e += __shfl_xor(e, m, 64);
  }
  if (act && lane == 0) {
    f_sr[3 * i] = fx;
    f_sr[3 * i + 1] = fy;
    f_sr[3 * i + 2] = fz;
  }
  const double te = block_sum((lane == 0) ? e : 0.0, red);
  if (threadIdx.x == 0) e_part[blockIdx.x] = te;
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
  double v0[3] = {vel[3 * i], vel[3 * i + 1], vel[3 * i + 2]};
  if (p.lgv) {
    // first Ornstein-Uhlenbeck half step (OVRVO)
    double z[3];
    langevin_normals(p.seed, p.step, 0, i, z);
    const double cs = sqrt(p.ou_b2 / mass[i]);
#pragma unroll
    for (int d = 0; d < 3; ++d) v0[d] = p.ou_a * v0[d] + cs * z[d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int k = 3 * i + d;
    const double v = v0[d] + c * (f_es[k] + f_sr[k]);
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
        w += 0.5 * (f_old[k] + f_es[k]) * (pos[k] - x_old[k]);
      }
    }
    if (do_kick && p.lgv) {
      // second Ornstein-Uhlenbeck half step (OVRVO)
      double z[3];
      langevin_normals(p.seed, p.step, 1, i, z);
      const double cs = sqrt(p.ou_b2 / m);
#pragma unroll
      for (int d = 0; d < 3; ++d) v[d] = p.ou_a * v[d] + cs * z[d];
    }
    if (do_kick) {
#pragma unroll
      for (int d = 0; d < 3; ++d) vel[3 * i + d] = v[d];
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

__global__ __launch_bounds__(kThreads) void k_md_finish(const double* part, int nb,
                                                        const double* e_part, int ne, int prime,
                                                        double* scalars) {
  __shared__ double red[8];
  const double e_sr = sum_partials(e_part, ne, red);
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

hipError_t launch_md_kick_drift(const maze_md_state& md, long long step, hipStream_t st) {
  MdParams p = md_params(md, 1.0, step);
  const int n = md.n_ions;
  hipLaunchKernelGGL(k_md_kick_drift, dim3(md_blocks(n)), dim3(kThreads), 0, st, p, md.pos_dev,
                     md.vel_dev, md.mass_dev, (const double*)md.f_es_dev,
                     (const double*)md.f_sr_dev, md.scratch_dev, md.scratch_dev + 3 * (size_t)n);
  return hipGetLastError();
}

// Tile search radius covering the cutoff (one more tile when the last tile
// of an axis is partial); 0 when the tile block would wrap onto itself, in
// which case the all-pairs kernel runs.
static int bmh_tile_radius(const DeviceState& d, double cutoff) {
  const double edge = kTile * d.h;
  int R = (int)std::ceil(cutoff / edge);
  if (d.N % kTile != 0) R += 1;
  return (2 * R + 1 <= d.ntx) ? R : 0;
}

int md_energy_partials(const DeviceState& d, double cutoff) {
  const int n = d.n_ions;
  if (bmh_tile_radius(d, cutoff) > 0)
    return (int)(((long long)n * kBmhLanes + kThreads - 1) / kThreads);
  return md_blocks(n);
}

hipError_t launch_md_bmh(const maze_md_state& md, const DeviceState& d, hipStream_t st) {
  MdParams p = md_params(md, d.box);
  const int n = md.n_ions;
  const int R = bmh_tile_radius(d, md.cutoff);
  if (R > 0) {
    BmhTiles t{d.tile_start, d.sorted_idx, d.s_cell, d.ntx, R};
    hipLaunchKernelGGL(k_md_bmh_tiles, dim3(md_energy_partials(d, md.cutoff)), dim3(kThreads), 0,
                       st, p, t, (const double*)md.pos_dev, md.species_dev, md.f_sr_dev,
                       d.md_epart);
  } else {
    hipLaunchKernelGGL(k_md_bmh, dim3(md_blocks(n)), dim3(kThreads), 0, st, p,
                       (const double*)md.pos_dev, md.species_dev, md.f_sr_dev, d.md_epart);
  }
  return hipGetLastError();
}

static hipError_t md_finish(const maze_md_state& md, const DeviceState& d, int do_kick,
                            long long step, hipStream_t st) {
  MdParams p = md_params(md, 1.0, step);
  const int n = md.n_ions, nb = md_blocks(n);
  double* part = md.scratch_dev + 6 * (size_t)n;
  hipLaunchKernelGGL(k_md_kick2, dim3(nb), dim3(kThreads), 0, st, p, (const double*)md.pos_dev,
                     md.vel_dev, md.mass_dev, (const double*)md.f_es_dev,
                     (const double*)md.f_sr_dev, (const double*)md.scratch_dev,
                     (const double*)(md.scratch_dev + 3 * (size_t)n), do_kick, part, nb);
  hipLaunchKernelGGL(k_md_finish, dim3(1), dim3(kThreads), 0, st, (const double*)part, nb,
                     (const double*)d.md_epart, md_energy_partials(d, md.cutoff),
                     do_kick ? 0 : 1, md.scalars_dev);
  return hipGetLastError();
}

hipError_t launch_md_finish(const maze_md_state& md, const DeviceState& d, long long step,
                            hipStream_t st) {
  return md_finish(md, d, 1, step, st);
}
hipError_t launch_md_prime(const maze_md_state& md, const DeviceState& d, hipStream_t st) {
  return md_finish(md, d, 0, 0, st);
}

}  // namespace maze
