// Per-atom virial, forces and HNEMD driving force of Tersoff's bond-order
// potential on the device (float64), following Sec. II.A of the paper:
//   F_ij  = dU_i/dr_ij - dU_j/dr_ji                           (Eq. 4)
//   W_i   = sum_{j != i} r_ij (x) dU_j/dr_ji                   (Eq. 8)
//   F_ext = E_i F_e + F_e . W_i                                 (Eq. 12)
// with the site energies
//   U_i     = 1/2 sum_j f_C(r_ij) [A exp(-l1 r_ij) - b_ij B exp(-l2 r_ij)]
//   b_ij    = (1 + beta^n zeta_ij^n)^(-1/(2n))
//   zeta_ij = sum_{k != j} f_C(r_ik) g(cos theta_ijk) exp(l3^m (r_ij - r_ik)^m)
//   g(c)    = gamma (1 + c0^2/d^2 - c0^2/(d^2 + (c - h)^2)).
//
// Pipeline (one thread per atom everywhere, deterministic):
//   neighbours (every few MD steps): cell of each atom (counting sort with
//     atomics), exclusive scan of the cell counts, cell fill, per-atom scan
//     of the 27 surrounding cells (minimum image, r < R + D), list sorted by
//     atom index (so the result does not depend on the order the atomics
//     filled the cells), reverse slots (where i sits in j's list);
//   per evaluation: k_tersoff_site -- pair vectors, bond orders, U_i and the
//     partials dU_i/dr_ij of atom i's own neighbours; k_tersoff_gather --
//     forces, the Eq. 8 virial (the partial dU_j/dr_ji read from j's list
//     through the reverse slot), Eq. 12 and the float32 copy of W_i in the
//     layout the modal-current push takes.
// Pair arrays are slot-major, [slot][N], so that the threads of a wave read
// consecutive addresses.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mhc_tersoff.h"

namespace mhc {

__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }

__device__ __forceinline__ int cell_coord(double x, double L, int nc) {
  const double w = x - L * floor(x / L);
  int c = (int)(w * nc / L);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// ------------------------------------------------------------- neighbour lists
__global__ void k_fill_zero_i32(int* __restrict__ p, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = 0;
}

__global__ void __launch_bounds__(256) k_cell_count(const double* __restrict__ pos, int64_t N, CellGrid cg,
                                                    int* __restrict__ cell_of, int* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int cx = cell_coord(pos[3 * i], cg.box[0], cg.nc[0]);
  const int cy = cell_coord(pos[3 * i + 1], cg.box[1], cg.nc[1]);
  const int cz = cell_coord(pos[3 * i + 2], cg.box[2], cg.nc[2]);
  const int c = (cx * cg.nc[1] + cy) * cg.nc[2] + cz;
  cell_of[i] = c;
  atomicAdd(&count[c], 1);
}

// Exclusive scan of n counts into start[0..n] (start[n] = total), one work-group.
__global__ void __launch_bounds__(1024) k_cell_scan(const int* __restrict__ count, int n, int* __restrict__ start) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = t * per, b1 = min(n, b0 + per);
  int s = 0;
  for (int c = b0; c < b1; ++c) s += count[c];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan of the partial sums
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t == 0 ? 0 : part[t - 1];
  for (int c = b0; c < b1; ++c) {
    start[c] = run;
    run += count[c];
  }
  if (t == 1023) start[n] = part[1023];
}

__global__ void __launch_bounds__(256) k_cell_fill(int64_t N, const int* __restrict__ cell_of,
                                                   const int* __restrict__ start, int* __restrict__ fill,
                                                   int* __restrict__ atoms) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = cell_of[i];
  const int k = atomicAdd(&fill[c], 1);
  atoms[start[c] + k] = (int)i;
}

__global__ void __launch_bounds__(256) k_neighbors(const double* __restrict__ pos, int64_t N, CellGrid cg,
                                                   double rc2, const int* __restrict__ cell_of,
                                                   const int* __restrict__ start, const int* __restrict__ atoms,
                                                   int max_nb, int* __restrict__ nbr, int* __restrict__ n_nb,
                                                   int* __restrict__ max_found) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  const int c = cell_of[i];
  const int cz0 = c % cg.nc[2], cy0 = (c / cg.nc[2]) % cg.nc[1], cx0 = c / (cg.nc[2] * cg.nc[1]);
  const int ox = cg.nc[0] >= 3 ? 1 : 0, oy = cg.nc[1] >= 3 ? 1 : 0, oz = cg.nc[2] >= 3 ? 1 : 0;
  int cnt = 0;
  for (int dx = -ox; dx <= ox; ++dx) {
    const int cx = (cx0 + dx + cg.nc[0]) % cg.nc[0];
    for (int dy = -oy; dy <= oy; ++dy) {
      const int cy = (cy0 + dy + cg.nc[1]) % cg.nc[1];
      for (int dz = -oz; dz <= oz; ++dz) {
        const int cz = (cz0 + dz + cg.nc[2]) % cg.nc[2];
        const int cc = (cx * cg.nc[1] + cy) * cg.nc[2] + cz;
        for (int q = start[cc]; q < start[cc + 1]; ++q) {
          const int j = atoms[q];
          if (j == (int)i) continue;
          const double ddx = min_image(pos[3 * (int64_t)j] - xi, cg.box[0]);
          const double ddy = min_image(pos[3 * (int64_t)j + 1] - yi, cg.box[1]);
          const double ddz = min_image(pos[3 * (int64_t)j + 2] - zi, cg.box[2]);
          if (ddx * ddx + ddy * ddy + ddz * ddz < rc2) {
            if (cnt < max_nb) nbr[(int64_t)cnt * N + i] = j;
            ++cnt;
          }
        }
      }
    }
  }
  const int n = cnt < max_nb ? cnt : max_nb;
  // ascending atom index: the list no longer depends on the cell fill order
  for (int a = 1; a < n; ++a) {
    const int key = nbr[(int64_t)a * N + i];
    int b = a - 1;
    while (b >= 0 && nbr[(int64_t)b * N + i] > key) {
      nbr[(int64_t)(b + 1) * N + i] = nbr[(int64_t)b * N + i];
      --b;
    }
    nbr[(int64_t)(b + 1) * N + i] = key;
  }
  n_nb[i] = n;
  atomicMax(max_found, cnt);
}

// rev[s][i] = slot of i in the list of j = nbr[s][i] (-1 if absent, which a
// symmetric distance test rules out; the host checks).
__global__ void __launch_bounds__(256) k_reverse(int64_t N, const int* __restrict__ nbr, const int* __restrict__ n_nb,
                                                 int* __restrict__ rev, int* __restrict__ missing) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int n = n_nb[i];
  for (int s = 0; s < n; ++s) {
    const int j = nbr[(int64_t)s * N + i];
    const int nj = n_nb[j];
    int r = -1;
    for (int t = 0; t < nj; ++t)
      if (nbr[(int64_t)t * N + j] == (int)i) r = t;
    rev[(int64_t)s * N + i] = r;
    if (r < 0) *missing = 1;
  }
}

// --------------------------------------------------------------- potential
__device__ __forceinline__ void cutoff_fn(const TersoffParams& p, double r, double* fc, double* dfc) {
  if (r < p.R - p.D) {
    *fc = 1.0;
    *dfc = 0.0;
  } else if (r > p.R + p.D) {
    *fc = 0.0;
    *dfc = 0.0;
  } else {
    double s, c;
    sincos(0.5 * M_PI * (r - p.R) / p.D, &s, &c);
    *fc = 0.5 - 0.5 * s;
    *dfc = -0.25 * M_PI / p.D * c;
  }
}

__device__ __forceinline__ void angle_fn(const TersoffParams& p, double cs, double* g, double* dg) {
  const double t = cs - p.h;
  const double den = p.d2 + t * t;
  *g = p.gamma * (1.0 + p.c2 / p.d2 - p.c2 / den);
  *dg = p.gamma * p.c2 * 2.0 * t / (den * den);
}

// exp(l3^m x^m) and its derivative in x (m = 1 or 3)
__device__ __forceinline__ void exp_fn(const TersoffParams& p, double x, double* e, double* de) {
  if (p.l3m == 0.0) {
    *e = 1.0;
    *de = 0.0;
    return;
  }
  const double xm1 = p.m == 3 ? x * x : 1.0;
  *e = exp(p.l3m * xm1 * x);
  *de = *e * p.m * p.l3m * xm1;
}

// Per atom i: pair vectors of its neighbours, the bond orders b_ij and
// db_ij/dzeta_ij, the site energy U_i and the partials dU_i/dr_ij.
__global__ void __launch_bounds__(256) k_tersoff_site(TersoffArgs a, TersoffParams p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = a.N;
  if (i >= N) return;
  const int n = a.n_nb[i];
  const double xi = a.pos[3 * i], yi = a.pos[3 * i + 1], zi = a.pos[3 * i + 2];
  double* rx = a.rv;
  double* ry = a.rv + (int64_t)a.max_nb * N;
  double* rz = a.rv + 2 * (int64_t)a.max_nb * N;
  double* rr = a.rv + 3 * (int64_t)a.max_nb * N;
  for (int s = 0; s < n; ++s) {
    const int64_t j = a.nbr[(int64_t)s * N + i];
    const double dx = min_image(a.pos[3 * j] - xi, a.box[0]);
    const double dy = min_image(a.pos[3 * j + 1] - yi, a.box[1]);
    const double dz = min_image(a.pos[3 * j + 2] - zi, a.box[2]);
    const int64_t e = (int64_t)s * N + i;
    rx[e] = dx;
    ry[e] = dy;
    rz[e] = dz;
    rr[e] = sqrt(dx * dx + dy * dy + dz * dz);
  }
  // bond orders and the site energy
  double u = 0.0;
  for (int s = 0; s < n; ++s) {
    const int64_t es = (int64_t)s * N + i;
    const double sx = rx[es], sy = ry[es], sz = rz[es], rs = rr[es];
    double z = 0.0;
    for (int q = 0; q < n; ++q) {
      if (q == s) continue;
      const int64_t eq = (int64_t)q * N + i;
      const double rq = rr[eq];
      double fc, dfc, g, dg, e, de;
      cutoff_fn(p, rq, &fc, &dfc);
      const double cs = (sx * rx[eq] + sy * ry[eq] + sz * rz[eq]) / (rs * rq);
      angle_fn(p, cs, &g, &dg);
      exp_fn(p, rs - rq, &e, &de);
      z += fc * g * e;
    }
    const double bz = pow(p.beta * z, p.n);
    const double b = pow(1.0 + bz, -0.5 / p.n);
    const double db = z == 0.0 ? 0.0 : -0.5 * bz / z * pow(1.0 + bz, -0.5 / p.n - 1.0);
    double fc, dfc;
    cutoff_fn(p, rs, &fc, &dfc);
    const double fa = p.B * exp(-p.l2 * rs);
    u += fc * (p.A * exp(-p.l1 * rs) - b * fa);
    a.bb[es] = b;
    a.adb[es] = fc * fa * db;           // a_ij db_ij/dzeta_ij, a_ij = f_C(r_ij) B exp(-l2 r_ij)
  }
  a.U[i] = 0.5 * u;
  // partials dU_i/dr_ij
  double* d0 = a.dd;
  double* d1 = a.dd + (int64_t)a.max_nb * N;
  double* d2 = a.dd + 2 * (int64_t)a.max_nb * N;
  for (int s = 0; s < n; ++s) {
    const int64_t es = (int64_t)s * N + i;
    const double sx = rx[es], sy = ry[es], sz = rz[es], rs = rr[es];
    const double ux = sx / rs, uy = sy / rs, uz = sz / rs;
    double fcs, dfcs;
    cutoff_fn(p, rs, &fcs, &dfcs);
    const double fr = p.A * exp(-p.l1 * rs), fa = p.B * exp(-p.l2 * rs);
    const double b = a.bb[es];
    const double radial = 0.5 * (dfcs * (fr - b * fa) + fcs * (-p.l1 * fr + p.l2 * b * fa));
    double gx = radial * ux, gy = radial * uy, gz = radial * uz;
    double zx = 0.0, zy = 0.0, zz = 0.0;          // d zeta_ij / d r_ij
    double kx = 0.0, ky = 0.0, kz = 0.0;          // sum_k a_ik db_ik d zeta_ik / d r_ij, k != j
    for (int q = 0; q < n; ++q) {
      if (q == s) continue;
      const int64_t eq = (int64_t)q * N + i;
      const double qx = rx[eq], qy = ry[eq], qz = rz[eq], rq = rr[eq];
      const double cs = (sx * qx + sy * qy + sz * qz) / (rs * rq);
      // d cos theta / d r_ij
      const double cx = qx / (rs * rq) - cs * sx / (rs * rs);
      const double cy = qy / (rs * rq) - cs * sy / (rs * rs);
      const double cz = qz / (rs * rq) - cs * sz / (rs * rs);
      double fcq, dfcq, g, dg, e1, de1, e2, de2;
      cutoff_fn(p, rq, &fcq, &dfcq);
      angle_fn(p, cs, &g, &dg);
      exp_fn(p, rs - rq, &e1, &de1);
      exp_fn(p, rq - rs, &e2, &de2);
      zx += fcq * (dg * cx * e1 + g * de1 * ux);
      zy += fcq * (dg * cy * e1 + g * de1 * uy);
      zz += fcq * (dg * cz * e1 + g * de1 * uz);
      const double w = a.adb[eq];
      kx += w * (dfcs * g * e2 * ux + fcs * dg * cx * e2 - fcs * g * de2 * ux);
      ky += w * (dfcs * g * e2 * uy + fcs * dg * cy * e2 - fcs * g * de2 * uy);
      kz += w * (dfcs * g * e2 * uz + fcs * dg * cz * e2 - fcs * g * de2 * uz);
    }
    const double w = a.adb[es];
    gx -= 0.5 * (w * zx + kx);
    gy -= 0.5 * (w * zy + ky);
    gz -= 0.5 * (w * zz + kz);
    d0[es] = gx;
    d1[es] = gy;
    d2[es] = gz;
  }
}

// Per atom i: F_i (Eq. 4 summed), W_i (Eq. 8), E_i and F_ext (Eq. 12).
__global__ void __launch_bounds__(256) k_tersoff_gather(TersoffArgs a, GatherArgs o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = a.N;
  if (i >= N) return;
  const int n = a.n_nb[i];
  const int64_t mn = (int64_t)a.max_nb * N;
  double f[3] = {0.0, 0.0, 0.0};
  double w[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < n; ++s) {
    const int64_t es = (int64_t)s * N + i;
    const int64_t j = a.nbr[es];
    const int64_t ej = (int64_t)a.rev[es] * N + j;
    const double r[3] = {a.rv[es], a.rv[mn + es], a.rv[2 * mn + es]};
    const double dij[3] = {a.dd[es], a.dd[mn + es], a.dd[2 * mn + es]};
    const double dji[3] = {a.dd[ej], a.dd[mn + ej], a.dd[2 * mn + ej]};
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      f[mu] += dij[mu] - dji[mu];
#pragma unroll
      for (int nu = 0; nu < 3; ++nu) w[3 * mu + nu] += r[mu] * dji[nu];
    }
  }
  if (o.F)
    for (int mu = 0; mu < 3; ++mu) o.F[3 * i + mu] = f[mu];
  if (o.W)
    for (int q = 0; q < 9; ++q) o.W[9 * i + q] = w[q];
  if (o.W32)
    for (int q = 0; q < 9; ++q) o.W32[9 * i + q] = (float)w[q];
  if (o.Fext) {
    double e = a.U[i];
    if (o.vel) {
      const double vx = o.vel[3 * i], vy = o.vel[3 * i + 1], vz = o.vel[3 * i + 2];
      e += 0.5 * o.mass[i] * (vx * vx + vy * vy + vz * vz) * o.ke_unit;
    }
#pragma unroll
    for (int nu = 0; nu < 3; ++nu)
      o.Fext[3 * i + nu] = e * o.fe[nu] + (o.fe[0] * w[nu] + o.fe[1] * w[3 + nu] + o.fe[2] * w[6 + nu]);
  }
}

// ------------------------------------------------------------- launchers
static inline unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_neighbors(hipStream_t s, const double* pos, int64_t N, const CellGrid& cg, double rc, int max_nb,
                            NeighborBufs b) {
  const int n_cells = cg.nc[0] * cg.nc[1] * cg.nc[2];
  hipError_t e;
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(blocks_of(n_cells, 256)), dim3(256), 0, s, b.count, n_cells);
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(blocks_of(n_cells, 256)), dim3(256), 0, s, b.fill, n_cells);
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(1), dim3(256), 0, s, b.flags, 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_count, dim3(blocks_of(N, 256)), dim3(256), 0, s, pos, N, cg, b.cell_of, b.count);
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, s, b.count, n_cells, b.start);
  hipLaunchKernelGGL(k_cell_fill, dim3(blocks_of(N, 256)), dim3(256), 0, s, N, b.cell_of, b.start, b.fill, b.atoms);
  hipLaunchKernelGGL(k_neighbors, dim3(blocks_of(N, 256)), dim3(256), 0, s, pos, N, cg, rc * rc, b.cell_of, b.start,
                     b.atoms, max_nb, b.nbr, b.n_nb, b.flags);
  hipLaunchKernelGGL(k_reverse, dim3(blocks_of(N, 256)), dim3(256), 0, s, N, b.nbr, b.n_nb, b.rev, b.flags + 1);
  return hipGetLastError();
}

hipError_t launch_tersoff(hipStream_t s, const TersoffArgs& a, const TersoffParams& p, const GatherArgs& o,
                          hipEvent_t e0, hipEvent_t e1) {
  if (e0) {
    hipError_t e = hipEventRecord(e0, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tersoff_site, dim3(blocks_of(a.N, 256)), dim3(256), 0, s, a, p);
  hipLaunchKernelGGL(k_tersoff_gather, dim3(blocks_of(a.N, 256)), dim3(256), 0, s, a, o);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && e1) e = hipEventRecord(e1, s);
  return e;
}

}  // namespace mhc
