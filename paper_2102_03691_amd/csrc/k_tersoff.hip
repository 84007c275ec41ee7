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
// Pipeline (deterministic: fixed summation orders, sorted lists):
//   neighbours (every few MD steps): cell of each atom (counting sort with
//     atomics), exclusive scan of the cell counts (per-block sums, their
//     scan, per-block scans), cell fill, per-atom scan of the 27 surrounding
//     cells (minimum image, r < R + D + skin), list sorted by atom index (so
//     the result does not depend on the order the atomics filled the cells),
//     reverse slots (where i sits in j's list);
//   per evaluation, LPA lanes per atom (one per neighbour slot, LPA the
//     next power of two >= the largest neighbour count, at least 4; the site
//     kernel runs 4 lanes x 2 slots where LPA is 8), the pair values of an
//     atom shared through LDS:
//     k_tersoff_site -- pair vector, f_C, the two exponentials, zeta_ij,
//       b_ij, db_ij/dzeta_ij; U_i (summed in slot order by the first lane);
//       the partial dU_i/dr_ij of the lane's pair;
//     k_tersoff_gather -- per pair dU_i/dr_ij - dU_j/dr_ji and
//       r_ij (x) dU_j/dr_ji (the second partial read from j's list through the
//       reverse slot), summed in slot order into F_i and W_i (Eq. 8), then
//       E_i, F_ext (Eq. 12) and the float32 copy of W_i in the layout the
//       modal-current push takes.
// Pair arrays are slot-major, [slot][N]: the lanes of a wave read 64/LPA
// consecutive atoms of each slot.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "mhc_tersoff.h"

namespace mhc {

// Minimum-image difference; iL = 1 / L.  For every pair closer than L / 2 by
// more than rounding (all listed pairs: each box edge exceeds twice the list
// cutoff) the shift is the same integer as with d / L, so the result is too.
__device__ __forceinline__ double min_image(double d, double L, double iL) { return d - L * rint(d * iL); }

__device__ __forceinline__ int cell_coord(double x, double L, int nc) {
  const double w = x - L * floor(x / L);
  int c = (int)(w * nc / L);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// ------------------------------------------------------------- neighbour lists
// atomicMax of v over the whole wave with one atomic per wave instead of one
// per lane (the lanes of an atom-per-lane kernel all target one counter, and
// 64 times fewer atomics on one address matter at 10^5..10^6 atoms).  Every
// lane of the wave must call it.
__device__ __forceinline__ void wave_atomic_max(int* addr, int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0 && v > 0) atomicMax(addr, v);
}

__global__ void k_set_i32(int* __restrict__ p, int value) {
  if (threadIdx.x == 0) *p = value;
}

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

// Exclusive scan of n counts into start[0..n] (start[n] = total) in three
// passes over tiles of SCAN_TILE counts: per-tile sums, an exclusive scan of
// the tile sums (one work-group), then every tile's own scan plus its offset.
constexpr int SCAN_TILE = 1024;

// Inclusive scan of one value per thread over a 1024-thread work-group.
__device__ __forceinline__ int block_scan_incl(int v, int* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_TILE; off <<= 1) {
    const int w = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += w;
    __syncthreads();
  }
  const int r = sh[t];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(1024) k_scan_tile_sums(const int* __restrict__ count, int n, int* __restrict__ sums) {
  __shared__ int sh[SCAN_TILE];
  const int c = blockIdx.x * SCAN_TILE + threadIdx.x;
  const int v = block_scan_incl(c < n ? count[c] : 0, sh);
  if (threadIdx.x == SCAN_TILE - 1) sums[blockIdx.x] = v;
}

// Exclusive scan of the tile sums in place (n_tiles values, any count).
__global__ void __launch_bounds__(1024) k_scan_tile_offsets(int* __restrict__ sums, int n_tiles) {
  __shared__ int sh[SCAN_TILE];
  __shared__ int total;
  int run = 0;
  for (int base = 0; base < n_tiles; base += SCAN_TILE) {
    const int c = base + threadIdx.x;
    const int v = c < n_tiles ? sums[c] : 0;
    const int incl = block_scan_incl(v, sh);
    if (c < n_tiles) sums[c] = run + incl - v;
    if (threadIdx.x == SCAN_TILE - 1) total = incl;
    __syncthreads();
    run += total;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_scan_apply(const int* __restrict__ count, int n,
                                                     const int* __restrict__ offsets, int* __restrict__ start) {
  __shared__ int sh[SCAN_TILE];
  const int c = blockIdx.x * SCAN_TILE + threadIdx.x;
  const int v = c < n ? count[c] : 0;
  const int incl = block_scan_incl(v, sh) + offsets[blockIdx.x];
  if (c < n) start[c] = incl - v;
  if (c == n - 1) start[n] = incl;
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

// The list of atom i; returns the number of atoms found inside rc (which may
// exceed max_nb: only max_nb are kept) and, in *n_b, the number inside rb
// (rb2 = rb^2; the bond lists' cutoff).
__device__ int neighbors_of(int64_t i, const double* __restrict__ pos, int64_t N, const CellGrid& cg, double rc2,
                            double rb2, const int* __restrict__ cell_of, const int* __restrict__ start,
                            const int* __restrict__ atoms, int max_nb, int* __restrict__ nbr,
                            int* __restrict__ n_nb, int* n_b) {
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  const int c = cell_of[i];
  const int cz0 = c % cg.nc[2], cy0 = (c / cg.nc[2]) % cg.nc[1], cx0 = c / (cg.nc[2] * cg.nc[1]);
  const int ox = cg.nc[0] >= 3 ? 1 : 0, oy = cg.nc[1] >= 3 ? 1 : 0, oz = cg.nc[2] >= 3 ? 1 : 0;
  int cnt = 0, cb = 0;
  // the atoms of atoms[q0 .. q1), 8 at a time with every load issued before
  // the first distance (the padding reads atom i itself, which is skipped)
  auto scan = [&](int q0, int q1) {
    constexpr int U = 8;
    for (int qb = q0; qb < q1; qb += U) {
      int jj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) jj[u] = qb + u < q1 ? atoms[qb + u] : (int)i;
      double px[U], py[U], pz[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        px[u] = pos[3 * (int64_t)jj[u]];
        py[u] = pos[3 * (int64_t)jj[u] + 1];
        pz[u] = pos[3 * (int64_t)jj[u] + 2];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (jj[u] == (int)i) continue;
        const double ddx = min_image(px[u] - xi, cg.box[0], cg.ibox[0]);
        const double ddy = min_image(py[u] - yi, cg.box[1], cg.ibox[1]);
        const double ddz = min_image(pz[u] - zi, cg.box[2], cg.ibox[2]);
        const double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
        if (d2 < rc2) {
          if (cnt < max_nb) nbr[(int64_t)cnt * N + i] = jj[u];
          ++cnt;
          if (d2 < rb2) ++cb;
        }
      }
    }
  };
  for (int dx = -ox; dx <= ox; ++dx) {
    const int cx = (cx0 + dx + cg.nc[0]) % cg.nc[0];
    for (int dy = -oy; dy <= oy; ++dy) {
      const int cy = (cy0 + dy + cg.nc[1]) % cg.nc[1];
      const int row = (cx * cg.nc[1] + cy) * cg.nc[2];
      if (oz == 1 && cz0 >= 1 && cz0 + 1 < cg.nc[2]) {
        // the three cells along z are consecutive, and so are their atoms
        scan(start[row + cz0 - 1], start[row + cz0 + 2]);
      } else {
        for (int dz = -oz; dz <= oz; ++dz) {
          const int cz = (cz0 + dz + cg.nc[2]) % cg.nc[2];
          scan(start[row + cz], start[row + cz + 1]);
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
  *n_b = cb;
  return cnt;
}

// flags[0] = largest count inside rc, flags[2] = largest count inside rb.
__global__ void __launch_bounds__(256) k_neighbors(const double* __restrict__ pos, int64_t N, CellGrid cg,
                                                   double rc2, double rb2, const int* __restrict__ cell_of,
                                                   const int* __restrict__ start, const int* __restrict__ atoms,
                                                   int max_nb, int* __restrict__ nbr, int* __restrict__ n_nb,
                                                   int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int cb = 0;
  const int cnt = i < N ? neighbors_of(i, pos, N, cg, rc2, rb2, cell_of, start, atoms, max_nb, nbr, n_nb, &cb) : 0;
  wave_atomic_max(&flags[0], cnt);
  wave_atomic_max(&flags[2], cb);
}

// rev[s][i] = slot of i in the list of j = nbr[s][i] (-1 if absent, which a
// symmetric distance test rules out; the host checks).  Lists are ascending
// (k_neighbors sorts them), so the slot is found by bisection.
// One lane per (atom, slot): threadIdx.x runs over 64 consecutive atoms (so a
// wave's list reads and writes are contiguous) and threadIdx.y over the slots
// y, y + REV_SLOTS, ...; each lane finds i in j's sorted list by bisection.
constexpr int REV_SLOTS = 16;
__global__ void __launch_bounds__(64 * REV_SLOTS) k_reverse(int64_t N, const int* __restrict__ nbr,
                                                            const int* __restrict__ n_nb, int* __restrict__ rev,
                                                            int* __restrict__ missing) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= N) return;
  const int n = n_nb[i];
  for (int s = threadIdx.y; s < n; s += REV_SLOTS) {
    const int j = nbr[(int64_t)s * N + i];
    const int nj = n_nb[j];
    int lo = 0, hi = nj;   // first slot of j's list whose entry is >= i
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (nbr[(int64_t)mid * N + j] < (int)i) lo = mid + 1;
      else hi = mid;
    }
    const int r = lo < nj && nbr[(int64_t)lo * N + j] == (int)i ? lo : -1;
    rev[(int64_t)s * N + i] = r;
    if (r < 0) *missing = 1;
  }
}

// Bond lists out of lists built with a skin: the listed pairs closer than rb
// (rb2 = rb^2, rb = R + D + delta with delta the bond lists' own skin), in
// list order (so still ascending j), at most max_b per atom.  mask[i] bit s =
// list slot s of i is kept; count[i] = pairs kept; ref[i] = pos[i] (the
// positions of the build, for the displacement test); flags[0] = largest
// count found (atomic max); flags[1] = 1 if an atom had more than max_b.
// need (null: always build) = the rebuild flag of this evaluation, one value
// read by every thread, so the whole grid builds or none of it does; clear
// (null: none) is the other evaluation's flag, zeroed here.
__global__ void __launch_bounds__(256) k_bonds(const double* __restrict__ pos, int64_t N, double Lx, double Ly,
                                               double Lz, double iLx, double iLy, double iLz,
                                               const int* __restrict__ nbr, const int* __restrict__ n_nb, double rb2,
                                               int max_b, int* __restrict__ bnbr, int* __restrict__ bcount,
                                               unsigned long long* __restrict__ mask, double* __restrict__ ref,
                                               int* __restrict__ flags, const int* __restrict__ need,
                                               int* __restrict__ clear) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (clear && i == 0) *clear = 0;
  if (need && *need == 0) return;
  const bool act = i < N;
  const int n = act ? n_nb[i] : 0;
  const double xi = act ? pos[3 * i] : 0.0, yi = act ? pos[3 * i + 1] : 0.0, zi = act ? pos[3 * i + 2] : 0.0;
  int c = 0, found = 0;
  unsigned long long m = 0;
  // 16 list slots at a time, every load issued before the first distance
  // (slots past the list read atom i itself and are masked out)
  constexpr int U = 16;
  for (int s0 = 0; s0 < n; s0 += U) {
    int jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) jj[u] = s0 + u < n ? nbr[(int64_t)(s0 + u) * N + i] : (int)i;
    double px[U], py[U], pz[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      px[u] = pos[3 * (int64_t)jj[u]];
      py[u] = pos[3 * (int64_t)jj[u] + 1];
      pz[u] = pos[3 * (int64_t)jj[u] + 2];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double x = min_image(px[u] - xi, Lx, iLx);
      const double y = min_image(py[u] - yi, Ly, iLy);
      const double z = min_image(pz[u] - zi, Lz, iLz);
      if (s0 + u < n && x * x + y * y + z * z < rb2) {
        ++found;
        m |= 1ull << (s0 + u);
        if (c < max_b) bnbr[(int64_t)(c++) * N + i] = jj[u];
      }
    }
  }
  if (act) {
    bcount[i] = c;
    mask[i] = m;
    ref[3 * i] = xi;
    ref[3 * i + 1] = yi;
    ref[3 * i + 2] = zi;
  }
  wave_atomic_max(&flags[0], found);
  if (found > max_b) flags[1] = 1;
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

// 1 / x for a positive normal x whose reciprocal is normal too: the hardware
// estimate refined by two Newton steps, within about an ulp of the rounded
// quotient (a full IEEE division adds scaling for the extremes of the range
// and a final correctly rounded step)
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Natural logarithm of a positive x (normal or subnormal): x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), log m = 2 atanh(s) with s = (m - 1) / (m + 1) summed as
// its odd power series (Abramowitz and Stegun 4.1.27; |s| < 0.1716, so the
// terms up to s^23 leave less than 1e-18), e ln 2 with ln 2 in two parts (the
// first with 21 significant bits, so e times it is exact).  Within 3 ulps of
// the true value from the subnormals up, at a fraction of the cost of the
// library routine, which carries double-length sums.
__device__ __forceinline__ double log_pos(double x) {
  int e;
  double m = frexp(x, &e);   // [0.5, 1)
  if (m < 0.70710678118654752440) {
    m += m;
    --e;
  }
  const double s = (m - 1.0) * recip(m + 1.0);
  const double s2 = s * s;
  double t = 1.0 / 23.0;
  t = fma(t, s2, 1.0 / 21.0);
  t = fma(t, s2, 1.0 / 19.0);
  t = fma(t, s2, 1.0 / 17.0);
  t = fma(t, s2, 1.0 / 15.0);
  t = fma(t, s2, 1.0 / 13.0);
  t = fma(t, s2, 1.0 / 11.0);
  t = fma(t, s2, 1.0 / 9.0);
  t = fma(t, s2, 1.0 / 7.0);
  t = fma(t, s2, 1.0 / 5.0);
  t = fma(t, s2, 1.0 / 3.0);
  const double lm = fma(2.0 * s * s2, t, 2.0 * s);
  const double de = (double)e;
  return fma(de, 0.6931467056274414, fma(de, 4.7493250390316726e-07, lm));
}

// log(1 + x) for x >= 0 by Goldberg's form x log(u) / (u - 1), u = 1 + x
// rounded (exact where u = 1): within 5 ulps for x below 2^1020
__device__ __forceinline__ double log1p_pos(double x) {
  const double u = 1.0 + x;
  return u == 1.0 ? x : (x * recip(u - 1.0)) * log_pos(u);
}

// g(cos theta) with t = cos theta - h, as gamma (1 + (c^2/d^2) t^2 / (d^2 + t^2)):
// the same function as gamma (1 + c^2/d^2 - c^2 / (d^2 + t^2)) without the
// cancellation of its two large terms (c^2/d^2 is about 4e7 for Si, g about 1e4)
__device__ __forceinline__ double angle_g(const TersoffParams& p, double cs) {
  const double t = cs - p.h;
  const double t2 = t * t;
  return fma(p.gc2d2 * t2, recip(p.d2 + t2), p.gamma);
}

// g and dg / dcos theta = 2 gamma c^2 t / (d^2 + t^2)^2
__device__ __forceinline__ void angle_fn(const TersoffParams& p, double cs, double* g, double* dg) {
  const double t = cs - p.h;
  const double t2 = t * t;
  const double inv = recip(p.d2 + t2);
  *g = fma(p.gc2d2 * t2, inv, p.gamma);
  *dg = p.g2c2 * t * inv * inv;
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

// LPA lanes per atom, SPL list slots per lane: lane s0 of the group handles
// the pairs (i, j = nbr[s][i]) of the slots s = s0 + k LPA, k < SPL.  Each
// pair's values go to LDS (field-major, sh[field][atom base + slot]) and
// every lane reads them after a barrier.  All sums run over the slots in list
// order, so the results do not depend on LPA and SPL.  With SPL = 2 a wave
// whose atoms all have at most LPA pairs skips the second slot of every lane.
// One wavefront per work-group: an atom's lanes never span two (LPA <= 64), so
// the barriers only order the wave's own LDS traffic, and waves of unequal
// length (atoms with more pairs) do not wait for each other.
constexpr int SITE_WG = 64;
template <int LPA, int SPL>
__global__ void __launch_bounds__(SITE_WG) k_tersoff_site(TersoffArgs a, TersoffParams p) {
  __shared__ double sh[8][SITE_WG * SPL];
  const int tid = threadIdx.x;
  const int s0 = tid & (LPA - 1);
  const int gb = (tid - s0) * SPL;   // this atom's slot 0 in LDS
  const int64_t N = a.N;
  const int64_t i = ((int64_t)blockIdx.x * SITE_WG + tid) / LPA;
  const int n = i < N ? a.n_nb[i] : 0;
  if (a.bond_need && *a.bond_need && n > 0) {
    // reverse slots of freshly built bond lists: bond s of i sits at the
    // s-th kept slot f of i's skin list, which is slot t = full_rev[f][i] in
    // the list of j; its bond slot in j's list is the number of j's kept
    // slots below t
    const unsigned long long mi = a.bond_mask[i];
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      const int s = s0 + k * LPA;
      if (s >= n) continue;
      unsigned long long m = mi;
      for (int c = 0; c < s; ++c) m &= m - 1;
      const int f = __builtin_ctzll(m);
      const int j = a.full_nbr[(int64_t)f * N + i];
      const int t = a.full_rev[(int64_t)f * N + i];
      int rr = -1;
      if (t >= 0) {
        const unsigned long long mj = a.bond_mask[j];
        if ((mj >> t) & 1ull) rr = __builtin_popcountll(mj & ((1ull << t) - 1ull));
      }
      a.bond_rev[(int64_t)s * N + i] = rr;
      if (rr < 0) a.bond_flags[2] = 1;
    }
  }
  double x[SPL], y[SPL], z[SPL], r[SPL], ir[SPL], fc[SPL], dfc[SPL], er[SPL], ea[SPL];
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int s = s0 + k * LPA;
    x[k] = y[k] = z[k] = 0.0;
    r[k] = ir[k] = 1.0;
    fc[k] = dfc[k] = er[k] = ea[k] = 0.0;
    if (s < n) {
      const int64_t j = a.nbr[(int64_t)s * N + i];
      x[k] = min_image(a.pos[3 * j] - a.pos[3 * i], a.box[0], a.ibox[0]);
      y[k] = min_image(a.pos[3 * j + 1] - a.pos[3 * i + 1], a.box[1], a.ibox[1]);
      z[k] = min_image(a.pos[3 * j + 2] - a.pos[3 * i + 2], a.box[2], a.ibox[2]);
      r[k] = sqrt(x[k] * x[k] + y[k] * y[k] + z[k] * z[k]);
      ir[k] = 1.0 / r[k];
      cutoff_fn(p, r[k], &fc[k], &dfc[k]);
      if (fc[k] != 0.0) {                    // a pair beyond R + D (listed with a skin) needs neither
        er[k] = p.A * exp(-p.l1 * r[k]);     // f_R
        ea[k] = p.B * exp(-p.l2 * r[k]);     // f_A (the attractive term enters as -b f_A)
      }
    }
    sh[0][gb + s] = x[k];
    sh[1][gb + s] = y[k];
    sh[2][gb + s] = z[k];
    sh[3][gb + s] = r[k];
    sh[4][gb + s] = ir[k];
    sh[5][gb + s] = fc[k];
  }
  __syncthreads();
  // Listed pairs beyond R + D (f_C = 0: lists built with a skin) add exact
  // zeros to every sum below, so they are skipped, and such a pair's own
  // slot has nothing to compute (its energy, bracket weight and partials are
  // zero).
  double b[SPL], adb[SPL];
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int s = s0 + k * LPA;
    b[k] = 1.0;
    adb[k] = 0.0;
    double u = 0.0;
    if (s < n && fc[k] != 0.0) {
      double zeta = 0.0;
      for (int q = 0; q < n; ++q) {
        if (q == s || sh[5][gb + q] == 0.0) continue;
        const int l = gb + q;
        const double cs = (x[k] * sh[0][l] + y[k] * sh[1][l] + z[k] * sh[2][l]) * (ir[k] * sh[4][l]);
        const double g = angle_g(p, cs);
        double e, de;
        exp_fn(p, r[k] - sh[3][l], &e, &de);
        zeta = fma(sh[5][l] * g, e, zeta);
      }
      // (beta zeta)^n and (1 + bz)^(-1/(2n)) through exp and log (bz = 0 where beta zeta = 0)
      const double bzeta = p.beta * zeta;
      const double bz = bzeta > 0.0 ? exp(p.n * log_pos(bzeta)) : 0.0;
      b[k] = exp(p.ninv2 * log1p_pos(bz));
      // db/dzeta = -1/2 beta^n zeta^(n-1) (1 + (beta zeta)^n)^(-1/(2n) - 1) = -b bz / (2 zeta (1 + bz))
      const double db = zeta == 0.0 ? 0.0 : -0.5 * b[k] * bz / (zeta * (1.0 + bz));
      adb[k] = fc[k] * ea[k] * db;
      u = fc[k] * (er[k] - b[k] * ea[k]);
    }
    sh[6][gb + s] = adb[k];
    sh[7][gb + s] = u;
  }
  __syncthreads();
  if (i < N && s0 == 0) {
    double acc = 0.0;
    for (int q = 0; q < n; ++q) acc += sh[7][gb + q];
    a.U[i] = 0.5 * acc;
  }
  const int64_t mn = (int64_t)a.max_nb * N;
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int s = s0 + k * LPA;
    if (s >= n) continue;
    const int64_t es = (int64_t)s * N + i;
    if (fc[k] == 0.0) {
      a.dd[es] = 0.0;
      a.dd[mn + es] = 0.0;
      a.dd[2 * mn + es] = 0.0;
      continue;
    }
    // dU_i/dr_ij for this slot's pair j
    const double ux = x[k] * ir[k], uy = y[k] * ir[k], uz = z[k] * ir[k];
    const double radial = 0.5 * (dfc[k] * (er[k] - b[k] * ea[k]) + fc[k] * (-p.l1 * er[k] + p.l2 * b[k] * ea[k]));
    const double ir2 = ir[k] * ir[k];
    double zx = 0.0, zy = 0.0, zz = 0.0;   // d zeta_ij / d r_ij
    double kx = 0.0, ky = 0.0, kz = 0.0;   // sum_{k != j} a_ik db_ik d zeta_ik / d r_ij
    for (int q = 0; q < n; ++q) {
      if (q == s || sh[5][gb + q] == 0.0) continue;
      const int l = gb + q;
      const double qx = sh[0][l], qy = sh[1][l], qz = sh[2][l], rq = sh[3][l];
      const double iri = ir[k] * sh[4][l];   // 1 / (r_ij r_ik)
      const double cs = (x[k] * qx + y[k] * qy + z[k] * qz) * iri;
      // d cos theta / d r_ij = r_ik / (r_ij r_ik) - cos theta r_ij / r_ij^2
      const double cr = cs * ir2;
      const double cx = fma(qx, iri, -x[k] * cr);
      const double cy = fma(qy, iri, -y[k] * cr);
      const double cz = fma(qz, iri, -z[k] * cr);
      double g, dg, e1, de1, e2, de2;
      angle_fn(p, cs, &g, &dg);
      exp_fn(p, r[k] - rq, &e1, &de1);
      exp_fn(p, rq - r[k], &e2, &de2);
      // zeta_ij's term: f_C(r_ik) (g' e1 dcos/dr_ij + g e1' u_ij)
      const double fcq = sh[5][l];
      const double za = fcq * dg * e1, zb = fcq * g * de1;
      zx = fma(za, cx, fma(zb, ux, zx));
      zy = fma(za, cy, fma(zb, uy, zy));
      zz = fma(za, cz, fma(zb, uz, zz));
      // zeta_ik's term through f_C(r_ij), g and e2 = exp(l3^m (r_ik - r_ij)^m), weighted by a_ik db_ik
      const double w = sh[6][l];
      const double ka = w * fc[k] * dg * e2, kb = w * g * (dfc[k] * e2 - fc[k] * de2);
      kx = fma(ka, cx, fma(kb, ux, kx));
      ky = fma(ka, cy, fma(kb, uy, ky));
      kz = fma(ka, cz, fma(kb, uz, kz));
    }
    a.dd[es] = radial * ux - 0.5 * (adb[k] * zx + kx);
    a.dd[mn + es] = radial * uy - 0.5 * (adb[k] * zy + ky);
    a.dd[2 * mn + es] = radial * uz - 0.5 * (adb[k] * zz + kz);
  }
}

// Atom i's sums over its pairs (the pair terms of its LPA lanes in sh, slot
// order) and every output of the gather kernel; with o.kick_vel, also the
// second half kick and thermostat scale of the step on its velocity (after
// E_i has read it) and the float32 copy.  Returns m_i |v_i|^2 after the kick
// (0 without one).
__device__ __forceinline__ double gather_atom(const TersoffArgs& a, const GatherArgs& o, const double (*sh)[256],
                                              int g0, int n, int64_t i) {
  double t[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) t[q] = 0.0;
  for (int k = 0; k < n; ++k)
#pragma unroll
    for (int q = 0; q < 12; ++q) t[q] += sh[q][g0 + k];
  const double* w = t + 3;
  double fx[3] = {0.0, 0.0, 0.0};
  if (o.Fext || o.add_ext) {
    double e = a.U[i];
    if (o.vel) {
      const double vx = o.vel[3 * i], vy = o.vel[3 * i + 1], vz = o.vel[3 * i + 2];
      e += 0.5 * o.mass[i] * (vx * vx + vy * vy + vz * vz) * o.ke_unit;
    }
#pragma unroll
    for (int nu = 0; nu < 3; ++nu)
      fx[nu] = e * o.fe[nu] + (o.fe[0] * w[nu] + o.fe[1] * w[3 + nu] + o.fe[2] * w[6 + nu]);
  }
  double f[3];
#pragma unroll
  for (int mu = 0; mu < 3; ++mu) f[mu] = o.add_ext ? t[mu] + fx[mu] : t[mu];
  if (o.F)
    for (int mu = 0; mu < 3; ++mu) o.F[3 * i + mu] = f[mu];
  if (o.W)
    for (int q = 0; q < 9; ++q) o.W[9 * i + q] = w[q];
  if (o.W32)
    for (int q = 0; q < 9; ++q) o.W32[9 * i + q] = (float)w[q];
  if (o.Fext)
    for (int nu = 0; nu < 3; ++nu) o.Fext[3 * i + nu] = fx[nu];
  double mv2 = 0.0;
  if (o.kick_vel) {   // end of an NVT step: v += c F / m, then v *= exp(-xi dt / 2)
    const double m = o.mass[i];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      double v = o.kick_vel[3 * i + mu];
      v = v + o.kick_c * f[mu] / m;
      v = v * o.kick_scale[2];
      o.kick_vel[3 * i + mu] = v;
      if (o.kick_v32) o.kick_v32[3 * i + mu] = (float)v;
      mv2 += m * v * v;
    }
  }
  return mv2;
}

// Per pair: dU_i/dr_ij - dU_j/dr_ji (Eq. 4) and r_ij (x) dU_j/dr_ji (Eq. 8);
// the first lane of each atom sums its pairs in slot order and writes F_i,
// W_i, E_i and F_ext (Eq. 12).
template <int LPA>
__global__ void __launch_bounds__(256) k_tersoff_gather(TersoffArgs a, GatherArgs o) {
  __shared__ double sh[12][256];
  const int tid = threadIdx.x;
  const int s = tid & (LPA - 1);
  const int g0 = tid - s;
  const int64_t N = a.N;
  const int64_t i = ((int64_t)blockIdx.x * 256 + tid) / LPA;
  const int n = i < N ? a.n_nb[i] : 0;
  // the pair's list entry and reverse slot are loaded with the count, not
  // after it (the rows below max_nb exist; entries at or past n are not used)
  const int64_t es = (int64_t)s * N + i;
  const bool row = i < N && s < a.max_nb;
  const int jl = row ? a.nbr[es] : 0, rl = row ? a.rev[es] : 0;
  double c[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) c[q] = 0.0;
  if (s < n) {
    const int64_t mn = (int64_t)a.max_nb * N;
    const int64_t j = jl;
    const int64_t ej = (int64_t)rl * N + j;
    const double r[3] = {min_image(a.pos[3 * j] - a.pos[3 * i], a.box[0], a.ibox[0]),
                         min_image(a.pos[3 * j + 1] - a.pos[3 * i + 1], a.box[1], a.ibox[1]),
                         min_image(a.pos[3 * j + 2] - a.pos[3 * i + 2], a.box[2], a.ibox[2])};
    // a pair beyond R + D has zero partials both ways (written so by the site
    // kernel): nothing to load or add
    if (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] < o.rcut2) {
      const double dij[3] = {a.dd[es], a.dd[mn + es], a.dd[2 * mn + es]};
      const double dji[3] = {a.dd[ej], a.dd[mn + ej], a.dd[2 * mn + ej]};
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        c[mu] = dij[mu] - dji[mu];
#pragma unroll
        for (int nu = 0; nu < 3; ++nu) c[3 + 3 * mu + nu] = r[mu] * dji[nu];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 12; ++q) sh[q][tid] = c[q];
  __syncthreads();
  const bool first = i < N && s == 0;
  double mv2 = 0.0;
  if (first) mv2 = gather_atom(a, o, sh, g0, n, i);
  if (o.ke_part) {   // the work-group's partial sum of m v^2 after the kick (uniform over the launch)
    constexpr int APB = 256 / LPA;   // atoms per work-group
    __shared__ double kp[APB];
    if (s == 0) kp[tid / LPA] = mv2;
    __syncthreads();
    for (int w = APB / 2; w > 0; w >>= 1) {
      if (tid < w) kp[tid] += kp[tid + w];
      __syncthreads();
    }
    if (tid == 0) o.ke_part[blockIdx.x] = kp[0];
  }
}

// ------------------------------------------------------------- launchers
static inline unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_zero_i32(hipStream_t s, int* p, int n) {
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(blocks_of(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_bonds(hipStream_t s, const double* pos, int64_t N, const double box[3], const int* nbr,
                        const int* n_nb, double rb, int max_b, BondBufs b, bool reset_flags, const int* need,
                        int* clear) {
  if (reset_flags) hipLaunchKernelGGL(k_fill_zero_i32, dim3(1), dim3(256), 0, s, b.flags, 3);
  const double rb2 = rb * rb * (1.0 + 1e-12);
  hipLaunchKernelGGL(k_bonds, dim3(blocks_of(N, 256)), dim3(256), 0, s, pos, N, box[0], box[1], box[2], 1.0 / box[0],
                     1.0 / box[1], 1.0 / box[2], nbr, n_nb, rb2, max_b, b.nbr, b.n_nb, b.mask, b.ref, b.flags, need,
                     clear);
  return hipGetLastError();
}

hipError_t launch_set_i32(hipStream_t s, int* p, int value) {
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, s, p, value);
  return hipGetLastError();
}

hipError_t launch_neighbors(hipStream_t s, const double* pos, int64_t N, const CellGrid& cg, double rc, double rb,
                            int max_nb, NeighborBufs b) {
  const int n_cells = cg.nc[0] * cg.nc[1] * cg.nc[2];
  const int n_tiles = (n_cells + SCAN_TILE - 1) / SCAN_TILE;
  hipError_t e;
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(blocks_of(n_cells, 256)), dim3(256), 0, s, b.count, n_cells);
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(blocks_of(n_cells, 256)), dim3(256), 0, s, b.fill, n_cells);
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(1), dim3(256), 0, s, b.flags, 3);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_count, dim3(blocks_of(N, 256)), dim3(256), 0, s, pos, N, cg, b.cell_of, b.count);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)n_tiles), dim3(SCAN_TILE), 0, s, b.count, n_cells, b.tile_sums);
  hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(SCAN_TILE), 0, s, b.tile_sums, n_tiles);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)n_tiles), dim3(SCAN_TILE), 0, s, b.count, n_cells, b.tile_sums,
                     b.start);
  hipLaunchKernelGGL(k_cell_fill, dim3(blocks_of(N, 256)), dim3(256), 0, s, N, b.cell_of, b.start, b.fill, b.atoms);
  hipLaunchKernelGGL(k_neighbors, dim3(blocks_of(N, 256)), dim3(256), 0, s, pos, N, cg, rc * rc,
                     rb * rb * (1.0 + 1e-12), b.cell_of, b.start, b.atoms, max_nb, b.nbr, b.n_nb, b.flags);
  hipLaunchKernelGGL(k_reverse, dim3(blocks_of(N, 64)), dim3(64, REV_SLOTS), 0, s, N, b.nbr, b.n_nb, b.rev,
                     b.flags + 1);
  return hipGetLastError();
}

template <int LPA>
static hipError_t launch_pair_kernels(hipStream_t s, const TersoffArgs& a, const TersoffParams& p, const GatherArgs& o,
                                      hipEvent_t e1) {
  // the site kernel for 5..8 pairs: 4 lanes x 2 slots (most atoms of a
  // crystal have 4 bonds, so most waves run one slot round)
  constexpr int SL = LPA == 8 ? 4 : LPA, SPL = LPA / SL;
  hipLaunchKernelGGL((k_tersoff_site<SL, SPL>), dim3(blocks_of(a.N * SL, SITE_WG)), dim3(SITE_WG), 0, s, a, p);
  if (e1) {
    hipError_t e = hipEventRecord(e1, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tersoff_gather<LPA>, dim3(blocks_of(a.N * LPA, 256)), dim3(256), 0, s, a, o);
  return hipSuccess;
}

// ------------------------------------------------ velocity Verlet (NVE)
// The work between two force evaluations.  With MD_KICK2: the second half kick of step s, v += c F / m with c = dt / (2 KE)
// (a = F / (m KE) in A/fs^2), and, with v32, that velocity in float32 (the
// push's velocity input of step s).  With MD_KICK1_DRIFT: the first half
// kick of step s + 1 with the same forces, then the drift x += dt v, wrapped
// into [0, L) per axis (x - floor(x / L) L, then one correction step against
// rounding at the edges), and, with ref, the bond lists' displacement test:
// *need = 1 if the atom is farther than sqrt(thr2) from ref (its position at
// the last bond build).  Each operation is the one the separate kick and
// drift would make, in the same order.
enum { MD_KICK2 = 1, MD_KICK1_DRIFT = 2 };

// One thread per atom component, 64 atoms (192 components, contiguous in
// memory) per work-group; the displacement test sums each atom's three
// squared components in LDS.
constexpr int MD_ATOMS = 64;

__global__ void __launch_bounds__(3 * MD_ATOMS) k_md_step(double* __restrict__ pos, double* __restrict__ vel,
                                                          const double* __restrict__ F,
                                                          const double* __restrict__ mass, double c, double dt,
                                                          double Lx, double Ly, double Lz, int64_t N, int parts,
                                                          float* __restrict__ v32, const double* __restrict__ ref,
                                                          double thr2, int* __restrict__ need) {
  __shared__ double sh[3 * MD_ATOMS];
  const int t = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * (3 * MD_ATOMS) + t;
  double d2 = 0.0;
  if (q < 3 * N) {
    const int a = (int)(q % 3);
    const double m = mass[q / 3];
    const double f = F[q];
    double v = vel[q];
    if (parts & MD_KICK2) {
      v = v + c * f / m;
      if (v32) v32[q] = (float)v;
    }
    if (parts & MD_KICK1_DRIFT) {
      v = v + c * f / m;
      const double L = a == 0 ? Lx : (a == 1 ? Ly : Lz);
      double x = pos[q] + dt * v;
      x -= floor(x / L) * L;
      if (x >= L) x -= L;
      if (x < 0.0) x += L;
      pos[q] = x;
      if (ref) {
        double d = x - ref[q];
        d -= L * rint(d / L);
        d2 = d * d;
      }
    }
    vel[q] = v;
  }
  if (!ref || !(parts & MD_KICK1_DRIFT)) return;   // uniform over the launch
  sh[t] = d2;
  __syncthreads();
  if (t < MD_ATOMS && sh[3 * t] + sh[3 * t + 1] + sh[3 * t + 2] > thr2) *need = 1;
}

hipError_t launch_md_step(hipStream_t s, double* pos, double* vel, const double* F, const double* mass, double c,
                          double dt, const double box[3], int64_t N, bool kick2, bool kick1_drift, float* v32,
                          const double* ref, double thr2, int* need) {
  const int parts = (kick2 ? MD_KICK2 : 0) | (kick1_drift ? MD_KICK1_DRIFT : 0);
  hipLaunchKernelGGL(k_md_step, dim3(blocks_of(N, MD_ATOMS)), dim3(3 * MD_ATOMS), 0, s, pos, vel, F, mass, c, dt,
                     box[0], box[1], box[2], N, parts, v32, ref, thr2, need);
  return hipGetLastError();
}

// ------------------------------------------------ Nose-Hoover thermostat
// Thermostat state on the device: st[0] = xi (1/fs), st[1] = eta (its time
// integral), st[2] = exp(-xi dt / 2), the velocity scale of the current step,
// st[3] = the last kinetic energy (eV).  Kinetic energies are summed in a fixed
// order: per work-group of 64 atoms in an LDS tree, then the work-groups'
// partials by one work-group.

// Sum of the 3 MD_ATOMS values in sh[] (every thread of the work-group calls it).
__device__ __forceinline__ double block_sum_192(double* sh) {
  const int t = threadIdx.x;
  __syncthreads();
  if (t < 64) sh[t] += sh[t + 64] + sh[t + 128];
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  return sh[0];
}

// Partial sums of m v^2, one per work-group of 64 atoms (the thermostat's
// kinetic energy at the entry of an NVT call; later steps take theirs from
// the gather kernel).
__global__ void __launch_bounds__(3 * MD_ATOMS) k_md_ke_partial(const double* __restrict__ vel,
                                                                const double* __restrict__ mass, int64_t N,
                                                                double* __restrict__ part) {
  __shared__ double sh[3 * MD_ATOMS];
  const int t = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * (3 * MD_ATOMS) + t;
  double mv2 = 0.0;
  if (q < 3 * N) mv2 = mass[q / 3] * vel[q] * vel[q];
  sh[t] = mv2;
  const double s = block_sum_192(sh);
  if (t == 0) part[blockIdx.x] = s;
}

// Thermostat update from the kinetic energy K = ke_unit / 2 sum of the
// partials: mode & 1 (end of a step): eta += dt/2 xi, xi += dt/2 G; mode & 2
// (start of a step): xi += dt/2 G, scale = exp(-xi dt / 2), eta += dt/2 xi;
// G = (2K - gkt) / Q.  One work-group of 256 threads.
__global__ void __launch_bounds__(256) k_thermostat(const double* __restrict__ part, int64_t n_part,
                                                    double* __restrict__ st, double dt, double Q, double gkt,
                                                    double ke_unit, int mode) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int64_t k = t; k < n_part; k += 256) acc += part[k];
  sh[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t != 0) return;
  const double K = 0.5 * sh[0] * ke_unit;
  const double G = (2.0 * K - gkt) / Q;
  double xi = st[0], eta = st[1];
  if (mode & 1) {
    eta += 0.5 * dt * xi;
    xi += 0.5 * dt * G;
  }
  if (mode & 2) {
    xi += 0.5 * dt * G;
    st[2] = exp(-0.5 * dt * xi);
    eta += 0.5 * dt * xi;
  }
  st[0] = xi;
  st[1] = eta;
  st[3] = K;
}

// Start of a step under the thermostat: the scale st[2], the first half kick,
// the drift and the bond lists' displacement test, as k_md_step.
__global__ void __launch_bounds__(3 * MD_ATOMS) k_md_nvt_start(double* __restrict__ pos, double* __restrict__ vel,
                                                               const double* __restrict__ F,
                                                               const double* __restrict__ mass, double c, double dt,
                                                               double Lx, double Ly, double Lz, int64_t N,
                                                               const double* __restrict__ st,
                                                               const double* __restrict__ ref, double thr2,
                                                               int* __restrict__ need) {
  __shared__ double sh[3 * MD_ATOMS];
  const int t = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * (3 * MD_ATOMS) + t;
  double d2 = 0.0;
  if (q < 3 * N) {
    const int a = (int)(q % 3);
    const double m = mass[q / 3];
    double v = vel[q] * st[2];
    v = v + c * F[q] / m;
    const double L = a == 0 ? Lx : (a == 1 ? Ly : Lz);
    double x = pos[q] + dt * v;
    x -= floor(x / L) * L;
    if (x >= L) x -= L;
    if (x < 0.0) x += L;
    pos[q] = x;
    vel[q] = v;
    if (ref) {
      double d = x - ref[q];
      d -= L * rint(d / L);
      d2 = d * d;
    }
  }
  if (!ref) return;   // uniform over the launch
  sh[t] = d2;
  __syncthreads();
  if (t < MD_ATOMS && sh[3 * t] + sh[3 * t + 1] + sh[3 * t + 2] > thr2) *need = 1;
}

__global__ void k_thermostat_set(double* st, double xi, double eta) {
  if (threadIdx.x == 0) {
    st[0] = xi;
    st[1] = eta;
    st[2] = 1.0;
    st[3] = 0.0;
  }
}

int64_t md_nvt_parts(int64_t N) { return (N + MD_ATOMS - 1) / MD_ATOMS; }

hipError_t launch_md_ke_partial(hipStream_t s, const double* vel, const double* mass, int64_t N, double* part) {
  hipLaunchKernelGGL(k_md_ke_partial, dim3((unsigned)md_nvt_parts(N)), dim3(3 * MD_ATOMS), 0, s, vel, mass, N, part);
  return hipGetLastError();
}

hipError_t launch_thermostat(hipStream_t s, const double* part, int64_t n_part, double* st, double dt, double Q,
                             double gkt, double ke_unit, int mode) {
  hipLaunchKernelGGL(k_thermostat, dim3(1), dim3(256), 0, s, part, n_part, st, dt, Q, gkt, ke_unit, mode);
  return hipGetLastError();
}

int64_t gather_blocks(int64_t N, int lpa) { return (int64_t)blocks_of(N * lpa, 256); }

hipError_t launch_md_nvt_start(hipStream_t s, double* pos, double* vel, const double* F, const double* mass, double c,
                               double dt, const double box[3], int64_t N, const double* st, const double* ref,
                               double thr2, int* need) {
  hipLaunchKernelGGL(k_md_nvt_start, dim3((unsigned)md_nvt_parts(N)), dim3(3 * MD_ATOMS), 0, s, pos, vel, F, mass, c,
                     dt, box[0], box[1], box[2], N, st, ref, thr2, need);
  return hipGetLastError();
}

hipError_t launch_thermostat_set(hipStream_t s, double* st, double xi, double eta) {
  hipLaunchKernelGGL(k_thermostat_set, dim3(1), dim3(64), 0, s, st, xi, eta);
  return hipGetLastError();
}

int tersoff_lanes(int max_count) {
  int l = 4;
  while (l < max_count) l *= 2;
  return l;
}

hipError_t launch_tersoff(hipStream_t s, const TersoffArgs& a, const TersoffParams& p, const GatherArgs& o, int lpa,
                          hipEvent_t e0, hipEvent_t e1, hipEvent_t e2) {
  hipError_t e = hipSuccess;
  if (e0 && (e = hipEventRecord(e0, s)) != hipSuccess) return e;
  switch (lpa) {
    case 4: e = launch_pair_kernels<4>(s, a, p, o, e1); break;
    case 8: e = launch_pair_kernels<8>(s, a, p, o, e1); break;
    case 16: e = launch_pair_kernels<16>(s, a, p, o, e1); break;
    case 32: e = launch_pair_kernels<32>(s, a, p, o, e1); break;
    case 64: e = launch_pair_kernels<64>(s, a, p, o, e1); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (e2) e = hipEventRecord(e2, s);
  return e;
}

}  // namespace mhc
