// Spectral heat current (Sec. II.C): the virial-velocity correlation of
// Eq. 21 accumulated in float64, and its transform (Eq. 22).
//
//   K^{mu nu}(tau) += sum_{t in block} sum_i Wmu[s0 + t - tau][nu Np + i] V[t][nu Np + i]
//
// Dofs are stored direction-major, column j = nu * Np + i (Np = N rounded up
// to 32, zero padded): Wmu[s][nu Np + i] = W_i^{mu nu}(s) in a ring of the
// last n_lags - 1 + T steps and V[t][nu Np + i] = v_i^nu(s0 + t).  Every
// work-group's dof range lies inside one direction segment, so its partial
// sums belong to one motion direction nu (the split of Sec. II, remark after
// Eq. 10) and Eq. 21 itself is the sum over nu.  The products of the float32
// inputs are formed exactly in float64 and summed in float64 in a fixed
// order, so the result is reproducible bit for bit.
#include "mhc_common.h"
#include "mhc_numeric.h"

namespace mhc {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- ring fill
// ring[(s % ring_len) * 3 + mu][nu Np + i] = W[t][i][mu][nu] and
// vt[t][nu Np + i] = v[t][i][nu] for the block's steps s = s0 + t, t < t_count
// (ld = 3 Np).  One thread per (t, i): 12 floats in, 12 out, consecutive
// atoms to consecutive columns.
__global__ void __launch_bounds__(256) k_shc_ring(const float* __restrict__ W, const float* __restrict__ v,
                                                 int t_count, int64_t N, int64_t Np, float* __restrict__ ring,
                                                 int64_t ring_len, int64_t ld, int64_t s0, float* __restrict__ vt) {
  const int t = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= t_count || i >= N) return;
  const float* src = W + ((int64_t)t * N + i) * 9;
  float w[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) w[c] = src[c];
  const float* vs = v + ((int64_t)t * N + i) * 3;
  const float v0 = vs[0], v1 = vs[1], v2 = vs[2];
  float* row = ring + ((s0 + t) % ring_len) * 3 * ld + i;
#pragma unroll
  for (int mu = 0; mu < 3; ++mu)
#pragma unroll
    for (int nu = 0; nu < 3; ++nu) row[mu * ld + nu * Np] = w[3 * mu + nu];
  float* vr = vt + (int64_t)t * ld + i;
  vr[0] = v0;
  vr[Np] = v1;
  vr[2 * Np] = v2;
}

hipError_t launch_shc_ring(hipStream_t s, const float* W, const float* v, int t_count, int64_t N, int64_t Np,
                           float* ring, int64_t ring_len, int64_t ld, int64_t s0, float* vt) {
  if (t_count <= 0) return hipSuccess;
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)t_count);
  hipLaunchKernelGGL(k_shc_ring, grid, dim3(256), 0, s, W, v, t_count, N, Np, ring, ring_len, ld, s0, vt);
  return hipGetLastError();
}

// ---------------------------------------------------------------- products
// Work-group (kc, a, b) (a 1-D grid; consecutive ids go to different XCDs,
// so ids are remapped to give each XCD a contiguous range, and the tiles of
// one dof range share that XCD's L2): steps t in [64a, 64a + 64) x lags tau in
// [64b, 64b + 64) x the 3 components mu, over the dof range of direction
// segment nu = kc / n_kcs: columns nu Np + [c dk, c dk + dk) with c = kc % n_kcs,
// cut at nu Np + N.  The origins s' = s0 + t - tau of the tile are 127
// consecutive ring rows r = t_loc - tau_loc + 63.  Dofs are staged 32 at a
// time through LDS; a thread holds the 4 x 4 x 3 products of steps 4tt + x
// and lags 4tl + y.  Threads are laid out along diagonals, tt = (tl + k) mod 16
// with k = tid / 16, so the 16 lanes of an LDS pass read one or two virial
// rows (broadcast); velocity rows are stored with one float4 of padding per
// four steps so that those reads spread over all banks.  Rows before the
// first sample, rows after the block's last step and steps past t_count are
// staged as zeros.  With one wave per SIMD the LDS latency is exposed, so the
// reads of a dof group go out in two batches (diagonals 0..3 and 4..6), each
// issued while the products of the previous batch run.  The thread's 4 steps
// are added, then the 16 step groups in order, giving part[kc][a][tau][mu] =
// sum over the tile's steps.
constexpr int SH_T = 64, SH_L = 64, SH_DC = 32;
constexpr int SH_ROWS = SH_T + SH_L - 1;                 // 127
constexpr int SH_VP = SH_T + SH_T / 4;                   // padded step index range of the V tile
constexpr int SH_WS = 3 * SH_DC + 28;                    // W row stride (floats): 96 used + room for the shift
// Row r of the W tile starts at r * SH_WS + 4 * ((r / 4) % 8) floats (the
// shift stays within the row's 28 spare floats): rows four apart, the rows one
// LDS pass reads, then fall on different bank groups.
__device__ __forceinline__ int sh_wrow(int r) { return r * SH_WS + 4 * ((r >> 2) & 7); }
constexpr int SH_WTILE = SH_ROWS * SH_WS + 28;

__global__ void __launch_bounds__(256) k_shc_gram(const float* __restrict__ vt, const float* __restrict__ ring,
                                                 int64_t ring_len, int64_t ld, int64_t N, int64_t Np, int t_count,
                                                 int64_t s0, int64_t dk, int n_kcs, int n_ttiles,
                                                 int n_lags_pad, double* __restrict__ part) {
  __shared__ f32x4 vs[SH_DC / 4][SH_VP];
  // the W tile (rows at sh_wrow), reused for the final step-group sums once the products are done
  __shared__ __attribute__((aligned(16))) float ws[SH_WTILE];
  double (*red)[SH_L][3] = reinterpret_cast<double (*)[SH_L][3]>(ws);     // [16][64][3] doubles: 24 KiB
  static_assert(16 * SH_L * 3 * sizeof(double) <= SH_WTILE * sizeof(float), "reduction fits in the W tile");
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  const int v = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const int n_tiles = n_ttiles * (n_lags_pad / SH_L);
  const int kc = v / n_tiles;
  const int a = (v % n_tiles) % n_ttiles;
  const int b = (v % n_tiles) / n_ttiles;
  const int tl = tid & 15;
  const int tt = (tl + (tid >> 4)) & 15;
  const int64_t seg0 = (int64_t)(kc / n_kcs) * Np;
  const int64_t j0 = seg0 + (int64_t)(kc % n_kcs) * dk;
  const int64_t j1 = min(seg0 + N, j0 + dk);
  const int64_t row0 = s0 + (int64_t)SH_T * a - (int64_t)SH_L * b - (SH_L - 1);   // origin of row r = 0
  const int64_t s_last = s0 + t_count - 1;

  double acc[4][4][3];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int m = 0; m < 3; ++m) acc[x][y][m] = 0.0;

  // Ring offset of each origin row of the tile (-1: before the first sample
  // or after the block's last step, staged as zeros).
  __shared__ int64_t roff[SH_ROWS];
  if (tid < SH_ROWS) {
    const int64_t sp = row0 + tid;
    roff[tid] = (sp >= 0 && sp <= s_last) ? (sp % ring_len) * 3 * ld : -1;
  }
  __syncthreads();
  // Staging of one 32-dof chunk through registers, W and V as float4 (16-byte
  // aligned: ld, Np, dk and the chunk start are multiples of 4).  A chunk never
  // crosses a multiple of dk or the end of its segment's Np columns, and the
  // pad columns past N are zero in both arrays.  The next chunk's loads are
  // issued before the current chunk's products.
  constexpr int WQ = SH_ROWS * 3 * (SH_DC / 4);           // 3048 float4 per chunk
  constexpr int WPT = (WQ + 255) / 256;                    // 12 per thread
  constexpr int VPT = SH_T * (SH_DC / 4) / 256;            // 2 per thread
  f32x4 wst[WPT], vst[VPT];
  auto load = [&](int64_t jc) {
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      const int e = tid + 256 * k;
      f32x4 x = {0.f, 0.f, 0.f, 0.f};
      if (e < WQ) {
        const int r = e / (3 * SH_DC / 4), rem = e % (3 * SH_DC / 4);
        const int mu = rem / (SH_DC / 4), q = rem % (SH_DC / 4);
        const int64_t off = roff[r];
        const int64_t j = jc + 4 * q;
        if (off >= 0 && j < j1) x = *reinterpret_cast<const f32x4*>(ring + off + mu * ld + j);
      }
      wst[k] = x;
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int e = tid + 256 * k;
      const int tr = e / (SH_DC / 4), q = e % (SH_DC / 4);
      const int t = SH_T * a + tr;
      const int64_t j = jc + 4 * q;
      f32x4 x = {0.f, 0.f, 0.f, 0.f};
      if (t < t_count && j < j1) x = *reinterpret_cast<const f32x4*>(vt + (int64_t)t * ld + j);
      vst[k] = x;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      const int e = tid + 256 * k;
      if (e < WQ) {
        const int r = e / (3 * SH_DC / 4), rem = e % (3 * SH_DC / 4);
        const int mu = rem / (SH_DC / 4), q = rem % (SH_DC / 4);
        *reinterpret_cast<f32x4*>(&ws[sh_wrow(r) + mu * SH_DC + 4 * q]) = wst[k];
      }
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int e = tid + 256 * k;
      const int tr = e / (SH_DC / 4), q = e % (SH_DC / 4);
      vs[q][tr + (tr >> 2)] = vst[k];
    }
  };

  load(j0);
  for (int64_t jc = j0; jc < j1; jc += SH_DC) {
    store();
    __syncthreads();
    if (jc + SH_DC < j1) load(jc + SH_DC);
    // LDS reads one batch ahead of the products: the rows of diagonals
    // q = 0..3 of dof group d4+1 (and its velocities) are read while the
    // products of q = 4..6 of group d4 run, those of q = 4..6 while q = 0..3 run
    auto rd_w = [&](int d4, int q0, int nq, f32x4 (*w)[3]) {
#pragma unroll
      for (int k = 0; k < nq; ++k) {
        const int r = 4 * (tt - tl) + (q0 + k - 3) + (SH_L - 1);
#pragma unroll
        for (int m = 0; m < 3; ++m) w[k][m] = *reinterpret_cast<const f32x4*>(&ws[sh_wrow(r) + m * SH_DC + 4 * d4]);
      }
    };
    auto rd_v = [&](int d4, f32x4* vv) {
#pragma unroll
      for (int x = 0; x < 4; ++x) vv[x] = vs[d4][5 * tt + x];
    };
    auto prod = [&](int q0, int nq, f32x4 (*w)[3], const f32x4* vv) {
#pragma unroll
      for (int k = 0; k < nq; ++k) {
        const int q = q0 + k;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const double w0 = w[k][m].x, w1 = w[k][m].y, w2 = w[k][m].z, w3 = w[k][m].w;
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            const int y = x - (q - 3);
            if (y < 0 || y > 3) continue;
            double s = acc[x][y][m];
            s = fma(w0, (double)vv[x].x, s);
            s = fma(w1, (double)vv[x].y, s);
            s = fma(w2, (double)vv[x].z, s);
            s = fma(w3, (double)vv[x].w, s);
            acc[x][y][m] = s;
          }
        }
      }
    };
    f32x4 vA[4], vB[4], wa[4][3], wb[3][3];
    rd_v(0, vA);
    rd_w(0, 0, 4, wa);
#pragma unroll
    for (int d4 = 0; d4 < SH_DC / 4; ++d4) {
      f32x4* vc = (d4 & 1) ? vB : vA;
      f32x4* vn = (d4 & 1) ? vA : vB;
      rd_w(d4, 4, 3, wb);
      __builtin_amdgcn_sched_barrier(0);
      prod(0, 4, wa, vc);
      __builtin_amdgcn_sched_barrier(0);
      if (d4 + 1 < SH_DC / 4) {
        rd_v(d4 + 1, vn);
        rd_w(d4 + 1, 0, 4, wa);
      }
      __builtin_amdgcn_sched_barrier(0);
      prod(4, 3, wb, vc);
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  }
  // sum the thread's 4 steps, then the 16 step groups in order
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int m = 0; m < 3; ++m)
      red[tt][4 * tl + y][m] = ((acc[0][y][m] + acc[1][y][m]) + acc[2][y][m]) + acc[3][y][m];
  __syncthreads();
  if (tid < SH_L * 3) {
    const int lt = tid / 3, m = tid % 3;
    double s = 0.0;
    for (int g = 0; g < 16; ++g) s += red[g][lt][m];
    part[(((int64_t)kc * n_ttiles + a) * n_lags_pad + (int64_t)SH_L * b + lt) * 3 + m] = s;
  }
}

// Fixed-order sum of the partials of one block into the running float64 sums
// of each motion direction (Neumaier): one thread per (nu, tau, mu), summing
// the n_kcs dof ranges of segment nu and the step tiles in order;
// ksum[nu][tau][mu].
__global__ void __launch_bounds__(256) k_shc_accum(const double* __restrict__ part, int n_kcs, int n_ttiles,
                                                  int n_lags, int n_lags_pad, double* __restrict__ ksum,
                                                  double* __restrict__ kcomp) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= 3 * n_lags * 3) return;
  const int nu = q / (n_lags * 3);
  const int r = q - nu * n_lags * 3;
  const int tau = r / 3, m = r % 3;
  double s = 0.0;
  for (int kc = nu * n_kcs; kc < (nu + 1) * n_kcs; ++kc)
    for (int a = 0; a < n_ttiles; ++a) s += part[(((int64_t)kc * n_ttiles + a) * n_lags_pad + tau) * 3 + m];
  neumaier_add(ksum[q], kcomp[q], s);
}

hipError_t launch_shc_block(hipStream_t s, const float* vt, const float* ring, int64_t ring_len, int64_t ld,
                            int64_t N, int64_t Np, int t_count, int64_t s0, int n_lags, int64_t dk, int n_kcs,
                            double* part, double* ksum, double* kcomp) {
  if (t_count <= 0) return hipSuccess;
  const int n_ttiles = (t_count + SH_T - 1) / SH_T;
  const int n_lags_pad = (n_lags + SH_L - 1) / SH_L * SH_L;
  const int n_ltiles = n_lags_pad / SH_L;
  hipLaunchKernelGGL(k_shc_gram, dim3((unsigned)(3 * n_kcs * n_ttiles * n_ltiles)), dim3(256), 0, s, vt, ring, ring_len,
                     ld, N, Np, t_count, s0, dk, n_kcs, n_ttiles, n_lags_pad, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_shc_accum, dim3((unsigned)((3 * n_lags * 3 + 255) / 256)), dim3(256), 0, s, part, n_kcs,
                     n_ttiles, n_lags, n_lags_pad, ksum, kcomp);
  return hipGetLastError();
}

// ---------------------------------------------------------------- read-out
// Kd[tau][mu][nu] = (ksum + kcomp)[nu][tau][mu] / (S - tau) and
// K[tau][mu] = (Kd[..][0] + Kd[..][1]) + Kd[..][2]; zero for lags with no origin.
__global__ void k_shc_finish(const double* __restrict__ ksum, const double* __restrict__ kcomp, int n_lags,
                             int64_t S, double* __restrict__ K, double* __restrict__ Kd) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_lags * 3) return;
  const int tau = q / 3;
  double k = 0.0;
#pragma unroll
  for (int nu = 0; nu < 3; ++nu) {
    const int e = nu * n_lags * 3 + q;
    const double d = (S > tau) ? (ksum[e] + kcomp[e]) / (double)(S - tau) : 0.0;
    Kd[q * 3 + nu] = d;
    k += d;
  }
  K[q] = k;
}

// Eq. 22 on the sampled lags, even extension, trapezoid rule, optional Hann
// window: Kw[w][m] = dt sum_tau c_tau K[tau][m] cos(omega_w tau dt), the lags
// summed in order, for the nc components m of each lag (3, or 9 for the split).
// One thread per (omega, m).
__global__ void k_shc_spectrum(const double* __restrict__ K, int n_lags, int nc, const double* __restrict__ omega,
                               int n_omega, double dt, int window, double* __restrict__ Kw) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_omega * nc) return;
  const int w = q / nc, m = q % nc;
  const double om = omega[w];
  double s = 0.0;
  for (int tau = 0; tau < n_lags; ++tau) {
    double c = (tau == 0 || tau == n_lags - 1) ? 1.0 : 2.0;
    if (window && n_lags > 1) c *= 0.5 * (1.0 + cos(M_PI * (double)tau / (double)(n_lags - 1)));
    s += c * K[tau * nc + m] * cos(om * (double)tau * dt);
  }
  Kw[q] = dt * s;
}

hipError_t launch_shc_finish(hipStream_t s, const double* ksum, const double* kcomp, int n_lags, int64_t S,
                             double* K, double* Kd) {
  hipLaunchKernelGGL(k_shc_finish, dim3((unsigned)((n_lags * 3 + 255) / 256)), dim3(256), 0, s, ksum, kcomp, n_lags,
                     S, K, Kd);
  return hipGetLastError();
}

hipError_t launch_shc_spectrum(hipStream_t s, const double* K, int n_lags, int nc, const double* omega, int n_omega,
                               double dt, int window, double* Kw) {
  if (n_omega <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shc_spectrum, dim3((unsigned)((n_omega * nc + 255) / 256)), dim3(256), 0, s, K, n_lags, nc,
                     omega, n_omega, dt, window, Kw);
  return hipGetLastError();
}

}  // namespace mhc
