// Spectral heat current (Sec. II.C): the virial-velocity correlation of
// Eq. 21 accumulated in float64, and its transform (Eq. 22).
//
//   K^mu(tau) += sum_{t in block} sum_j Wmu[s0 + t - tau][j] V[t][j]
//
// with j = 3i + nu over atoms and the contracted Cartesian index,
// Wmu[s][3i + nu] = W_i^{mu nu}(s) (a ring of the last n_lags - 1 + T steps)
// and V[t][3i + nu] = v_i^nu(s0 + t) (the block's input as pushed).  The
// products of the float32 inputs are formed exactly in float64 and summed in
// float64 in a fixed order, so the result is reproducible bit for bit.
#include "mhc_common.h"
#include "mhc_numeric.h"

namespace mhc {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- ring fill
// ring[(s % ring_len) * 3 + mu][3i + nu] = W[t][i][mu][nu] for the block's
// steps s = s0 + t, t < t_count.  One thread per (t, i, mu): 3 floats in,
// 3 floats out.
__global__ void __launch_bounds__(256) k_shc_ring(const float* __restrict__ W, int t_count, int64_t N,
                                                 float* __restrict__ ring, int64_t ring_len, int64_t ld,
                                                 int64_t s0) {
  const int t = blockIdx.y;
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;     // (i, mu)
  if (t >= t_count || q >= 3 * N) return;
  const int64_t i = q / 3;
  const int mu = (int)(q - i * 3);
  const float* src = W + ((int64_t)t * N + i) * 9 + mu * 3;
  float* dst = ring + (((s0 + t) % ring_len) * 3 + mu) * ld + 3 * i;
  dst[0] = src[0];
  dst[1] = src[1];
  dst[2] = src[2];
}

hipError_t launch_shc_ring(hipStream_t s, const float* W, int t_count, int64_t N, float* ring, int64_t ring_len,
                           int64_t ld, int64_t s0) {
  if (t_count <= 0) return hipSuccess;
  dim3 grid((unsigned)((3 * N + 255) / 256), (unsigned)t_count);
  hipLaunchKernelGGL(k_shc_ring, grid, dim3(256), 0, s, W, t_count, N, ring, ring_len, ld, s0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- products
// Work-group (kc, a, b): steps t in [64a, 64a + 64) x lags tau in
// [64b, 64b + 64) x the 3 components mu, over the dof range
// [kc * dk, kc * dk + dk).  The origins s' = s0 + t - tau of the tile are 127
// consecutive ring rows r = t_loc - tau_loc + 63.  Dofs are staged 32 at a
// time through LDS; a thread holds the 4 x 4 x 3 products of steps 4tt + x
// and lags 4tl + y.  Threads are laid out along diagonals, tt = (tl + k) mod 16
// with k = tid / 16, so the 16 lanes of an LDS pass read one or two virial
// rows (broadcast); velocity rows are stored with one float4 of padding per
// four steps so that those reads spread over all banks.  Rows before the
// first sample, rows after the block's last step and steps past t_count are
// staged as zeros.  The thread's 4 steps are added, then the 16 step groups
// in order, giving part[kc][a][tau][mu] = sum over the tile's steps.
constexpr int SH_T = 64, SH_L = 64, SH_DC = 32;
constexpr int SH_ROWS = SH_T + SH_L - 1;                 // 127
constexpr int SH_VP = SH_T + SH_T / 4;                   // padded step index range of the V tile
constexpr int SH_WS = 3 * SH_DC + 28;                    // W row stride (floats): 96 used + room for the shift
// Row r of the W tile starts at r * SH_WS + 4 * ((r / 4) % 8) floats (the
// shift stays within the row's 28 spare floats): rows four apart, the rows one
// LDS pass reads, then fall on different bank groups.
__device__ __forceinline__ int sh_wrow(int r) { return r * SH_WS + 4 * ((r >> 2) & 7); }
constexpr int SH_WTILE = SH_ROWS * SH_WS + 28;

__global__ void __launch_bounds__(256) k_shc_gram(const float* __restrict__ v, const float* __restrict__ ring,
                                                 int64_t ring_len, int64_t ld, int64_t N3, int t_count,
                                                 int64_t s0, int64_t dk, int n_lags_pad,
                                                 double* __restrict__ part) {
  __shared__ f32x4 vs[SH_DC / 4][SH_VP];
  // the W tile (rows at sh_wrow), reused for the final step-group sums once the products are done
  __shared__ __attribute__((aligned(16))) float ws[SH_WTILE];
  double (*red)[SH_L][3] = reinterpret_cast<double (*)[SH_L][3]>(ws);     // [16][64][3] doubles: 24 KiB
  static_assert(16 * SH_L * 3 * sizeof(double) <= SH_WTILE * sizeof(float), "reduction fits in the W tile");
  const int tid = threadIdx.x;
  const int kc = blockIdx.x;
  const int a = blockIdx.y;
  const int b = blockIdx.z;
  const int tl = tid & 15;
  const int tt = (tl + (tid >> 4)) & 15;
  const int64_t j0 = (int64_t)kc * dk;
  const int64_t j1 = min(N3, j0 + dk);
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
  // Staging of one 32-dof chunk through registers: W as float4 (16-byte
  // aligned: ld and the chunk start are multiples of 4; the ring's pad columns
  // past 3N are zero), V element-wise (its rows are 3N floats long).  The next
  // chunk's loads are issued before the current chunk's products.
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
      if (t < t_count) {
        const float* src = v + (int64_t)t * N3 + j;
        x.x = (j + 0 < j1) ? src[0] : 0.f;
        x.y = (j + 1 < j1) ? src[1] : 0.f;
        x.z = (j + 2 < j1) ? src[2] : 0.f;
        x.w = (j + 3 < j1) ? src[3] : 0.f;
      }
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
#pragma unroll 2
    for (int d4 = 0; d4 < SH_DC / 4; ++d4) {
      f32x4 vv[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) vv[x] = vs[d4][5 * tt + x];           // step 4tt + x, padded index
#pragma unroll
      for (int q = 0; q < 7; ++q) {                                       // q = x - y + 3
        const int r = 4 * (tt - tl) + (q - 3) + (SH_L - 1);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const f32x4 w4 = *reinterpret_cast<const f32x4*>(&ws[sh_wrow(r) + m * SH_DC + 4 * d4]);
          const double w0 = w4.x, w1 = w4.y, w2 = w4.z, w3 = w4.w;
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
    part[(((int64_t)kc * gridDim.y + a) * n_lags_pad + (int64_t)SH_L * b + lt) * 3 + m] = s;
  }
}

// Fixed-order sum of the partials of one block into the running float64 sums
// (Neumaier): one thread per (tau, mu).
__global__ void __launch_bounds__(256) k_shc_accum(const double* __restrict__ part, int n_kc, int n_ttiles,
                                                  int n_lags, int n_lags_pad, double* __restrict__ ksum,
                                                  double* __restrict__ kcomp) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_lags * 3) return;
  const int tau = q / 3, m = q % 3;
  double s = 0.0;
  for (int kc = 0; kc < n_kc; ++kc)
    for (int a = 0; a < n_ttiles; ++a) s += part[(((int64_t)kc * n_ttiles + a) * n_lags_pad + tau) * 3 + m];
  neumaier_add(ksum[q], kcomp[q], s);
}

hipError_t launch_shc_block(hipStream_t s, const float* v, const float* ring, int64_t ring_len, int64_t ld,
                            int64_t N3, int t_count, int64_t s0, int n_lags, int t_block, int64_t dk, int n_kc,
                            double* part, double* ksum, double* kcomp) {
  if (t_count <= 0) return hipSuccess;
  const int n_ttiles = (t_count + SH_T - 1) / SH_T;
  const int n_lags_pad = (n_lags + SH_L - 1) / SH_L * SH_L;
  const int n_ltiles = n_lags_pad / SH_L;
  (void)t_block;
  hipLaunchKernelGGL(k_shc_gram, dim3((unsigned)n_kc, (unsigned)n_ttiles, (unsigned)n_ltiles), dim3(256), 0, s, v,
                     ring, ring_len, ld, N3, t_count, s0, dk, n_lags_pad, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_shc_accum, dim3((unsigned)((n_lags * 3 + 255) / 256)), dim3(256), 0, s, part, n_kc, n_ttiles,
                     n_lags, n_lags_pad, ksum, kcomp);
  return hipGetLastError();
}

// ---------------------------------------------------------------- read-out
// K[tau][mu] = (ksum + kcomp) / (S - tau), zero for lags with no origin.
__global__ void k_shc_finish(const double* __restrict__ ksum, const double* __restrict__ kcomp, int n_lags,
                             int64_t S, double* __restrict__ K) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_lags * 3) return;
  const int tau = q / 3;
  K[q] = (S > tau) ? (ksum[q] + kcomp[q]) / (double)(S - tau) : 0.0;
}

// Eq. 22 on the sampled lags, even extension, trapezoid rule, optional Hann
// window: Kw[w][mu] = dt sum_tau c_tau K[tau][mu] cos(omega_w tau dt), the
// lags summed in order.  One thread per (omega, mu).
__global__ void k_shc_spectrum(const double* __restrict__ K, int n_lags, const double* __restrict__ omega,
                               int n_omega, double dt, int window, double* __restrict__ Kw) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_omega * 3) return;
  const int w = q / 3, m = q % 3;
  const double om = omega[w];
  double s = 0.0;
  for (int tau = 0; tau < n_lags; ++tau) {
    double c = (tau == 0 || tau == n_lags - 1) ? 1.0 : 2.0;
    if (window && n_lags > 1) c *= 0.5 * (1.0 + cos(M_PI * (double)tau / (double)(n_lags - 1)));
    s += c * K[tau * 3 + m] * cos(om * (double)tau * dt);
  }
  Kw[q] = dt * s;
}

hipError_t launch_shc_finish(hipStream_t s, const double* ksum, const double* kcomp, int n_lags, int64_t S,
                             double* K) {
  hipLaunchKernelGGL(k_shc_finish, dim3((unsigned)((n_lags * 3 + 255) / 256)), dim3(256), 0, s, ksum, kcomp, n_lags,
                     S, K);
  return hipGetLastError();
}

hipError_t launch_shc_spectrum(hipStream_t s, const double* K, int n_lags, const double* omega, int n_omega, double dt,
                               int window, double* Kw) {
  if (n_omega <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shc_spectrum, dim3((unsigned)((n_omega * 3 + 255) / 256)), dim3(256), 0, s, K, n_lags, omega,
                     n_omega, dt, window, Kw);
  return hipGetLastError();
}

}  // namespace mhc
