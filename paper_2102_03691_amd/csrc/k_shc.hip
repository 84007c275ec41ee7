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
__device__ __forceinline__ void shc_ring_atom(const float* __restrict__ W, const float* __restrict__ v,
                                              int t_count, int64_t N, int64_t Np, float* __restrict__ ring,
                                              int64_t ring_len, int64_t ld, int64_t s0, float* __restrict__ vt,
                                              int t, int64_t i) {
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

__global__ void __launch_bounds__(256) k_shc_ring(const float* __restrict__ W, const float* __restrict__ v,
                                                 int t_count, int64_t N, int64_t Np, float* __restrict__ ring,
                                                 int64_t ring_len, int64_t ld, int64_t s0, float* __restrict__ vt) {
  shc_ring_atom(W, v, t_count, N, Np, ring, ring_len, ld, s0, vt, blockIdx.y, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// The system of work-group (or block) b of a grouped launch: the last
// descriptor whose first index is <= b (n_sys is small; a linear scan).
__device__ __forceinline__ int shc_system_of(const ShcBlockDesc* __restrict__ d, int n_sys, int64_t b, int which) {
  int q = 0;
  for (int k = 1; k < n_sys; ++k) {
    const int64_t f = which == 0 ? d[k].ring_blk0 : (which == 1 ? d[k].gram_wg0 : d[k].acc_blk0);
    if (f <= b) q = k;
  }
  return q;
}

__global__ void __launch_bounds__(256) k_shc_ring_group(const ShcBlockDesc* __restrict__ d, int n_sys) {
  const int q = shc_system_of(d, n_sys, blockIdx.x, 0);
  const ShcBlockDesc& e = d[q];
  shc_ring_atom(e.W, e.v, e.t_count, e.N, e.Np, e.ring, e.ring_len, e.ld, e.s0, e.vt, blockIdx.y,
                (int64_t)(blockIdx.x - e.ring_blk0) * 256 + threadIdx.x);
}

hipError_t launch_shc_ring_group(hipStream_t s, const ShcBlockDesc* d, int n_sys, int64_t n_blocks, int t_count) {
  if (t_count <= 0 || n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shc_ring_group, dim3((unsigned)n_blocks, (unsigned)t_count), dim3(256), 0, s, d, n_sys);
  return hipGetLastError();
}

hipError_t launch_shc_ring(hipStream_t s, const float* W, const float* v, int t_count, int64_t N, int64_t Np,
                           float* ring, int64_t ring_len, int64_t ld, int64_t s0, float* vt) {
  if (t_count <= 0) return hipSuccess;
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)t_count);
  hipLaunchKernelGGL(k_shc_ring, grid, dim3(256), 0, s, W, v, t_count, N, Np, ring, ring_len, ld, s0, vt);
  return hipGetLastError();
}

// ---------------------------------------------------------------- products
// The partial sums on the FP64 matrix cores, in Gram form.  Work-group
// (kc, mu, a, b) covers steps t in [64a, 64a + 64), lags tau in
// [128b, 128b + 128) and one component mu over the dof range of kc (a 1-D
// grid; consecutive ids go to different XCDs, so ids are remapped to give
// each XCD a contiguous range, and the tiles of one dof range are adjacent,
// sharing that XCD's L2).  Its origins s' = s0 + t - tau are 192 consecutive
// ring rows R (origin row0 + R); wave w takes steps 64a + 16w + c (c < 16)
// and rows R = 16w + rho, rho < 144 (9 blocks of 16), and accumulates
//   G[rho][c] = sum_j Wmu[row0 + 16w + rho][j] V[64a + 16w + c][j]
// with v_mfma_f64_16x16x4f64: A = a block of virial rows, B = velocity rows,
// 4 dofs per product (lane l supplies row or step l % 16 at dof l / 16 of the
// product's 4), and lane l's register i of the result is entry
// [4i + l / 16][l % 16].  The entry with lag tau = 128b + lambda lies at
// rho = 127 + c - lambda, so a work-group's partial for lambda is the sum of
// G along that diagonal over the 4 waves and 16 steps, taken in a fixed order
// after the dof loop.  Of the 9 x 256 products per wave and dof, the 16 x 128
// on those diagonals are used.  Dofs are staged 32 at a time in LDS (float32,
// double-buffered; rows padded to 36 floats) and converted to float64 as the
// operands are read; the products of float32 inputs are exact in float64.  G
// is summed in the LDS of the staging buffers, so a work-group takes 73 KiB
// and two fit on a CU, whose waves hide each other's load and LDS latency.
constexpr int SM_T = 64, SM_L = 128, SM_DC = 32;
constexpr int SM_RB = (SM_L + 16) / 16;                 // 9 row blocks per wave
constexpr int SM_ROWS = SM_T - 16 + 16 * SM_RB;         // 192 staged rows
constexpr int SM_WS = SM_DC + 4;                        // LDS row stride (floats)

typedef double f64x4 __attribute__((ext_vector_type(4)));
// Loads and stores of the tile go through pointers in the global address
// space: a pointer read from a descriptor in memory (grouped launches) is
// otherwise generic to the compiler, whose flat loads also count against the
// LDS wait counter, so that every LDS wait of the loop would wait for the
// next chunk's loads as well.
typedef __attribute__((address_space(1))) const f32x4 gcf32x4;
typedef __attribute__((address_space(1))) double gdouble;

// One work-group's tile; v = its index among the launch's work-groups of this
// system after the XCD remapping.
__device__ __forceinline__ void shc_gram_tile(const float* __restrict__ vt, const float* __restrict__ ring,
                                              int64_t ring_len, int64_t ld, int64_t N, int64_t Np, int t_count,
                                              int64_t s0, int64_t dk, int n_kcs, int n_ttiles, int n_lags_pad,
                                              double* __restrict__ part, int v) {
  // staging buffers, and after the products the G of the 4 waves
  constexpr int WSH = 2 * SM_ROWS * SM_WS, VSH = 2 * SM_T * SM_WS;          // floats
  constexpr int RED = 4 * 16 * SM_RB * 16;                                  // doubles
  constexpr int SMEM = (WSH + VSH) * 4 > RED * 8 ? (WSH + VSH) * 4 : RED * 8;
  __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
  float (*wsh)[SM_ROWS][SM_WS] = reinterpret_cast<float (*)[SM_ROWS][SM_WS]>(smem);
  float (*vsh)[SM_T][SM_WS] = reinterpret_cast<float (*)[SM_T][SM_WS]>(smem + WSH * 4);
  double (*red)[16 * SM_RB][16] = reinterpret_cast<double (*)[16 * SM_RB][16]>(smem);
  __shared__ int64_t roff[SM_ROWS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int n_ab = n_ttiles * (n_lags_pad / SM_L);
  const int kc = v / (3 * n_ab);
  const int mu = (v / n_ab) % 3;
  const int a = (v % n_ab) % n_ttiles;
  const int b = (v % n_ab) / n_ttiles;
  const int64_t seg0 = (int64_t)(kc / n_kcs) * Np;
  const int64_t j0 = seg0 + (int64_t)(kc % n_kcs) * dk;
  const int64_t j1 = min(seg0 + N, j0 + dk);
  const int64_t row0 = s0 + (int64_t)SM_T * a - (int64_t)SM_L * b - (SM_L - 1);
  const int64_t s_last = s0 + t_count - 1;
  if (tid < SM_ROWS) {
    const int64_t sp = row0 + tid;
    roff[tid] = (sp >= 0 && sp <= s_last) ? (sp % ring_len) * 3 * ld + mu * ld : -1;
  }
  __syncthreads();

  // staging of one 32-dof chunk: W as 192 rows x 8 float4 (6 per thread), V
  // as 64 steps x 8 float4 (2 per thread); zeros outside the sampled rows,
  // the block's steps and the dof range
  constexpr int WPT = SM_ROWS * (SM_DC / 4) / 256, VPT = SM_T * (SM_DC / 4) / 256;
  static_assert(WPT * 256 == SM_ROWS * (SM_DC / 4) && VPT * 256 == SM_T * (SM_DC / 4), "staging shape");
  f32x4 wst[WPT], vst[VPT];
  auto load = [&](int64_t jc) {
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      const int e = tid + 256 * k;
      const int r = e / (SM_DC / 4), q = e % (SM_DC / 4);
      const int64_t off = roff[r];
      const int64_t j = jc + 4 * q;
      f32x4 x = {0.f, 0.f, 0.f, 0.f};
      if (off >= 0 && j < j1) x = *(gcf32x4*)(ring + off + j);
      wst[k] = x;
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int e = tid + 256 * k;
      const int tr = e / (SM_DC / 4), q = e % (SM_DC / 4);
      const int t = SM_T * a + tr;
      const int64_t j = jc + 4 * q;
      f32x4 x = {0.f, 0.f, 0.f, 0.f};
      if (t < t_count && j < j1) x = *(gcf32x4*)(vt + (int64_t)t * ld + j);
      vst[k] = x;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      const int e = tid + 256 * k;
      const int r = e / (SM_DC / 4), q = e % (SM_DC / 4);
      *reinterpret_cast<f32x4*>(&wsh[buf][r][4 * q]) = wst[k];
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int e = tid + 256 * k;
      const int tr = e / (SM_DC / 4), q = e % (SM_DC / 4);
      *reinterpret_cast<f32x4*>(&vsh[buf][tr][4 * q]) = vst[k];
    }
  };

  f64x4 acc[SM_RB];
#pragma unroll
  for (int rb = 0; rb < SM_RB; ++rb) acc[rb] = f64x4{0.0, 0.0, 0.0, 0.0};

  load(j0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t jc = j0; jc < j1; jc += SM_DC) {
    const bool more = jc + SM_DC < j1;
    if (more) load(jc + SM_DC);
    // two 16-dof halves; lane (c, g) supplies dofs 16 h + 4 g .. + 3
#pragma unroll
    for (int h = 0; h < SM_DC / 16; ++h) {
      const f32x4 vb = *reinterpret_cast<const f32x4*>(&vsh[buf][16 * wave + c][16 * h + 4 * g]);
      f32x4 wa[SM_RB];
#pragma unroll
      for (int rb = 0; rb < SM_RB; ++rb)
        wa[rb] = *reinterpret_cast<const f32x4*>(&wsh[buf][16 * wave + 16 * rb + c][16 * h + 4 * g]);
      // the 9 independent accumulators between two products on the same one
#pragma unroll
      for (int rb = 0; rb < SM_RB; ++rb)
        acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)wa[rb].x, (double)vb.x, acc[rb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < SM_RB; ++rb)
        acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)wa[rb].y, (double)vb.y, acc[rb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < SM_RB; ++rb)
        acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)wa[rb].z, (double)vb.z, acc[rb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < SM_RB; ++rb)
        acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)wa[rb].w, (double)vb.w, acc[rb], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // lane (c, g) holds G[16 rb + 4 i + g][c] in acc[rb][i]
#pragma unroll
  for (int rb = 0; rb < SM_RB; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wave][16 * rb + 4 * i + g][c] = acc[rb][i];
  __syncthreads();
  if (tid < SM_L) {
    const int lam = tid;
    double s = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int cc = 0; cc < 16; ++cc) s += red[w][(SM_L - 1) + cc - lam][cc];
    ((gdouble*)part)[(((int64_t)kc * n_ttiles + a) * n_lags_pad + (int64_t)SM_L * b + lam) * 3 + mu] = s;
  }
}

// Consecutive work-group ids go to different XCDs: ids are remapped so that
// each XCD takes a contiguous range (the tiles of one dof range are adjacent
// and share that XCD's L2).
__device__ __forceinline__ int shc_xcd_remap(int b, int G) { return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b; }

__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
k_shc_gram(const float* __restrict__ vt, const float* __restrict__ ring, int64_t ring_len, int64_t ld, int64_t N,
           int64_t Np, int t_count, int64_t s0, int64_t dk, int n_kcs, int n_ttiles, int n_lags_pad,
           double* __restrict__ part) {
  shc_gram_tile(vt, ring, ring_len, ld, N, Np, t_count, s0, dk, n_kcs, n_ttiles, n_lags_pad, part,
                shc_xcd_remap(blockIdx.x, gridDim.x));
}

// Several systems' products in one launch: the remapped id picks the system
// (systems in order, each its work-groups in the single-system order).
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
k_shc_gram_group(const ShcBlockDesc* __restrict__ d, int n_sys) {
  const int v = shc_xcd_remap(blockIdx.x, gridDim.x);
  const int q = shc_system_of(d, n_sys, v, 1);
  const ShcBlockDesc& e = d[q];
  shc_gram_tile(e.vt, e.ring, e.ring_len, e.ld, e.N, e.Np, e.t_count, e.s0, e.dk, e.n_kcs, e.n_ttiles,
                e.n_lags_pad, e.part, (int)(v - e.gram_wg0));
}

// Fixed-order sum of the partials of one block into the running float64 sums
// of each motion direction (Neumaier): one thread per (nu, tau, mu), summing
// the n_kcs dof ranges of segment nu and the step tiles in order;
// ksum[nu][tau][mu].
__device__ __forceinline__ void shc_accum_one(const double* __restrict__ part, int n_kcs, int n_ttiles, int n_lags,
                                              int n_lags_pad, double* __restrict__ ksum, double* __restrict__ kcomp,
                                              int q) {
  if (q >= 3 * n_lags * 3) return;
  const int nu = q / (n_lags * 3);
  const int r = q - nu * n_lags * 3;
  const int tau = r / 3, m = r % 3;
  // partials (kc, a) of segment nu, kc-major: loads eight at a time, added in that order
  const int n_p = n_kcs * n_ttiles;
  const double* base = part + ((int64_t)nu * n_p * n_lags_pad + tau) * 3 + m;
  const int64_t stride = (int64_t)n_lags_pad * 3;
  double s = 0.0;
  for (int p0 = 0; p0 < n_p; p0 += 8) {
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = base[(int64_t)min(p0 + k, n_p - 1) * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (p0 + k < n_p) s += x[k];
  }
  neumaier_add(ksum[q], kcomp[q], s);
}

__global__ void __launch_bounds__(256) k_shc_accum(const double* __restrict__ part, int n_kcs, int n_ttiles,
                                                  int n_lags, int n_lags_pad, double* __restrict__ ksum,
                                                  double* __restrict__ kcomp) {
  shc_accum_one(part, n_kcs, n_ttiles, n_lags, n_lags_pad, ksum, kcomp, blockIdx.x * 256 + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_shc_accum_group(const ShcBlockDesc* __restrict__ d, int n_sys) {
  const int q = shc_system_of(d, n_sys, blockIdx.x, 2);
  const ShcBlockDesc& e = d[q];
  shc_accum_one(e.part, e.n_kcs, e.n_ttiles, e.n_lags, e.n_lags_pad, e.ksum, e.kcomp,
                (int)(blockIdx.x - e.acc_blk0) * 256 + threadIdx.x);
}

hipError_t launch_shc_products(hipStream_t s, const float* vt, const float* ring, int64_t ring_len, int64_t ld,
                               int64_t N, int64_t Np, int t_count, int64_t s0, int n_lags, int64_t dk, int n_kcs,
                               double* part) {
  if (t_count <= 0) return hipSuccess;
  const int n_ttiles = (t_count + SM_T - 1) / SM_T;
  const int n_lags_pad = (n_lags + SM_L - 1) / SM_L * SM_L;
  const int n_ltiles = n_lags_pad / SM_L;
  hipLaunchKernelGGL(k_shc_gram, dim3((unsigned)(9 * n_kcs * n_ttiles * n_ltiles)), dim3(256), 0, s, vt, ring,
                     ring_len, ld, N, Np, t_count, s0, dk, n_kcs, n_ttiles, n_lags_pad, part);
  return hipGetLastError();
}

hipError_t launch_shc_gram_group(hipStream_t s, const ShcBlockDesc* d, int n_sys, int64_t n_wgs) {
  if (n_wgs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shc_gram_group, dim3((unsigned)n_wgs), dim3(256), 0, s, d, n_sys);
  return hipGetLastError();
}

hipError_t launch_shc_accum_group(hipStream_t s, const ShcBlockDesc* d, int n_sys, int64_t n_blocks) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shc_accum_group, dim3((unsigned)n_blocks), dim3(256), 0, s, d, n_sys);
  return hipGetLastError();
}

// Work-groups of one system's product launch and blocks of its accumulation
// launch for a block of t_count steps (the grouped launches concatenate them).
int64_t shc_gram_wgs(int t_count, int n_lags, int n_kcs) {
  const int n_ttiles = (t_count + SM_T - 1) / SM_T;
  const int n_ltiles = (n_lags + SM_L - 1) / SM_L;
  return (int64_t)9 * n_kcs * n_ttiles * n_ltiles;
}
int64_t shc_accum_blocks(int n_lags) { return (3 * (int64_t)n_lags * 3 + 255) / 256; }

hipError_t launch_shc_accum(hipStream_t s, const double* part, int t_count, int n_lags, int n_kcs, double* ksum,
                            double* kcomp) {
  if (t_count <= 0) return hipSuccess;
  const int n_ttiles = (t_count + SM_T - 1) / SM_T;
  const int n_lags_pad = (n_lags + SM_L - 1) / SM_L * SM_L;
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
