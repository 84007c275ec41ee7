// Frequency binning, float64 time accumulation and the GKMA correlation.
//
//   J_b^mu(t) = sum_{n in b} J_n^mu(t)                 (frequency bins, Sec. III.A)
//   HNEMA:  S_b^mu += sum_t J_b^mu(t), S^mu += sum_t J^mu(t)   (Eq. 19 numerator)
//   GKMA:   C_b^{mu nu}(tau) += sum_t J_b^mu(t) J^nu(t - tau)  (Eq. 17 integrand)
// Modes are stored in bin-sorted slots, so bin b is the contiguous slot range
// [bin_off[b], bin_off[b+1]).  All sums are float64 in a fixed order (no
// atomics), so results are reproducible bit for bit; long running sums use
// Neumaier compensation.
#include "mhc_common.h"
#include "mhc_back_group.h"
#include "mhc_numeric.h"

namespace mhc {

// Fixed-order sum of one double per thread over a 256-thread work-group.
// Every thread receives the result.
__device__ __forceinline__ double block_sum256(double x, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = x;
  __syncthreads();
#pragma unroll
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ reduce
__device__ __forceinline__ void reduce_body(ReduceArgs a, int b) {
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  if (a.t0_dev) a.t0 = *a.t0_dev;
  if (b < a.nb) {
    const int64_t lo = a.bin_off[b], hi = a.bin_off[b + 1];
    const int64_t n = hi - lo;
    if (!a.layout_g) {
      // HNEMA-only: parts [p][slot][mu], already summed over each part's steps
      double s3[3] = {0.0, 0.0, 0.0};
      const int per_part = (int)(n * 3);
      for (int p = 0; p < a.n_parts; ++p) {
        const float* base = a.in + ((int64_t)p * a.M_pad + lo) * 3;
        int mu = tid % 3;                       // e % 3, and 256 % 3 == 1
        for (int e = tid; e < per_part; e += 256) {
          const double val = (double)base[e];
          if (mu == 0) s3[0] += val; else if (mu == 1) s3[1] += val; else s3[2] += val;
          mu = (mu == 2) ? 0 : mu + 1;
        }
      }
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        const double tot = block_sum256(s3[mu], sh);
        if (tid == 0) neumaier_add(a.hsum[b * 3 + mu], a.hcomp[b * 3 + mu], tot);
      }
    } else {
      // GKMA: X[(b*3+mu)][t] = sum over the bin's segment rows in segment order
      // (from k_reduce_seg); thread t of the work-group, steps strided by 256.
      const int64_t P = (int64_t)a.n_seg + a.nb;
      const int64_t sg0 = lo / REDUCE_SEG, sg1 = (hi - 1) / REDUCE_SEG;
      const int64_t xo = a.xoff_dev ? *a.xoff_dev : a.xoff;
      double h3[3] = {0.0, 0.0, 0.0};
      for (int t = tid; t < a.t_count; t += 256) {
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          double s = 0.0;
          if (n > 0)
            for (int64_t sg = sg0; sg <= sg1; ++sg) s += a.seg_part[((int64_t)mu * P + sg + b) * a.ld + t];
          a.X[((int64_t)b * 3 + mu) * a.ldx + xo + t] = s;
          if (a.bring) a.bring[((int64_t)b * a.ring_len + (a.t0 + t) % a.ring_len) * 3 + mu] = s;
          h3[mu] += s;
        }
      }
      if (a.hsum) {
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const double tot = block_sum256(h3[mu], sh);
          if (tid == 0) neumaier_add(a.hsum[b * 3 + mu], a.hcomp[b * 3 + mu], tot);
        }
      }
    }
    return;
  }
  // last work-group: per-step total current of Eq. 10 (already summed over atoms)
  double h3[3] = {0.0, 0.0, 0.0};
  const int64_t xo = a.X ? (a.xoff_dev ? *a.xoff_dev : a.xoff) : 0;
  for (int t = tid; t < a.t_count; t += 256) {
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const double j = a.jtot[t * 3 + mu];
      h3[mu] += j;
      if (a.X) {
        a.X[((int64_t)a.nb * 3 + mu) * a.ldx + xo + t] = j;
        a.ring[((a.t0 + t) % a.ring_len) * 3 + mu] = j;
      }
    }
  }
  if (a.tsum) {
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const double tot = block_sum256(h3[mu], sh);
      if (tid == 0) neumaier_add(a.tsum[mu], a.tcomp[mu], tot);
    }
  }
  if (a.tdsum) {   // motion-direction split of the Eq. 10 total
    double d3[3] = {0.0, 0.0, 0.0};
    for (int t = tid; t < a.t_count; t += 256)
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) d3[mu] += a.jdtot[t * 3 + mu];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const double tot = block_sum256(d3[mu], sh);
      if (tid == 0) neumaier_add(a.tdsum[mu], a.tdcomp[mu], tot);
    }
  }
}

__global__ void __launch_bounds__(256) k_reduce(ReduceArgs a) { reduce_body(a, blockIdx.x); }

// Eq. 10 summed over atoms: one wave per step adds the float64 partials of
// the atom chunks in a fixed order.
__device__ __forceinline__ void total_body(const double* __restrict__ jt_part, int n_chunks,
                                           double* __restrict__ jtot, int t) {
  const int lane = threadIdx.x;
  double j0 = 0.0, j1 = 0.0, j2 = 0.0;
  const double* p = jt_part + (int64_t)t * n_chunks * 3;
  for (int c = lane; c < n_chunks; c += 64) {
    j0 += p[c * 3 + 0];
    j1 += p[c * 3 + 1];
    j2 += p[c * 3 + 2];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    j0 += __shfl_xor(j0, off);
    j1 += __shfl_xor(j1, off);
    j2 += __shfl_xor(j2, off);
  }
  if (lane == 0) {
    jtot[t * 3 + 0] = j0;
    jtot[t * 3 + 1] = j1;
    jtot[t * 3 + 2] = j2;
  }
}

__global__ void __launch_bounds__(64) k_total(const double* __restrict__ jt_part, int n_chunks,
                                              double* __restrict__ jtot) {
  total_body(jt_part, n_chunks, jtot, blockIdx.x);
}

hipError_t launch_total(hipStream_t s, const double* jt_part, int n_chunks, int t_count, double* jtot) {
  if (t_count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_total, dim3((unsigned)t_count), dim3(64), 0, s, jt_part, n_chunks, jtot);
  return hipGetLastError();
}

// GKMA segment pass: TT = 64, 128 or 256 lanes per segment (the smallest that
// covers t_count; steps strided by TT), 256 / TT segments per work-group.  A
// segment's REDUCE_SEG slots are summed in slot order, bin by bin, into
// seg_part[mu][seg + b][t] (every bin the segment touches).
__device__ __forceinline__ void reduce_seg_body(const ReduceArgs& a, int blk) {
  __shared__ int32_t sb[4][REDUCE_SEG];
  const int tid = threadIdx.x;
  const int TT = a.t_count <= 64 ? 64 : (a.t_count <= 128 ? 128 : 256);
  const int G = 256 / TT;
  const int g = tid / TT, tl = tid % TT;
  const int64_t seg = (int64_t)blk * G + g;
  const int64_t slot0 = seg * REDUCE_SEG;
  if (tl < REDUCE_SEG) sb[g][tl] = (seg < a.n_seg && slot0 + tl < a.M_pad) ? a.slot_bin[slot0 + tl] : -1;
  __syncthreads();
  if (seg >= a.n_seg) return;
  const int64_t P = (int64_t)a.n_seg + a.nb;
  const float* __restrict__ in = a.in;
  double* __restrict__ out = a.seg_part;
  for (int t = tl; t < a.t_count; t += TT) {
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      // all of the segment's values first (independent, unconditional loads:
      // padding rows exist in the contraction output and hold zeros), then
      // the bin-by-bin sums in slot order
      const float* col = in + ((int64_t)mu * a.M_pad + slot0) * a.ld + t;
      float x[REDUCE_SEG];
#pragma unroll
      for (int q = 0; q < REDUCE_SEG; ++q) x[q] = col[(int64_t)q * a.ld];
      double s = 0.0;
      int cur = sb[g][0];
#pragma unroll
      for (int q = 0; q < REDUCE_SEG; ++q) {
        const int bq = sb[g][q];
        if (bq != cur) {
          if (cur >= 0) out[((int64_t)mu * P + seg + cur) * a.ld + t] = s;
          cur = bq;
          s = 0.0;
        }
        s += (double)(bq >= 0 ? x[q] : 0.f);
      }
      if (cur >= 0) out[((int64_t)mu * P + seg + cur) * a.ld + t] = s;
    }
  }
}

__global__ void __launch_bounds__(256) k_reduce_seg(ReduceArgs a) { reduce_seg_body(a, blockIdx.x); }

hipError_t launch_reduce(hipStream_t s, const ReduceArgs& a) {
  if (a.layout_g && a.t_count > 0 && a.n_seg > 0) {
    const int TT = a.t_count <= 64 ? 64 : (a.t_count <= 128 ? 128 : 256);
    const int G = 256 / TT;
    hipLaunchKernelGGL(k_reduce_seg, dim3((unsigned)((a.n_seg + G - 1) / G)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)(a.nb + 1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// -------------------------------------------------------------- correlation
// Sums are stored lag-contiguous: C[(r*3 + nu)*L + tau].
// Work-group tile: 64 rows r x 64 lags tau (x 3 nu); X and the needed window
// of the history ring are staged in LDS per chunk of 64 steps.  The update of
// one chunk is a float64 matrix product on the matrix cores: with the window
// entry q = j + 63 - lambda holding the total at step j of the chunk minus lag
// tau0 + lambda,
//   C[r][lambda][nu] += sum_j X[r][j] * window[nu][j + 63 - lambda],
// done by v_mfma_f64_16x16x4f64 over 4 steps at a time (A = 16 rows x 4
// steps of X, B = 4 steps x 16 lags of the window, its lane (k, c) reading
// entry j + k + 63 - lambda_c).  Wave w owns rows 16w .. 16w + 15 and all 64
// lags (4 blocks of 16) for the 3 nu: 12 accumulators; lane l's register i of
// an accumulator is row 4i + l / 16, lag l % 16 of its block.  Steps past the
// block's end are staged as zeros, so every 4-step product is complete.
constexpr int CT = 64;   // steps per chunk
constexpr int CR = 64;   // rows per tile
constexpr int CL = 64;   // lags per tile

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void corr_body(const double* __restrict__ X, int64_t ldx, int t_count, int64_t R3,
                                          int L, const double* __restrict__ ring, int64_t ring_len, int64_t t0,
                                          double* __restrict__ csum, double* __restrict__ ccomp,
                                          const int64_t* __restrict__ t0_dev, const int64_t* __restrict__ tbuf_dev,
                                          int bx, int by) {
  if (tbuf_dev) {
    // buffered steps ending with this block (the same value in every thread)
    const int64_t tb = *tbuf_dev;
    if (tb <= 0) return;
    t0 = *t0_dev + t_count - tb;
    t_count = (int)tb;
  } else if (t0_dev) {
    t0 = *t0_dev;
  }
  __shared__ double xs[CT][CR + 2];          // xs[t][r]
  __shared__ double rs[3][CT + CL + 2];      // ring window, rs[nu][q]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)bx * CR;
  const int tau0 = by * CL;
  f64x4 acc[4][3];                           // [lag block][nu]
#pragma unroll
  for (int lb = 0; lb < 4; ++lb)
#pragma unroll
    for (int n = 0; n < 3; ++n) acc[lb][n] = f64x4{0.0, 0.0, 0.0, 0.0};

  // Staging of a chunk: X rows r0.. (t-major in LDS) and the ring window
  // (q in [0, CT + CL) <-> global time t0 + tc - tau0 - (CL - 1) + q).  The
  // next chunk's values are loaded into registers while the current chunk's
  // products run, and written to LDS after them.  Loads are unconditional,
  // from clamped in-range addresses, with the value selected afterwards, so
  // that they all issue back to back.
  constexpr int XPT = CR * CT / 256;                    // X values per thread
  constexpr int RPT = ((CT + CL) * 3 + 255) / 256;      // ring values per thread
  double xr[XPT], rr[RPT];
  auto fetch = [&](int tc) {
#pragma unroll
    for (int k = 0; k < XPT; ++k) {
      const int idx = tid + 256 * k;
      const int j = idx % CT, i = idx / CT;
      const int64_t r = r0 + i;
      const int tg = tc + j;
      const double x = X[min(r, R3 - 1) * ldx + min(tg, t_count - 1)];
      xr[k] = (r < R3 && tg < t_count) ? x : 0.0;
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int idx = min(tid + 256 * k, (CT + CL) * 3 - 1);
      const int q = idx / 3, nu = idx % 3;
      const int64_t gt = t0 + tc - tau0 - (CL - 1) + q;
      const bool ok = gt >= 0 && gt < t0 + t_count;
      const double x = ring[(max(gt, (int64_t)0) % ring_len) * 3 + nu];
      rr[k] = ok ? x : 0.0;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int k = 0; k < XPT; ++k) {
      const int idx = tid + 256 * k;
      xs[idx % CT][idx / CT] = xr[k];
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int idx = tid + 256 * k;
      if (idx < (CT + CL) * 3) rs[idx % 3][idx / 3] = rr[k];
    }
  };
  fetch(0);
  for (int tc = 0; tc < t_count; tc += CT) {
    stage();
    __syncthreads();
    if (tc + CT < t_count) fetch(tc + CT);
    const int jmax = min(CT, t_count - tc);
    for (int j0 = 0; j0 < jmax; j0 += 4) {
      const int j = j0 + g;
      const double a = xs[j][16 * wave + c];
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        const int q = j + (CL - 1) - (16 * lb + c);
#pragma unroll
        for (int n = 0; n < 3; ++n) acc[lb][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, rs[n][q], acc[lb][n], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // Neumaier update of the lane's 4 rows x 4 lags x 3: every load issues
  // from a clamped in-range address, only the stores are conditional
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + 16 * wave + 4 * i + g;
    const int64_t rc = min(r, R3 - 1);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      double sm[4], cp[4];
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        const int64_t o = (rc * 3 + n) * L + min(tau0 + 16 * lb + c, L - 1);
        sm[lb] = csum[o];
        cp[lb] = ccomp[o];
      }
#pragma unroll
      for (int lb = 0; lb < 4; ++lb) {
        const int tau = tau0 + 16 * lb + c;
        neumaier_add(sm[lb], cp[lb], acc[lb][n][i]);
        if (r < R3 && tau < L) {
          const int64_t o = (r * 3 + n) * L + tau;
          csum[o] = sm[lb];
          ccomp[o] = cp[lb];
        }
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_corr(const double* __restrict__ X, int64_t ldx, int t_count, int64_t R3,
                                              int L, const double* __restrict__ ring, int64_t ring_len, int64_t t0,
                                              double* __restrict__ csum, double* __restrict__ ccomp,
                                              const int64_t* __restrict__ t0_dev, const int64_t* __restrict__ tbuf_dev,
                                              int64_t ring_zs, int64_t out_zs) {
  // grid z: one history ring of 3 columns and one slice of sums per z
  corr_body(X, ldx, t_count, R3, L, ring + (int64_t)blockIdx.z * ring_zs, ring_len, t0,
            csum + (int64_t)blockIdx.z * out_zs, ccomp + (int64_t)blockIdx.z * out_zs, t0_dev, tbuf_dev, blockIdx.x,
            blockIdx.y);
}

hipError_t launch_corr(hipStream_t s, const double* X, int64_t ldx, int t_count, int64_t R3, int L,
                       const double* ring, int64_t ring_len, int64_t t0, double* csum, double* ccomp,
                       const int64_t* t0_dev, const int64_t* tbuf_dev, int nz, int64_t ring_zs, int64_t out_zs) {
  if (t_count <= 0 || nz <= 0) return hipSuccess;
  dim3 grid((unsigned)((R3 + CR - 1) / CR), (unsigned)((L + CL - 1) / CL), (unsigned)nz);
  hipLaunchKernelGGL(k_corr, grid, dim3(256), 0, s, X, ldx, t_count, R3, L, ring, ring_len, t0, csum, ccomp, t0_dev,
                     tbuf_dev, ring_zs, out_zs);
  return hipGetLastError();
}

// ----------------------------------------------------------------- read-out
__global__ void __launch_bounds__(256) k_corr_finish(const double* __restrict__ csum, const double* __restrict__ ccomp,
                                                     const double* __restrict__ psum, const double* __restrict__ pcomp,
                                                     int64_t R3, int L, int64_t S, double dt,
                                                     double* __restrict__ corr, double* __restrict__ integral) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // series (r, nu)
  if (q >= R3 * 3) return;
  double G = 0.0, prev = 0.0;
  for (int tau = 0; tau < L; ++tau) {
    const int64_t src = q * L + tau;               // sums are lag-contiguous
    const int64_t o = (int64_t)tau * R3 * 3 + q;   // output [tau][r][nu]
    const int64_t cnt = S - tau;
    double sum = csum[src] + ccomp[src];
    if (psum) sum += psum[src] + pcomp[src];       // steps not yet in the running sums
    const double c = (cnt > 0) ? sum / (double)cnt : 0.0;
    corr[o] = c;
    if (tau > 0) G += dt * 0.5 * (prev + c);
    integral[o] = G;
    prev = c;
  }
}

hipError_t launch_corr_finish(hipStream_t s, const double* csum, const double* ccomp, const double* psum,
                              const double* pcomp, int64_t R3, int L, int64_t S, double dt, double* corr,
                              double* integral) {
  const int64_t n = R3 * 3;
  hipLaunchKernelGGL(k_corr_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, csum, ccomp, psum, pcomp, R3,
                     L, S, dt, corr, integral);
  return hipGetLastError();
}

__global__ void k_hnema_finish(const double* __restrict__ sum, const double* __restrict__ comp, int64_t n, int64_t S,
                               double* __restrict__ avg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) avg[i] = (S > 0) ? (sum[i] + comp[i]) / (double)S : 0.0;
}

hipError_t launch_hnema_finish(hipStream_t s, const double* sum, const double* comp, int64_t n, int64_t S,
                               double* avg) {
  hipLaunchKernelGGL(k_hnema_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sum, comp, n, S, avg);
  return hipGetLastError();
}

// ------------------------------------------------------- grouped back end
// The back end of every system of a group in four launches (totals, segment
// sums, bin sums, correlations); work-group w belongs to the last system i
// with wg0[i] <= w (systems with no work-groups in a launch are skipped).
__device__ __forceinline__ int back_system(const int* __restrict__ wg0, int n, int w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wg0[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(64) k_total_group(const BackDesc* __restrict__ d, int t_count) {
  const BackDesc& s = d[blockIdx.x / t_count];
  total_body(s.jt_part, s.n_chunks, s.jtot, blockIdx.x % t_count);
}

__global__ void __launch_bounds__(256) k_reduce_seg_group(const ReduceArgs* __restrict__ a,
                                                          const int* __restrict__ wg0, int n) {
  const int i = back_system(wg0, n, blockIdx.x);
  reduce_seg_body(a[i], blockIdx.x - wg0[i]);
}

__global__ void __launch_bounds__(256) k_reduce_group(const ReduceArgs* __restrict__ a, const int* __restrict__ wg0,
                                                      int n) {
  const int i = back_system(wg0, n, blockIdx.x);
  reduce_body(a[i], blockIdx.x - wg0[i]);
}

__global__ void __launch_bounds__(256) k_corr_group(const BackDesc* __restrict__ d, const int* __restrict__ wg0, int n,
                                                    int t_count) {
  const int i = back_system(wg0, n, blockIdx.x);
  const BackDesc& s = d[i];
  const int local = blockIdx.x - wg0[i];
  corr_body(s.X, s.ldx, t_count, s.R3, s.L, s.ring, s.ring_len, 0, s.csum, s.ccomp, s.t0_dev, s.tbuf_dev,
            local % s.n_rt, local / s.n_rt);
}

hipError_t launch_back_group(hipStream_t s, const BackGroup& b, int n, int t_count) {
  hipLaunchKernelGGL(k_total_group, dim3((unsigned)(n * t_count)), dim3(64), 0, s, b.d, t_count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (b.n_wg_seg > 0) {
    hipLaunchKernelGGL(k_reduce_seg_group, dim3((unsigned)b.n_wg_seg), dim3(256), 0, s, b.red, b.wg0_seg, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reduce_group, dim3((unsigned)b.n_wg_red), dim3(256), 0, s, b.red, b.wg0_red, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (b.n_wg_corr > 0) {
    hipLaunchKernelGGL(k_corr_group, dim3((unsigned)b.n_wg_corr), dim3(256), 0, s, b.d, b.wg0_corr, n, t_count);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace mhc
