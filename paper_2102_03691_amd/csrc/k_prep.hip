// Load-time basis conversion and per-block input preparation.
//
// Basis: E^T rows arrive in float64 (eigenvectors e_{i,n}, Sec. II.B) and are
// stored once in the contraction's operand format and fragment layout
// (see mhc_common.h), in bin-sorted slot order.
//
// Inputs: per step, u_j = sqrt(m_i) v_i^alpha (Eq. 13) and
// w^mu_j = W_i^{mu alpha} / sqrt(m_i) (the bracket of Eq. 16), j = 3i + alpha,
// written as the B operand of the contraction; the total potential heat
// current J^mu = sum_i sum_nu W_i^{mu nu} v_i^nu (Eq. 10) is summed in float64
// per chunk of atoms.
#include "mhc_common.h"
#include "mhc_prep_group.h"
#include "mhc_numeric.h"

namespace mhc {

// ------------------------------------------------------------ basis store
// One thread per output piece: FP32 piece = 4 floats, BF16 piece = 8 hi + 8 lo.
// With n3 > 0 the dofs are stored direction-major: dof 3 i + nu at
// k = nu * n3 + i (the direction split's operand order), zero for i >= K / 3.
template <int PREC>
__global__ void __launch_bounds__(256) k_basis_store(const double* __restrict__ rows, int64_t n_rows,
                                                     int64_t K, const int32_t* __restrict__ slot_of_row,
                                                     void* __restrict__ E, int64_t K_pad, int gemv, int64_t n3) {
  constexpr int PW = (PREC == PREC_FP32) ? 4 : 8;     // dofs per piece
  const int64_t pieces = K_pad / PW;
  const int64_t r = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rows || p >= pieces) return;
  const int32_t slot = slot_of_row[r];
  if (slot < 0) return;
  const int64_t k0 = p * PW;
  const double* row = rows + r * K;
  const int64_t rb = slot >> 5;
  const int rr = slot & 31;
  auto val = [&](int64_t k) -> double {
    if (n3 > 0) {
      const int64_t i = k % n3, nu = k / n3;
      return (3 * i < K && nu < 3) ? row[3 * i + nu] : 0.0;
    }
    return k < K ? row[k] : 0.0;
  };
  if constexpr (PREC == PREC_FP32) {
    const int64_t kc = k0 >> 3;
    const int h = (int)((k0 >> 2) & 1);
    const int lane = rr + 32 * h;
    float4 o;
    o.x = (float)val(k0 + 0);
    o.y = (float)val(k0 + 1);
    o.z = (float)val(k0 + 2);
    o.w = (float)val(k0 + 3);
    float4* dst = reinterpret_cast<float4*>(E);
    if (gemv)   // row-major layout of the per-step path
      dst[(int64_t)slot * (K_pad >> 2) + (k0 >> 2)] = o;
    else
      dst[(rb * (K_pad >> 3) + kc) * 64 + lane] = o;
  } else {
    const int64_t kc = k0 >> 4;
    const int h = (int)((k0 >> 3) & 1);
    const int lane = rr + 32 * h;
    uint32_t hi[4], lo[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      uint16_t h0, l0, h1, l1;
      split_bf16_from_f64(val(k0 + e), h0, l0);
      split_bf16_from_f64(val(k0 + e + 1), h1, l1);
      hi[e / 2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
      lo[e / 2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
    uint4* dst = reinterpret_cast<uint4*>(E);
    const int64_t base = ((rb * (K_pad >> 4) + kc) * 2) * 64;
    dst[base + lane] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
    dst[base + 64 + lane] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
  }
}

hipError_t launch_basis_store(hipStream_t s, int prec, const double* rows, int64_t n_rows, int64_t K,
                              const int32_t* slot_of_row, void* E, int64_t K_pad, int gemv, int64_t n3) {
  if (n_rows <= 0) return hipSuccess;
  if (n3 > 0 && (gemv || 3 * n3 != K_pad || 3 * n3 < K)) return hipErrorInvalidValue;
  const int PW = (prec == PREC_FP32) ? 4 : 8;
  const int64_t pieces = K_pad / PW;
  dim3 grid((unsigned)((pieces + 255) / 256), (unsigned)n_rows);
  if (prec == PREC_FP32)
    hipLaunchKernelGGL(k_basis_store<PREC_FP32>, grid, dim3(256), 0, s, rows, n_rows, K, slot_of_row, E, K_pad,
                       gemv, n3);
  else
    hipLaunchKernelGGL(k_basis_store<PREC_BF16X3>, grid, dim3(256), 0, s, rows, n_rows, K, slot_of_row, E, K_pad,
                       0, n3);
  return hipGetLastError();
}

// e4m3 storage: one work-group per row.  s_n = max_j |E[j][n]| / 448 (the
// per-mode scale), then 16-dof pieces of E/s_n are rounded to e4m3 (and, for
// the hi/lo form, the residual to a second e4m3).  Piece layout per row block
// (32 rows), lane l = row%32 + 32*h, dofs k = 64*kc + 32*h + 16*q + [0, 16):
//   FP8X3  unit kc*256 + (part*2 + q)*64 + lane     (part 0 = hi, 1 = lo)
//   FP8    unit kc*128 + q*64 + lane
template <bool X3>
__global__ void __launch_bounds__(256) k_basis_store_fp8(const double* __restrict__ rows, int64_t K,
                                                         const int32_t* __restrict__ slot_of_row, void* __restrict__ E,
                                                         int64_t K_pad, float* __restrict__ row_scale, int64_t n3) {
  __shared__ double sh[256];
  const int64_t r = blockIdx.x;
  const int32_t slot = slot_of_row[r];
  if (slot < 0) return;
  const double* row = rows + r * K;
  double mx = 0.0;
  for (int64_t k = threadIdx.x; k < K; k += 256) mx = fmax(mx, fabs(row[k]));
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  const double scale = sh[0] > 0.0 ? sh[0] / (double)FP8_MAX : 1.0;
  if (threadIdx.x == 0) row_scale[slot] = (float)scale;
  const double inv = 1.0 / scale;
  const int64_t rb = slot >> 5;
  const int rr = slot & 31;
  const int64_t per_blk = (X3 ? 4 : 2) * K_pad;                 // 16-byte units per row block
  uint4* dst = reinterpret_cast<uint4*>(E) + rb * per_blk;
  for (int64_t p = threadIdx.x; p < K_pad / 16; p += 256) {
    const int64_t k0 = p * 16;
    float x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t k = k0 + e;
      double v = 0.0;
      if (n3 > 0) {   // direction-major: dof 3 i + nu at k = nu n3 + i
        const int64_t i = k % n3, nu = k / n3;
        if (3 * i < K && nu < 3) v = row[3 * i + nu];
      } else if (k < K) {
        v = row[k];
      }
      x[e] = (float)(v * inv);
    }
    uint32_t hi[4], lo[4];
    quant16_fp8(x, hi, lo, X3);
    const int64_t kc = k0 >> 6;
    const int h = (int)((k0 >> 5) & 1), q = (int)((k0 >> 4) & 1);
    const int lane = rr + 32 * h;
    if (X3) {
      dst[kc * 256 + (0 * 2 + q) * 64 + lane] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
      dst[kc * 256 + (1 * 2 + q) * 64 + lane] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    } else {
      dst[kc * 128 + q * 64 + lane] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
    }
  }
}

hipError_t launch_basis_store_fp8(hipStream_t s, bool x3, const double* rows, int64_t n_rows, int64_t K,
                                  const int32_t* slot_of_row, void* E, int64_t K_pad, float* row_scale, int64_t n3) {
  if (n_rows <= 0) return hipSuccess;
  if (n3 > 0 && (3 * n3 != K_pad || 3 * n3 < K)) return hipErrorInvalidValue;
  if (x3)
    hipLaunchKernelGGL(k_basis_store_fp8<true>, dim3((unsigned)n_rows), dim3(256), 0, s, rows, K, slot_of_row, E, K_pad,
                       row_scale, n3);
  else
    hipLaunchKernelGGL(k_basis_store_fp8<false>, dim3((unsigned)n_rows), dim3(256), 0, s, rows, K, slot_of_row, E,
                       K_pad, row_scale, n3);
  return hipGetLastError();
}

// Per-column scales of the e4m3 activations: for step t and channel c,
// s_{c,t} = max_j |B_c[t][j]| / 448 (1 if the column is zero).  Work-group
// (t, cc) takes the maxima over atoms [cc A, (cc+1) A), A = COLSCALE_ATOMS,
// into col_part[cc][c][t]; the input prep combines the chunks (max is exact
// in any order).  With tab != NULL the input pointers are read from tab[0],
// tab[1] (device memory), so a captured graph can be fed new inputs.  With
// dir in {0, 1, 2} the virial channels hold column dir of W only (the
// motion-direction split), and their maxima are taken over that column.
__device__ __forceinline__ void col_scale_body(const float* v, const float* W, const float* __restrict__ sqrt_m,
                                               const float* __restrict__ inv_sqrt_m, int64_t N, int t_count,
                                               int t_pad, float* __restrict__ col_part,
                                               const float* const* __restrict__ tab, int dir, int t, int cc) {
  __shared__ float sh[4][256];
  if (tab) {
    v = tab[0];
    W = tab[1];
  }
  float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;
  if (t < t_count) {
    const int64_t i1 = min(N, (int64_t)(cc + 1) * COLSCALE_ATOMS);
    for (int64_t i = (int64_t)cc * COLSCALE_ATOMS + threadIdx.x; i < i1; i += 256) {
      const float* vp = v + ((int64_t)t * N + i) * 3;
      const float* Wp = W + ((int64_t)t * N + i) * 9;
      const float sm = sqrt_m[i], ism = inv_sqrt_m[i];
      m0 = fmaxf(m0, sm * fmaxf(fmaxf(fabsf(vp[0]), fabsf(vp[1])), fabsf(vp[2])));
      if (dir < 0) {
        m1 = fmaxf(m1, ism * fmaxf(fmaxf(fabsf(Wp[0]), fabsf(Wp[1])), fabsf(Wp[2])));
        m2 = fmaxf(m2, ism * fmaxf(fmaxf(fabsf(Wp[3]), fabsf(Wp[4])), fabsf(Wp[5])));
        m3 = fmaxf(m3, ism * fmaxf(fmaxf(fabsf(Wp[6]), fabsf(Wp[7])), fabsf(Wp[8])));
      } else {
        m1 = fmaxf(m1, ism * fabsf(Wp[dir]));
        m2 = fmaxf(m2, ism * fabsf(Wp[3 + dir]));
        m3 = fmaxf(m3, ism * fabsf(Wp[6 + dir]));
      }
    }
  }
  sh[0][threadIdx.x] = m0; sh[1][threadIdx.x] = m1; sh[2][threadIdx.x] = m2; sh[3][threadIdx.x] = m3;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = fmaxf(sh[c][threadIdx.x], sh[c][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 4) col_part[((int64_t)cc * 4 + threadIdx.x) * t_pad + t] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_col_scale(const float* v, const float* W,
                                                   const float* __restrict__ sqrt_m,
                                                   const float* __restrict__ inv_sqrt_m, int64_t N, int t_count,
                                                   int t_pad, float* __restrict__ col_part,
                                                   const float* const* __restrict__ tab, int dir) {
  col_scale_body(v, W, sqrt_m, inv_sqrt_m, N, t_count, t_pad, col_part, tab, dir, blockIdx.x, blockIdx.y);
}

// System of a grouped work-group: the last i with wg0[i] <= wg (wg0 ascending).
__device__ __forceinline__ int group_system(const PrepDesc* __restrict__ d, int n, int wg, bool prep) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int w0 = prep ? d[mid].wg0_prep : d[mid].wg0_cs;
    if (w0 <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The column maxima of every system of a group in one launch: work-group wg
// is work-group (t, cc) of its system's own grid (t_pad x n_cc).
__global__ void __launch_bounds__(256) k_col_scale_group(const PrepDesc* __restrict__ d, int n, int t_count) {
  const int i = group_system(d, n, blockIdx.x, false);
  const PrepDesc& s = d[i];
  const int local = blockIdx.x - s.wg0_cs;
  col_scale_body(nullptr, nullptr, s.sqrt_m, s.inv_sqrt_m, s.N, t_count, s.t_pad, s.col_part, s.tab, -1,
                 local % s.t_pad, local / s.t_pad);
}

hipError_t launch_col_scale(hipStream_t s, const float* v, const float* W, const float* sqrt_m,
                            const float* inv_sqrt_m, int64_t N, int t_count, int t_pad, float* col_part,
                            const float* const* tab, int dir) {
  const int n_cc = (int)((N + COLSCALE_ATOMS - 1) / COLSCALE_ATOMS);
  hipLaunchKernelGGL(k_col_scale, dim3((unsigned)t_pad, (unsigned)n_cc), dim3(256), 0, s, v, W, sqrt_m, inv_sqrt_m,
                     N, t_count, t_pad, col_part, tab, dir);
  return hipGetLastError();
}

// ------------------------------------------------------------- input prep
// Work-group = 32 atoms (96 dofs) x 32 steps, 256 threads.
// Phase A: thread (tl = tid / 8, sub = tid % 8) handles atoms sub, sub+8, ...
//          of step tl: channels into LDS and the Eq. 10 partial in float64.
// Phase B: the LDS tile is written out in the operand layout.
// Motion-direction split (dir in {0, 1, 2}): the virial channels keep only
// dof alpha = dir of each atom, W_i^{mu dir} / sqrt(m_i), so the contraction
// gives the bracket of Eq. 16 restricted to that direction; the velocity
// channel is whole.  jd_part then receives the split Eq. 10 partials
// sum_i W_i^{mu dir} v_i^dir beside the whole ones.
constexpr int PREP_T = 32;
constexpr int PREP_K = 3 * ATOMS_PER_PREP;   // 96 dofs

template <int MODE>   // 0 = plain, 1 = FP32, 2 = BF16 hi/lo, 3 = e4m3, 4 = e4m3 hi/lo fragments
__device__ __forceinline__ void input_prep_body(const float* v, const float* W, const float* __restrict__ sqrt_m,
                                                const float* __restrict__ inv_sqrt_m, int64_t N, int t_count,
                                                int t_pad, void* __restrict__ B, int64_t K_pad,
                                                double* __restrict__ jt_part, float* __restrict__ col_scale,
                                                const float* __restrict__ col_part,
                                                const float* const* __restrict__ tab, int dir,
                                                double* __restrict__ jd_part, int chunk, int n_chunks, int tb) {
  __shared__ float ch[4][PREP_T][PREP_K + 4];
  __shared__ float csc[4][PREP_T];
  if (tab) {   // inputs named through device memory (graph replay)
    v = tab[0];
    W = tab[1];
  }
  const int tid = threadIdx.x;
  const int tl = tid >> 3;
  const int sub = tid & 7;
  const int t = tb * PREP_T + tl;
  const int64_t i0 = (int64_t)chunk * ATOMS_PER_PREP;

  // dir == DIR_ALL: all three directions in one operand, K direction-major
  // (dof (i, nu) at k = nu * K_pad / 3 + i), and the split partials of every
  // direction; otherwise atom-major (k = 3 i + alpha)
  const bool dm = (dir == DIR_ALL);
  double j0 = 0.0, j1 = 0.0, j2 = 0.0;
  double dd[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};   // split partials [nu][mu] (dir >= 0)
#pragma unroll
  for (int q = 0; q < ATOMS_PER_PREP / 8; ++q) {
    const int a = sub + 8 * q;
    const int64_t i = i0 + a;
    float u[3] = {0.f, 0.f, 0.f}, w[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    if (t < t_count && i < N) {
      const float* vp = v + ((int64_t)t * N + i) * 3;
      const float* Wp = W + ((int64_t)t * N + i) * 9;
      const float vx = vp[0], vy = vp[1], vz = vp[2];
      const float sm = sqrt_m[i], ism = inv_sqrt_m[i];
      float Wl[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) Wl[c] = Wp[c];
      u[0] = sm * vx; u[1] = sm * vy; u[2] = sm * vz;
#pragma unroll
      for (int mu = 0; mu < 3; ++mu)
#pragma unroll
        for (int nu = 0; nu < 3; ++nu) w[mu][nu] = (dir < 0 || dm || nu == dir) ? Wl[3 * mu + nu] * ism : 0.f;
      // Eq. 10 in float64: J^mu += sum_nu W^{mu nu} v^nu
      const double dvx = vx, dvy = vy, dvz = vz;
      j0 += (double)Wl[0] * dvx + (double)Wl[1] * dvy + (double)Wl[2] * dvz;
      j1 += (double)Wl[3] * dvx + (double)Wl[4] * dvy + (double)Wl[5] * dvz;
      j2 += (double)Wl[6] * dvx + (double)Wl[7] * dvy + (double)Wl[8] * dvz;
      if (dm) {
        const double vv[3] = {dvx, dvy, dvz};
#pragma unroll
        for (int nu = 0; nu < 3; ++nu)
#pragma unroll
          for (int mu = 0; mu < 3; ++mu) dd[nu][mu] += (double)Wl[3 * mu + nu] * vv[nu];
      } else if (dir >= 0) {
        const double vd = dir == 0 ? dvx : (dir == 1 ? dvy : dvz);
        dd[0][0] += (double)Wl[dir] * vd;
        dd[0][1] += (double)Wl[3 + dir] * vd;
        dd[0][2] += (double)Wl[6 + dir] * vd;
      }
    }
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      const int pos = dm ? al * ATOMS_PER_PREP + a : 3 * a + al;
      ch[0][tl][pos] = u[al];
      ch[1][tl][pos] = w[0][al];
      ch[2][tl][pos] = w[1][al];
      ch[3][tl][pos] = w[2][al];
    }
  }
  // fixed-order reduction over the 8 threads of a step
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) {
    j0 += __shfl_xor(j0, off);
    j1 += __shfl_xor(j1, off);
    j2 += __shfl_xor(j2, off);
  }
  if (sub == 0 && t < t_pad) {
    double* jp = jt_part + ((int64_t)t * n_chunks + chunk) * 3;
    jp[0] = j0; jp[1] = j1; jp[2] = j2;
  }
  if (dir >= 0) {
    // jd_part[nu][t][chunk][mu] (one direction: nu = 0 only)
    const int n_nu = dm ? 3 : 1;
#pragma unroll
    for (int nu = 0; nu < 3; ++nu) {
      if (nu >= n_nu) break;
#pragma unroll
      for (int off = 1; off < 8; off <<= 1)
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) dd[nu][mu] += __shfl_xor(dd[nu][mu], off);
      if (sub == 0 && t < t_pad) {
        double* jp = jd_part + ((int64_t)nu * t_pad + t) * n_chunks * 3 + (int64_t)chunk * 3;
        jp[0] = dd[nu][0]; jp[1] = dd[nu][1]; jp[2] = dd[nu][2];
      }
    }
  }
  __syncthreads();

  const int64_t k_base = (int64_t)chunk * PREP_K;
  // global k of local position l (the first of a piece; pieces never cross a
  // direction's 32 positions)
  const int64_t n3 = K_pad / 3;
  auto k_of = [&](int l) -> int64_t {
    return dm ? (int64_t)(l / ATOMS_PER_PREP) * n3 + (int64_t)chunk * ATOMS_PER_PREP + l % ATOMS_PER_PREP
              : k_base + l;
  };
  if constexpr (MODE == 0) {
    // plain [t][4][K_pad]: 4 * 32 * 96 floats, coalesced along k
    for (int idx = tid; idx < 4 * PREP_T * PREP_K; idx += 256) {
      const int k = idx % PREP_K;
      const int c = (idx / PREP_K) & 3;
      const int tt = idx / (4 * PREP_K);
      const int tg = tb * PREP_T + tt;
      if (tg >= t_count) continue;
      float* Bp = reinterpret_cast<float*>(B);
      Bp[((int64_t)tg * 4 + c) * K_pad + k_base + k] = ch[c][tt][k];
    }
  } else if constexpr (MODE == 1) {
    // FP32 fragments: piece = (c, 4-dof group g, column tt): 4 * 24 * 32 pieces
    const int ntb = t_pad / 32;
    const int64_t KC = K_pad >> 3;
    float4* Bp = reinterpret_cast<float4*>(B);
    for (int idx = tid; idx < 4 * (PREP_K / 4) * PREP_T; idx += 256) {
      const int tt = idx & 31;
      const int g = (idx >> 5) % (PREP_K / 4);
      const int c = (idx >> 5) / (PREP_K / 4);
      const int64_t k = k_of(4 * g);
      const int64_t kc = k >> 3;
      const int h = (int)((k >> 2) & 1);
      const int64_t cb = (int64_t)c * ntb + tb;
      float4 o = make_float4(ch[c][tt][4 * g], ch[c][tt][4 * g + 1], ch[c][tt][4 * g + 2], ch[c][tt][4 * g + 3]);
      Bp[(cb * KC + kc) * 64 + tt + 32 * h] = o;
    }
  } else if constexpr (MODE == 3 || MODE == 4) {
    // e4m3 fragments: piece = (c, 16-dof group g, column tt) of B/s_{c,t}.
    // The scales of this tile's steps from the atom-chunk maxima (the
    // work-groups of chunk 0 also publish them for the contraction epilogue).
    if (tid < 4 * PREP_T) {
      const int c = tid / PREP_T, tt = tid % PREP_T;
      const int tg = tb * PREP_T + tt;
      const int n_cc = (int)((N + COLSCALE_ATOMS - 1) / COLSCALE_ATOMS);
      float mx = 0.f;
      for (int cc = 0; cc < n_cc; ++cc) mx = fmaxf(mx, col_part[((int64_t)cc * 4 + c) * t_pad + tg]);
      const float sc = mx > 0.f ? mx / FP8_MAX : 1.f;
      csc[c][tt] = sc;
      if (chunk == 0) col_scale[c * t_pad + tg] = sc;
    }
    __syncthreads();
    constexpr bool X3 = (MODE == 4);
    const int ntb = t_pad / 32;
    const int64_t per_blk = (X3 ? 4 : 2) * K_pad;
    uint4* Bp = reinterpret_cast<uint4*>(B);
    for (int idx = tid; idx < 4 * (PREP_K / 16) * PREP_T; idx += 256) {
      const int tt = idx & 31;
      const int g = (idx >> 5) % (PREP_K / 16);
      const int c = (idx >> 5) / (PREP_K / 16);
      const int64_t k0 = k_of(16 * g);
      const int64_t cb = (int64_t)c * ntb + tb;
      const float inv = 1.f / csc[c][tt];
      float x[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) x[e] = ch[c][tt][16 * g + e] * inv;
      uint32_t hi[4], lo[4];
      quant16_fp8(x, hi, lo, X3);
      const int64_t kc = k0 >> 6;
      const int h = (int)((k0 >> 5) & 1), q = (int)((k0 >> 4) & 1);
      const int lane = tt + 32 * h;
      uint4* dst = Bp + cb * per_blk;
      if (X3) {
        dst[kc * 256 + (0 * 2 + q) * 64 + lane] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        dst[kc * 256 + (1 * 2 + q) * 64 + lane] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
      } else {
        dst[kc * 128 + q * 64 + lane] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
      }
    }
  } else {
    // BF16 fragments: piece = (c, 8-dof group g, column tt), hi and lo
    const int ntb = t_pad / 32;
    const int64_t KC = K_pad >> 4;
    uint4* Bp = reinterpret_cast<uint4*>(B);
    for (int idx = tid; idx < 4 * (PREP_K / 8) * PREP_T; idx += 256) {
      const int tt = idx & 31;
      const int g = (idx >> 5) % (PREP_K / 8);
      const int c = (idx >> 5) / (PREP_K / 8);
      const int64_t k = k_of(8 * g);
      const int64_t kc = k >> 4;
      const int h = (int)((k >> 3) & 1);
      const int64_t cb = (int64_t)c * ntb + tb;
      uint32_t hi[4], lo[4];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        uint16_t h0, l0, h1, l1;
        split_bf16_from_f32(ch[c][tt][8 * g + e], h0, l0);
        split_bf16_from_f32(ch[c][tt][8 * g + e + 1], h1, l1);
        hi[e / 2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
        lo[e / 2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
      }
      const int64_t base = ((cb * KC + kc) * 2) * 64 + tt + 32 * h;
      Bp[base] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
      Bp[base + 64] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    }
  }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_input_prep(const float* v, const float* W,
                                                    const float* __restrict__ sqrt_m,
                                                    const float* __restrict__ inv_sqrt_m, int64_t N,
                                                    int t_count, int t_pad, void* __restrict__ B,
                                                    int64_t K_pad, double* __restrict__ jt_part,
                                                    float* __restrict__ col_scale,
                                                    const float* __restrict__ col_part,
                                                    const float* const* __restrict__ tab, int dir,
                                                    double* __restrict__ jd_part) {
  input_prep_body<MODE>(v, W, sqrt_m, inv_sqrt_m, N, t_count, t_pad, B, K_pad, jt_part, col_scale, col_part, tab,
                        dir, jd_part, blockIdx.x, gridDim.x, blockIdx.y);
}

// The input prep of every system of a group in one launch: work-group wg is
// work-group (chunk, tb) of its system's own grid (n_chunks x t_pad / 32).
template <int MODE>
__global__ void __launch_bounds__(256) k_input_prep_group(const PrepDesc* __restrict__ d, int n, int t_count) {
  const int i = group_system(d, n, blockIdx.x, true);
  const PrepDesc& s = d[i];
  const int local = blockIdx.x - s.wg0_prep;
  input_prep_body<MODE>(nullptr, nullptr, s.sqrt_m, s.inv_sqrt_m, s.N, t_count, s.t_pad, s.B, s.K_pad, s.jt_part,
                        s.col_scale, s.col_part, s.tab, s.dir, s.jd_part, local % s.n_chunks, s.n_chunks,
                        local / s.n_chunks);
}

hipError_t launch_prep_group(hipStream_t s, int prec, const PrepDesc* d, int n, int t_count, int n_wg_cs,
                             int n_wg_prep) {
  if (prec == PREC_FP8 || prec == PREC_FP8X3) {
    hipLaunchKernelGGL(k_col_scale_group, dim3((unsigned)n_wg_cs), dim3(256), 0, s, d, n, t_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
#define MHC_PREPG(M) hipLaunchKernelGGL(k_input_prep_group<M>, dim3((unsigned)n_wg_prep), dim3(256), 0, s, d, n, t_count)
  if (prec == PREC_FP32) MHC_PREPG(1);
  else if (prec == PREC_BF16X3) MHC_PREPG(2);
  else if (prec == PREC_FP8) MHC_PREPG(3);
  else MHC_PREPG(4);
#undef MHC_PREPG
  return hipGetLastError();
}

// Non-finite scan of n floats: any NaN or Inf stores 1 to *flag (every
// writer stores the same value, so the unordered stores need no atomic).
// 16-byte loads where the pointer allows, the ragged ends one float at a time.
__global__ void __launch_bounds__(256) k_nonfinite(const float* __restrict__ p, int64_t n, int* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t head = (int64_t)((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15) / 4;
  const int64_t h = head < n ? head : n;
  const int64_t n4 = (n - h) / 4;
  const float4* q = reinterpret_cast<const float4*>(p + h);
  bool bad = false;
  for (int64_t i = tid; i < n4; i += stride) {
    const float4 x = q[i];
    bad |= !isfinite(x.x) | !isfinite(x.y) | !isfinite(x.z) | !isfinite(x.w);
  }
  if (tid < h) bad |= !isfinite(p[tid]);
  const int64_t tail = h + 4 * n4;
  if (tail + tid < n) bad |= !isfinite(p[tail + tid]);
  if (bad) *flag = 1;
}

hipError_t launch_nonfinite(hipStream_t s, const float* p, int64_t n, int* flag) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n / 4 + 255) / 256;
  const unsigned grid = (unsigned)(want < 2048 ? (want < 1 ? 1 : want) : 2048);
  hipLaunchKernelGGL(k_nonfinite, dim3(grid), dim3(256), 0, s, p, n, flag);
  return hipGetLastError();
}

hipError_t launch_input_prep(hipStream_t s, int prec, int plain, const float* v, const float* W,
                             const float* sqrt_m, const float* inv_sqrt_m, int64_t N, int t_count, int t_pad,
                             void* B, int64_t K_pad, double* jt_part, float* col_scale,
                             const float* col_part, const float* const* tab, int dir, double* jd_part) {
  const int n_chunks = (int)((N + ATOMS_PER_PREP - 1) / ATOMS_PER_PREP);
  if (dir == DIR_ALL && (plain || K_pad % 96 != 0 || K_pad / 3 < (int64_t)n_chunks * ATOMS_PER_PREP))
    return hipErrorInvalidValue;
  dim3 grid((unsigned)n_chunks, (unsigned)((t_pad + PREP_T - 1) / PREP_T));
#define MHC_PREP(M)                                                                                          \
  hipLaunchKernelGGL(k_input_prep<M>, grid, dim3(256), 0, s, v, W, sqrt_m, inv_sqrt_m, N, t_count, t_pad, B, \
                     K_pad, jt_part, col_scale, col_part, tab, dir, jd_part)
  if (plain) MHC_PREP(0);
  else if (prec == PREC_FP32) MHC_PREP(1);
  else if (prec == PREC_BF16X3) MHC_PREP(2);
  else if (prec == PREC_FP8) MHC_PREP(3);
  else MHC_PREP(4);
#undef MHC_PREP
  return hipGetLastError();
}

}  // namespace mhc
