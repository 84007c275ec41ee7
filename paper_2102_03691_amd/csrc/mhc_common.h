// Internal declarations shared by the host library and the HIP kernels of
// libmodalhc.  Not part of the public ABI (see include/mhc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhc {

// ---------------------------------------------------------------- layouts
// Row block = 32 slots (modes in bin-sorted order); the contraction dimension
// (dofs, K) is split into chunks whose size matches one matrix-core operand:
//   FP32   chunk of 8 dofs:  fragment [64 lanes][4 floats]   (1 KiB)
//   BF16   chunk of 16 dofs: fragment [64 lanes][8 bf16]     (1 KiB) x {hi, lo}
// Inside a fragment, lane l carries row (l % 32) and dofs
//   FP32: k = 8*kc + 4*(l/32) + e,  e = 0..3
//   BF16: k = 16*kc + 8*(l/32) + e, e = 0..7
// Eigenvectors (A operand) and activations (B operand) use the same map, so
// every matrix-core product pairs equal k on both sides.
//
//   E  FP32   [M_pad/32][K_pad/8][64][4]            float
//   E  BF16   [M_pad/32][K_pad/16][2 (hi,lo)][64][8] bf16
//   E  FP8    [M_pad/32][K_pad/64][2 (q)][64][16] e4m3        (+ per-slot scale)
//   E  FP8X3  [M_pad/32][K_pad/64][2 (hi,lo)][2 (q)][64][16] e4m3
//   B  plain  [T][4][K_pad]                           float  (per-step path)
//   B  FP32   [4*NTB][K_pad/8][64][4]                 float  (cb = c*NTB + tb)
//   B  BF16   [4*NTB][K_pad/16][2][64][8]             bf16
// Channels c: 0 = u = sqrt(m) v, 1..3 = w^mu = W^{mu .} / sqrt(m).
constexpr int DIR_ALL = 3;     // input prep: every direction, K direction-major
constexpr int K_ALIGN = 128;    // K_pad multiple (one e4m3 stage is 128 dofs)
constexpr int K_ALIGN_GEMV = 512;  // per-step path: rows of 128 units, 2 x 64 lanes per iteration pair
constexpr int M_ALIGN = 256;    // M_pad multiple
constexpr int ATOMS_PER_PREP = 32;  // atoms per input-prep work-group (96 dofs)
constexpr int COLSCALE_ATOMS = 1024;  // atoms per work-group of the e4m3 column maxima

enum Prec { PREC_FP32 = 0, PREC_BF16X3 = 1, PREC_FP8 = 2, PREC_FP8X3 = 3 };

// ------------------------------------------------------------- launchers
// Every launcher queues work on `s` and returns the launch status.

// Convert n_rows float64 E^T rows (device, row r = mode r0 + r) into the
// storage layout.  slot_of_row[r] is the destination slot (-1 = skip).
// gemv = 1 (FP32 only): the row-major layout of the per-step path.  n3 > 0
// (T-batched layouts, K_pad = 3 n3): dofs direction-major, dof 3 i + nu
// at k = nu n3 + i (the one-contraction direction split).
hipError_t launch_basis_store(hipStream_t s, int prec, const double* rows, int64_t n_rows,
                              int64_t K, const int32_t* slot_of_row, void* E, int64_t K_pad, int gemv, int64_t n3);

// e4m3 basis store: per-mode scale s_n = max|E[.][n]| / 448 into row_scale[slot],
// then E/s_n as e4m3 (x3: plus the e4m3 residual); n3 as for launch_basis_store.
hipError_t launch_basis_store_fp8(hipStream_t s, bool x3, const double* rows, int64_t n_rows, int64_t K,
                                  const int32_t* slot_of_row, void* E, int64_t K_pad, float* row_scale, int64_t n3);

// Maxima behind the per-(channel, step) scales of the e4m3 activations, per
// chunk of COLSCALE_ATOMS atoms: col_part[chunk][c][t_pad] (the input prep
// turns them into col_scale).  With tab != NULL, v and W are ignored and read
// from tab[0], tab[1] (device).  dir = -1: whole virial rows; dir in {0,1,2}:
// the virial channels of the motion-direction split (column dir of W only).
hipError_t launch_col_scale(hipStream_t s, const float* v, const float* W, const float* sqrt_m,
                            const float* inv_sqrt_m, int64_t N, int t_count, int t_pad, float* col_part,
                            const float* const* tab, int dir);

// Input preparation for one block of t_pad columns (t_count real steps):
// B operand in the layout of `prec` (or plain when plain != 0) and the
// per-atom-chunk partial total currents jt_part[t][chunk][3] (float64).
// e4m3 precisions divide by col_scale[c][t] = max over chunks of col_part
// / 448 (1 for a zero column), which the chunk-0 work-groups also store in
// col_scale for the contraction epilogue.  tab as for launch_col_scale.
// dir in {0,1,2} builds the virial channels of the motion-direction split
// (W_i^{mu dir} / sqrt(m_i) on dof alpha = dir only) and writes the split
// partial currents sum_i W_i^{mu dir} v_i^dir to jd_part[t][chunk][3];
// dir = DIR_ALL (T-batched layouts) builds the whole operand with K
// direction-major (dof 3 i + nu at k = nu K_pad / 3 + i; K_pad / 3 covers
// every atom chunk) and writes the split partials of all three directions to
// jd_part[nu][t][chunk][3]; dir = -1 builds the whole operand atom-major and
// leaves jd_part alone.
hipError_t launch_input_prep(hipStream_t s, int prec, int plain, const float* v, const float* W,
                             const float* sqrt_m, const float* inv_sqrt_m, int64_t N,
                             int t_count, int t_pad, void* B, int64_t K_pad, double* jt_part,
                             float* col_scale, const float* col_part, const float* const* tab, int dir,
                             double* jd_part);

// Non-finite scan: stores 1 to *flag when any of the n floats at p (device)
// is NaN or Inf; the caller clears *flag first (launch_fill_i32).
hipError_t launch_nonfinite(hipStream_t s, const float* p, int64_t n, int* flag);

// Per-step matrix-vector path (FP32): for steps t = 0..n_steps-1 of a plain
// B buffer, J_n^mu = Xdot_n A_n^mu for every slot.  Output either
//   hnema: out[t][M_pad][3]   (layout_g == 0)
//   gkma : out[3][M_pad][ld]  at column t (layout_g == 1)
hipError_t launch_gemv_f32(hipStream_t s, const float* E, const float* B, int n_steps, int64_t M_pad,
                           int64_t K_pad, float* out, int layout_g, int64_t ld);

// Geometry of one system's T-batched contraction (plain data, shared with
// the grouped launch, which keeps an array of these in device memory).
struct GemmGeom {
  const void* E;              // basis (A operand)
  const void* B;              // activations (B operand)
  float* out;                 // modal currents
  int64_t K_pad, M_pad;
  int ntb, n_ntiles, n_stages;
  int64_t total_iters, ipw;   // iteration space and iterations per work-group
  int layout_g;
  const float* row_scale;     // e4m3 only: per-slot scale of E
  const float* col_scale;     // e4m3 only: [4][ntb*32] activation scales
  // direction split as one contraction (grouped systems): s3 > 0 stages per
  // third of K, out regions of `region` floats per direction, and two bracket
  // slots per work-group in ws (0 / nullptr: an unsplit system)
  int s3;
  int64_t region;
  float* ws;
};
struct GroupTile {
  int sys;
  int tile;
};

// Tile shapes of the matrix-core contraction (slots x t-blocks of 32 steps):
// 0 = 128 x 4, 1 = 256 x 2, 2 = 256 x 1.
int gemm_shape_rows(int shape);
int gemm_shape_tbs(int shape);
bool gemm_shape_valid(int shape, int ntb);
void gemm_geom(int prec, int shape, const void* E, const void* B, float* out, int64_t M_pad, int64_t K_pad, int ntb,
               int layout_g, const float* row_scale, const float* col_scale, GemmGeom* g, int* n_mtiles);

// Persistent launch over the tiles of several systems (same precision and
// tile shape): n_wg work-groups pull tiles[] in order through *counter, which
// must be zero at launch (launch_fill_i32).  with_dir: some system has the
// one-contraction direction split (GemmGeom::s3 > 0).
hipError_t launch_gemm_group(hipStream_t s, int prec, int shape, const GemmGeom* d_sys, const GroupTile* d_tiles,
                             int n_tiles, int* counter, int n_wg, bool with_dir);
hipError_t launch_fill_i32(hipStream_t s, int* p, int n, int v);

// T-batched matrix-core contraction with fused modal-current epilogue.
//   ntb     t-blocks of 32 steps in the block (t_pad = 32*ntb)
//   hnema:  out[ntile][M_pad][3]   sum over the tile's steps
//   gkma :  out[3][M_pad][t_pad]
//   ws      stream-K workspace (ws_floats floats); n_cu = compute units
//   sched   0 = automatic, 1 = one tile per work-group, 2 = stream-K
// Returns the number of column tiles through *n_parts.
hipError_t launch_gemm(hipStream_t s, int prec, const void* E, const void* B, int64_t M_pad,
                       int64_t K_pad, int ntb, float* out, int layout_g, int* n_parts, float* ws,
                       int64_t ws_floats, int* tile_cnt, int n_cu, int sched, const float* row_scale,
                       const float* col_scale, int* used);

// Motion-direction split as one contraction: K ordered direction-major
// (third nu = dofs (i, nu) at k = nu*n3 + i, n3 a multiple of the precision's
// k-stage, stage_dofs_of), out = three regions of `region` floats (direction
// nu at out + nu * region), each laid out as launch_gemm's out.  ws holds two
// bracket slots per work-group (ws_floats floats); n_cu = compute units;
// row_scale / col_scale as for launch_gemm (e4m3; whole-column activation
// scales, the same for every third).
hipError_t launch_gemm_dir(hipStream_t s, int prec, const void* E, const void* B, int64_t M_pad, int64_t n3, int ntb,
                           float* out, int64_t region, int layout_g, int* n_parts, float* ws, int64_t ws_floats,
                           int n_cu, const float* row_scale, const float* col_scale);

// dofs per k-stage of a precision's T-batched contraction.
int stage_dofs_of(int prec);

// Bin reduction + float64 accumulation.
//   HNEMA-only: part sums in[n_parts][M_pad][3] -> hsum/hcomp[nb][3] (Neumaier)
//   GKMA:       per-step in[3][M_pad][ld]      -> X[(b*3+mu)][ld] float64, and
//               (if hsum) the HNEMA sums of the same steps.
//   The last work-group distributes the per-step totals jtot[t][3]:
//   X rows 3*nb..3*nb+2 (GKMA), the history ring (GKMA), tsum/tcomp (HNEMA).
// GKMA layout: the slots are first summed in segments of REDUCE_SEG (bin by
// bin inside each segment) into seg_part[mu][seg + b][ld] (float64; row seg + b
// is unique because bins are slot-ordered), then each bin adds its segments'
// rows in order.  slot_bin[slot] is the bin of a slot (-1: padding).
constexpr int REDUCE_SEG = 64;
struct ReduceArgs {
  const float* in; int layout_g; int n_parts; int64_t M_pad; int64_t ld; int t_count;
  const int32_t* bin_off; int nb;
  const int32_t* slot_bin; double* seg_part; int n_seg;      // GKMA segment pass
  const double* jtot;
  double* hsum; double* hcomp; double* tsum; double* tcomp;  // HNEMA (may be null)
  double* X;                                                 // GKMA (may be null)
  double* ring; int64_t ring_len; int64_t t0;                // GKMA history
  const int64_t* t0_dev;    // if set, the block's first step index is read here instead of t0
  const double* jdtot; double* tdsum; double* tdcomp;        // split Eq. 10 totals (may be null)
  double* bring;            // cross-correlation: bin history [nb][ring_len][3] (may be null)
  int64_t ldx;              // leading dimension of X (>= ld: X keeps several blocks)
  int64_t xoff;             // column of X where this block's first step goes
  const int64_t* xoff_dev;  // if set, xoff is read here (the group's block table)
};
hipError_t launch_reduce(hipStream_t s, const ReduceArgs& a);

// Per-step total current: jtot[t][mu] = sum over atom chunks of jt_part[t][chunk][mu].
hipError_t launch_total(hipStream_t s, const double* jt_part, int n_chunks, int t_count, double* jtot);

// GKMA correlation update: for r < R3 = 3(nb+1), tau < L, nu < 3
//   C[r][nu][tau] += sum_{t < t_count, t0+t-tau >= 0} X[r][t] * ring[(t0+t-tau) % ring_len][nu]
// accumulated with Neumaier compensation into csum/ccomp (lag-contiguous);
// X column t holds global step t0 + t.  With tbuf_dev (the group's block
// table) the kernels read t0 from t0_dev and the number of buffered steps tb
// from tbuf_dev: tb = 0 means no update this block, otherwise the update
// covers the tb steps ending with the block of t_count steps at *t0_dev.
// nz > 1 repeats it for nz rings at ring + z ring_zs into sums at + z out_zs
// (the cross-correlation: one ring per second bin).
hipError_t launch_corr(hipStream_t s, const double* X, int64_t ldx, int t_count, int64_t R3, int L,
                       const double* ring, int64_t ring_len, int64_t t0, double* csum, double* ccomp,
                       const int64_t* t0_dev, const int64_t* tbuf_dev = nullptr, int nz = 1, int64_t ring_zs = 0,
                       int64_t out_zs = 0);

// Read-out of the GKMA accumulators: C = (csum + ccomp [+ psum + pcomp]) /
// (S - tau) (zero when S <= tau; psum, pcomp optional: the correlation of
// steps not yet added to the running sums) and its trapezoid running integral
// with step dt, written as corr/integral[tau][r][nu].
hipError_t launch_corr_finish(hipStream_t s, const double* csum, const double* ccomp, const double* psum,
                              const double* pcomp, int64_t R3, int L, int64_t S, double dt, double* corr,
                              double* integral);

// Read-out of the HNEMA accumulators: avg = (sum + comp) / S (zero when S = 0).
hipError_t launch_hnema_finish(hipStream_t s, const double* sum, const double* comp, int64_t n,
                               int64_t S, double* avg);

// ------------------------------------------------------------ spectral heat current
// Direction-major dof columns nu * Np + i (Np = N rounded up to 32, ld = 3 Np):
// ring[(s % ring_len) * 3 + mu][nu Np + i] = W[t][i][mu][nu] and
// vt[t][nu Np + i] = v[t][i][nu], s = s0 + t, t < t_count.
hipError_t launch_shc_ring(hipStream_t s, const float* W, const float* v, int t_count, int64_t N, int64_t Np,
                           float* ring, int64_t ring_len, int64_t ld, int64_t s0, float* vt);
// Partial K^{mu nu}(tau) of one block: sum_{t < t_count} sum_i ring[s0 + t - tau][mu][nu Np + i]
// vt[t][nu Np + i] for tau < n_lags, origins s0 + t - tau >= 0 only, per dof range and 64-step
// tile; each direction segment splits into n_kcs ranges of dk (multiple of 32) dofs; part holds
// [3 n_kcs][ceil(t_count/64)][round_up(n_lags, 128)][3] doubles.
hipError_t launch_shc_products(hipStream_t s, const float* vt, const float* ring, int64_t ring_len, int64_t ld,
                               int64_t N, int64_t Np, int t_count, int64_t s0, int n_lags, int64_t dk, int n_kcs,
                               double* part);
// The block's partials added to the running sums ksum, kcomp [3 nu][n_lags][3 mu] in a fixed
// order (dof ranges, then step tiles), Neumaier.
hipError_t launch_shc_accum(hipStream_t s, const double* part, int t_count, int n_lags, int n_kcs, double* ksum,
                            double* kcomp);
// One system's block in the grouped launches of several systems (the same
// kernels' work, concatenated): the arguments of launch_shc_ring /
// _products / _accum for that system, and where its part of each launch
// starts (ring: blocks of 256 atoms; products: work-groups; accumulation:
// blocks of 256 sums).
struct ShcBlockDesc {
  const float* W;
  const float* v;
  float* ring;
  float* vt;
  double* part;
  double* ksum;
  double* kcomp;
  int64_t N, Np, ring_len, ld, s0, dk;
  int t_count, n_kcs, n_ttiles, n_lags, n_lags_pad;
  int64_t ring_blk0, gram_wg0, acc_blk0;
};
// Sizes of one system's share of the grouped launches.
int64_t shc_gram_wgs(int t_count, int n_lags, int n_kcs);
int64_t shc_accum_blocks(int n_lags);
// The grouped launches over n_sys descriptors (device memory); n_blocks /
// n_wgs: the launch's total (the sum over the systems).
hipError_t launch_shc_ring_group(hipStream_t s, const ShcBlockDesc* d, int n_sys, int64_t n_blocks, int t_count);
hipError_t launch_shc_gram_group(hipStream_t s, const ShcBlockDesc* d, int n_sys, int64_t n_wgs);
hipError_t launch_shc_accum_group(hipStream_t s, const ShcBlockDesc* d, int n_sys, int64_t n_blocks);
// Kd[tau][mu][nu] = (ksum + kcomp)[nu][tau][mu] / (S - tau) (zero where S <= tau) and
// K[tau][mu] = sum over nu in order.
hipError_t launch_shc_finish(hipStream_t s, const double* ksum, const double* kcomp, int n_lags, int64_t S,
                             double* K, double* Kd);
// Kw[w][m] = dt sum_tau c_tau K[tau][m] cos(omega_w tau dt), c = 1, 2, ..., 2, 1 (times the Hann
// window), for the nc components of each lag.
hipError_t launch_shc_spectrum(hipStream_t s, const double* K, int n_lags, int nc, const double* omega, int n_omega,
                               double dt, int window, double* Kw);

}  // namespace mhc
