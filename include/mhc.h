/*
 * mhc.h -- C ABI of libmodalhc: the modal heat-current hot path of
 * velocity-decomposition spectral thermal conductivity (HNEMA and GKMA) on
 * one AMD Instinct MI355X (gfx950).
 *
 * Method: Gabourie, Fan, Ala-Nissila, Pop, "Spectral Decomposition of
 * Thermal Conductivity: Comparing Velocity Decomposition Methods in
 * Homogeneous Molecular Dynamics Simulations", arXiv:2102.03691.
 *
 * Per sampled MD step s the library computes
 *   Xdot_n(s)   = sum_i sqrt(m_i) e_{i,n} . v_i(s)                (Eq. 13)
 *   J_n^mu(s)   = (sum_i m_i^{-1/2} (W_i(s) e_{i,n})^mu) Xdot_n(s) (Eq. 16)
 *   J_b^mu(s)   = sum over the modes n of frequency bin b of J_n^mu(s)
 *   J^mu(s)     = sum_i sum_nu W_i^{mu nu}(s) v_i^nu(s)             (Eq. 10)
 * and accumulates either the HNEMA time average <J_b^mu> (Eq. 19 numerator,
 * Sec. II.B.ii) or the GKMA correlation <J_b^mu(t+tau) J^nu(t)> and its
 * running time integral (Eq. 17, Sec. II.B.i).  Dividing by T V F_e or by
 * k_B T^2 V to obtain kappa is left to the caller (scalar prefactors).
 * Options: every modal output split by the direction of the atoms' motion
 * (MHC_DIRECTIONAL) and bin-bin cross-correlations of the modal currents
 * (MHC_CROSS).  The spectral-heat-current method (Sec. II.C, Eqs. 20-23) has
 * its own object, mhc_shc (end of this header), which needs no eigenvectors.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Units      amu, Angstrom, fs, eV for the physics helpers; the kernels
 *             are unit-agnostic.  Outputs are float64.
 *  Indexing   atom i in [0, N); dof j = 3*i + alpha; mode n in [0, M), M <= 3N.
 *  Virial     W_i^{mu nu} stored row-major W[mu][nu]; the first index is the
 *             heat-current direction: (W v)^mu = sum_nu W^{mu nu} v^nu.
 *  Ownership  The caller owns every pointer it passes.  Load calls copy
 *             before returning.  mhc_push with on_device = 0 copies the host
 *             data before returning; with on_device = 1 the device pointers
 *             must stay valid until the work queued on the context stream has
 *             completed (mhc_synchronize, or any read call).  The library owns
 *             all device memory it allocates and frees it in mhc_destroy.
 *  Errors     Every call returns an mhc_status; no C++ exception crosses the
 *             ABI.  A failed call leaves the context as it was (except for
 *             MHC_ERR_HIP, which is sticky: later calls report it until
 *             mhc_destroy).  mhc_last_error gives a message.
 *  Threads    A context is used by one host thread at a time.
 *  Streams    Work is queued on the context's HIP stream in call order;
 *             calls return before the GPU has finished unless stated.
 */
#ifndef MHC_H
#define MHC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MHC_ABI_VERSION 1

typedef struct mhc_ctx mhc_ctx;

typedef enum {
  MHC_OK = 0,
  MHC_ERR_INVALID_ARG = 1,  /* bad pointer, size, range or value            */
  MHC_ERR_STATE = 2,        /* call not allowed in the context's state      */
  MHC_ERR_OOM = 3,          /* device or host allocation failed             */
  MHC_ERR_HIP = 4,          /* HIP runtime error (sticky)                   */
  MHC_ERR_UNSUPPORTED = 5,  /* valid request the library does not implement */
  MHC_ERR_NONFINITE = 6     /* non-finite input found (check_finite = 1)    */
} mhc_status;

/* Arithmetic of the two contractions of Eqs. 13 and 16.  Sums over steps,
 * bins and lags are float64 in every mode.
 *   FP32    float32 eigenvectors and operands, float32 accumulation
 *   BF16X3  split bfloat16: E = E_hi + E_lo and x = x_hi + x_lo, the product
 *           is hi*hi + hi*lo + lo*hi on bf16 matrix cores with float32
 *           accumulation (the lo*lo term is dropped)
 *   FP8     OCP e4m3 eigenvectors with a float32 scale per mode and e4m3
 *           activations with a float32 scale per (channel, step), one e4m3
 *           product, float32 accumulation (about 4-6e-2 relative error on
 *           random-phase inputs: it misses a 1e-2 accuracy bar; only FP8X3
 *           meets it)
 *   FP8X3   the same scales, each operand split into e4m3 hi + lo, products
 *           hi*hi + hi*lo + lo*hi (about 1e-3 relative error)
 * FP8 and FP8X3 need t_block > 1.                                          */
typedef enum {
  MHC_PREC_FP32 = 0,
  MHC_PREC_BF16X3 = 1,
  MHC_PREC_FP8 = 2,
  MHC_PREC_FP8X3 = 3
} mhc_precision;

/* methods bitmask.  MHC_DIRECTIONAL adds the split of every modal output by
 * the Cartesian direction nu of the atoms' motion (Sec. II, remark after
 * Eq. 10; closing remark of Sec. II.C: e.g. in-plane against out-of-plane
 * motion of a 2D material):
 *   J_n^{mu nu}(s) = Xdot_n(s) sum_i m_i^{-1/2} W_i^{mu nu}(s) e_{i,n}^nu,
 * so that sum_nu J_n^{mu nu} = J_n^mu, and J^{mu nu}(s) = sum_i W_i^{mu nu}(s)
 * v_i^nu(s) for the Eq. 10 total.  T-batched contexts run it as one
 * contraction per block (K ordered by direction, so the three brackets are
 * the contraction over its three thirds while Xdot runs over all of K: the
 * MFMA work of the unsplit contraction; e4m3 activations keep one scale per
 * whole column); t_block = 1 runs one contraction per direction.  It is read with
 * mhc_read_hnema_dir / mhc_read_gkma_dir
 * (mhc_read_hnema and mhc_read_gkma then return the sums over nu), grouped
 * pushes take it, and mhc_read_block_currents does not keep it
 * (UNSUPPORTED). */
enum { MHC_HNEMA = 1, MHC_GKMA = 2, MHC_DIRECTIONAL = 4, MHC_CROSS = 8 };
/* MHC_CROSS (with MHC_GKMA, not with MHC_DIRECTIONAL) adds the bin-bin
 * cross-correlations of the modal currents, <J_b^mu(t+tau) J_b2^nu(t)>
 * (Sec. II.B.i: mode-mode interactions from cross-correlations of modal heat
 * currents; Sec. III.C.i: available from the GKMA currents), read with
 * mhc_read_gkma_cross.  Cost per block about nb times the GKMA correlation
 * update; device memory 2 nb * 3(nb+1) * 3 * L doubles, so it suits a few
 * coarse bins.  Grouped pushes carry it like the GKMA correlation. */

typedef struct {
  int32_t methods;       /* MHC_HNEMA | MHC_GKMA (at least one), | MHC_DIRECTIONAL
                            or | MHC_CROSS (see above)                             */
  int32_t precision;     /* mhc_precision                                           */
  int32_t t_block;       /* steps per contraction: 1 = per-step matrix-vector path,
                            otherwise 32..512 and a multiple of 32 (T-batched GEMM)  */
  int32_t corr_len;      /* GKMA lags L (tau = 0..L-1), 1..65536; ignored for HNEMA  */
  double dt;             /* sample interval for the GKMA integral (> 0)             */
  int32_t check_finite;  /* 1: mhc_push / mhc_group_push reject non-finite v or W
                            (device inputs: a scan kernel, and the push synchronizes) */
  int32_t schedule;      /* T-batched work split: one of MHC_SCHED_* (below)         */
  int32_t reserved[2];   /* must be zero                                            */
} mhc_run_config;

/* Work split of the T-batched contraction (results agree to rounding; each
 * choice is deterministic for a given device):
 *   AUTO     SPLIT where it shortens the launch by 5 % or more, else TILES
 *   TILES    one output tile per work-group
 *   STREAMK  equal contiguous ranges of (tile, k-stage) iterations per CU,
 *            split tiles summed in a fixed order by a second kernel
 *   SPLIT    one work-group per CU: whole tiles round by round, then the
 *            tiles of the last, partial round cut along k so that every CU
 *            takes part; the pieces of a tile are summed in a fixed order
 *            by whichever work-group finishes its piece last              */
enum { MHC_SCHED_AUTO = 0, MHC_SCHED_TILES = 1, MHC_SCHED_STREAMK = 2, MHC_SCHED_SPLIT = 3 };

/* ---------------------------------------------------------------- lifetime */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * queue work on (NULL: the library creates and owns one).  The stream must
 * belong to `device` and outlive the context.
 * Errors: INVALID_ARG (out == NULL), HIP (no such device / runtime failure). */
mhc_status mhc_create(int device, void *hip_stream, mhc_ctx **out);

/* Wait for queued work, free all device memory, destroy the context.
 * NULL is accepted and ignored. */
mhc_status mhc_destroy(mhc_ctx *ctx);

/* Message of the last failed call on ctx (never NULL; owned by ctx, valid
 * until the next call on ctx).  With ctx == NULL: the last mhc_create error. */
const char *mhc_last_error(const mhc_ctx *ctx);

/* Static name of a status code. */
const char *mhc_status_string(mhc_status status);

/* Library ABI version (MHC_ABI_VERSION of the build). */
int mhc_abi_version(void);

/* ------------------------------------------------------------------ loading
 * Order: load_system -> set_bins* -> configure -> load_eigvec_rows (any
 * number of calls, any row order) -> finalize.  Any other order gives STATE. */

/* Atoms and modes of the system (Sec. II.B: 3N modes; Sec. III.C allows a
 * subset of M < 3N modes).
 *   n_atoms   N >= 1
 *   mass_amu  [N] host array of masses > 0 (finite)
 *   n_modes   M, 1 <= M <= 3N
 *   freq_thz  [M] host array of mode frequencies (finite; used for binning)
 * Errors: INVALID_ARG, STATE (already loaded), OOM. */
mhc_status mhc_load_system(mhc_ctx *ctx, int64_t n_atoms, const double *mass_amu,
                           int64_t n_modes, const double *freq_thz);

/* Explicit bin map (Sec. III.A bins by frequency; Sec. III.C.ii bins by mode
 * count -- any grouping works).
 *   n_bins       nb, 1 <= nb <= 1<<20
 *   bin_of_mode  [M] host array, values in [-1, nb); -1 excludes the mode
 * Errors: INVALID_ARG, STATE (no system, or eigenvector rows already loaded). */
mhc_status mhc_set_bins(mhc_ctx *ctx, int32_t n_bins, const int32_t *bin_of_mode);

/* Uniform frequency bins on [f_lo, f_hi]: width d = (f_hi - f_lo)/nb,
 * b = min(floor((f - f_lo)/d + 1e-9), nb - 1) in float64 (ties at an edge
 * go to the upper bin, f == f_hi to the last bin), f outside [f_lo, f_hi]
 * excluded.  Same rule as mhc_bins_uniform.  Errors as mhc_set_bins, plus
 * INVALID_ARG unless f_hi > f_lo (both finite). */
mhc_status mhc_set_bins_uniform(mhc_ctx *ctx, int32_t n_bins, double f_lo, double f_hi);

/* Host-only helper, no context and no GPU: the bin map mhc_set_bins_uniform
 * would build.  out_bins [n_modes] is written.  Errors: INVALID_ARG. */
mhc_status mhc_bins_uniform(int64_t n_modes, const double *freq_thz, int32_t n_bins,
                            double f_lo, double f_hi, int32_t *out_bins);

/* Run configuration (see mhc_run_config).  Allowed after load_system and
 * before the first eigenvector row.  Errors: INVALID_ARG, STATE. */
mhc_status mhc_configure(mhc_ctx *ctx, const mhc_run_config *cfg);

/* Rows mode0 .. mode0+n_rows-1 of E^T (Eqs. 13-16 eigenvectors e_{i,n}):
 *   rows  [n_rows][3N] float64, row n holds e_{i,n}^alpha at column 3*i+alpha;
 *         a host pointer (on_device = 0) or a device pointer on the context's
 *         device (on_device = 1).  Real bases only (e* = e).
 * The rows are converted on the GPU to the configured storage format and
 * placed in bin-sorted order; rows of excluded modes are ignored.  Device
 * memory for the whole basis is allocated on the first call.
 * Errors: INVALID_ARG (range, pointer), STATE, OOM (basis does not fit). */
mhc_status mhc_load_eigvec_rows(mhc_ctx *ctx, int64_t mode0, int64_t n_rows,
                                const double *rows, int on_device);

/* Check that every binned mode's row was loaded, allocate the per-block
 * work buffers and accumulators, and clear the accumulators.
 * Errors: STATE (missing rows / wrong order), OOM. */
mhc_status mhc_finalize(mhc_ctx *ctx);

/* --------------------------------------------------------------- stepping */

/* Push n_steps consecutive samples.
 *   v  [n_steps][N][3]     float32 velocities (A/fs)
 *   W  [n_steps][N][3][3]  float32 per-atom virials (eV), W[mu][nu]
 * Host pointers (on_device = 0) are copied before the call returns; device
 * pointers (on_device = 1) are read asynchronously on the context stream.
 * Steps are processed in blocks of t_block; a trailing partial block is
 * processed as a shorter block, so results do not depend on how a
 * trajectory is split into calls.
 * Errors: INVALID_ARG, STATE (not finalized), NONFINITE (check_finite and an
 * input holds NaN/Inf; nothing is pushed -- for device inputs the check is a
 * scan kernel whose result is read back, so the call synchronizes the
 * stream), OOM, HIP. */
mhc_status mhc_push(mhc_ctx *ctx, int32_t n_steps, const float *v, const float *W, int on_device);

/* Allocation-free push, for callers that cannot allocate memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same inputs, work and results as mhc_push with on_device = 1 (device
 * pointers only; they must stay valid until the queued work completes), and
 * the same work split, so the same bits.  It calls no allocating routine
 * (no hipMalloc / hipFree, no event or stream creation): everything the
 * context needs was allocated by mhc_finalize, and the T-batched
 * contraction's workspace (the partial tiles of the split and stream-K
 * schedules and the split's arrival counters) is a static device array of
 * the library instead of the context's own, 128 MiB + 1 KiB (two 256 KiB
 * partial tiles per compute unit, for at most 256 compute units).  Each
 * device the library is loaded on holds its own copy until the process ends.
 * Every call on one device shares that copy, and each call clears the
 * counters (with a kernel) before its first contraction: calls queued on one
 * stream are ordered and safe, but two calls whose work overlaps on the same
 * device (other streams, other contexts in flight) race and give wrong
 * results.  Kernel timing (mhc_set_timing) is not recorded for these calls,
 * and check_finite is not applied (its device check reads a flag back, which
 * a graph capture does not allow).
 * Errors: as mhc_push; UNSUPPORTED when the device has more than 256 compute
 * units (its workspace would not fit the array); HIP if the array's device
 * address cannot be obtained. */
mhc_status mhc_push_noalloc(mhc_ctx *ctx, int32_t n_steps, const float *v, const float *W);

/* Wait for all queued work of the context. Errors: HIP. */
mhc_status mhc_synchronize(mhc_ctx *ctx);

/* ---------------------------------------------------------------- reading
 * Read calls synchronize the context stream and write host arrays. */

/* HNEMA (Eq. 19 numerator): time averages since the last reset.
 *   avg        [nb][3]  <J_b^mu>        (NULL: skip)
 *   total_avg  [3]      <J^mu> of Eq. 10 (NULL: skip)
 *   n_samples  number of samples S       (NULL: skip)
 * With S = 0 the averages are zero.  Errors: STATE (HNEMA not enabled). */
mhc_status mhc_read_hnema(mhc_ctx *ctx, double *avg, double *total_avg, int64_t *n_samples);

/* GKMA (Eq. 17): for tau = 0 .. L-1
 *   corr      [L][nb][3][3]  C_b^{mu nu}(tau) = <J_b^mu(t+tau) J^nu(t)>, the
 *                            average over the S - tau available origins
 *                            (zero when S <= tau)                  (NULL: skip)
 *   integral  [L][nb][3][3]  trapezoid running integral of corr over tau with
 *                            step dt, integral[0] = 0              (NULL: skip)
 *   hcacf     [L][3][3]      <J^mu(t+tau) J^nu(t)> of the total current (NULL: skip)
 *   n_samples S                                                    (NULL: skip)
 * Errors: STATE (GKMA not enabled). */
mhc_status mhc_read_gkma(mhc_ctx *ctx, double *corr, double *integral, double *hcacf,
                         int64_t *n_samples);

/* Direction-resolved HNEMA (MHC_DIRECTIONAL):
 *   avg        [nb][3][3]  <J_b^{mu nu}>, mu the current direction, nu the
 *                          direction of the atoms' motion          (NULL: skip)
 *   total_avg  [3][3]      <J^{mu nu}> = <sum_i W_i^{mu nu} v_i^nu>  (NULL: skip)
 *   n_samples  S                                                   (NULL: skip)
 * Errors: STATE (HNEMA or the split not enabled). */
mhc_status mhc_read_hnema_dir(mhc_ctx *ctx, double *avg, double *total_avg, int64_t *n_samples);

/* Direction-resolved GKMA (MHC_DIRECTIONAL), tau = 0 .. L-1:
 *   corr      [L][nb][3][3][3]  <J_b^{mu nu}(t+tau) J^{mu2}(t)>, indices
 *                               [tau][b][mu][nu][mu2]; the total current J is
 *                               whole (not split)                   (NULL: skip)
 *   integral  [L][nb][3][3][3]  its trapezoid running integral     (NULL: skip)
 *   n_samples S                                                    (NULL: skip)
 * Errors: STATE (GKMA or the split not enabled). */
mhc_status mhc_read_gkma_dir(mhc_ctx *ctx, double *corr, double *integral, int64_t *n_samples);

/* Bin-bin cross-correlations (MHC_CROSS), tau = 0 .. L-1:
 *   corr      [L][nb][nb][3][3]  <J_b^mu(t+tau) J_b2^nu(t)>, indices
 *                                [tau][b][b2][mu][nu], averaged over the S - tau
 *                                available origins (zero when S <= tau)  (NULL: skip)
 *   integral  [L][nb][nb][3][3]  trapezoid running integral over tau     (NULL: skip)
 *   n_samples S                                                          (NULL: skip)
 * With every mode binned, the sum over b2 equals mhc_read_gkma's corr up to
 * rounding (the binned currents then sum to the Eq. 10 total).
 * Errors: STATE (cross-correlations not enabled). */
mhc_status mhc_read_gkma_cross(mhc_ctx *ctx, double *corr, double *integral, int64_t *n_samples);

/* Binned modal currents of the most recent block, per step:
 *   jb  [t_count][nb][3] float64 J_b^mu(s) for the last t_count pushed steps
 *       of the last block (t_count <= the size of that block)
 * Available when GKMA is enabled (the per-step series exists only then).
 * Errors: STATE, INVALID_ARG (t_count larger than the last block),
 * UNSUPPORTED (MHC_DIRECTIONAL: the per-step series is not kept). */
mhc_status mhc_read_block_currents(mhc_ctx *ctx, int32_t t_count, double *jb);

/* Clear accumulators, sample count and the GKMA history; keep the basis. */
mhc_status mhc_reset(mhc_ctx *ctx);

/* Accumulator state (sums, compensation terms, sample count, GKMA history):
 * mhc_save_state with buf == NULL sets *len to the size needed; otherwise
 * writes *len bytes.  mhc_load_state restores a buffer saved from a context
 * with the same system, bins and configuration.
 * Errors: INVALID_ARG (size / format mismatch), STATE. */
mhc_status mhc_save_state(mhc_ctx *ctx, void *buf, size_t *len);
mhc_status mhc_load_state(mhc_ctx *ctx, const void *buf, size_t len);

/* ------------------------------------------------------------ diagnostics */

/* Enable (1) or disable (0, the default) HIP-event timing of the dominant
 * contraction kernel (one event pair per launch on the context stream).
 * Errors: INVALID_ARG. */
mhc_status mhc_set_timing(mhc_ctx *ctx, int enable);

/* Launch count and summed duration (milliseconds) of the timed contraction
 * launches since the last call; synchronizes the stream and resets the
 * counters.  Errors: HIP. */
mhc_status mhc_kernel_timing(mhc_ctx *ctx, int64_t *launches, double *total_ms);

/* Bytes of device memory held by the context (basis, buffers, accumulators). */
mhc_status mhc_device_bytes(mhc_ctx *ctx, int64_t *bytes);

/* Work split the last T-batched contraction of this context actually used
 * (MHC_SCHED_TILES, _STREAMK or _SPLIT; what AUTO resolved to), or 0 when no
 * batched block has run yet (also for t_block = 1).  Errors: INVALID_ARG. */
mhc_status mhc_last_schedule(mhc_ctx *ctx, int32_t *schedule);

/* ------------------------------------------------------- grouped systems
 * Many independent systems (uneven sizes, HNEMA and GKMA mixed) advanced
 * together: per block of t_block steps the input preparation of every
 * system, ONE persistent contraction launch over the tiles of all systems
 * (work-groups pull tiles largest-first from a queue), and the binning /
 * accumulation of every system.  Results equal pushing each system alone bit
 * for bit when those single pushes use schedule MHC_SCHED_TILES and the
 * group keeps its untuned tile shape (no MHC_GROUP_AUTOTUNE); otherwise they
 * agree to float32 rounding (a single push with AUTO may take the split
 * schedule, which adds k-pieces in float32, and another tile shape changes
 * the float32 per-tile step sums of HNEMA).  The group borrows the contexts:
 * they must stay alive, and must not be pushed on their own while a group
 * push is running. */
typedef struct mhc_group mhc_group;

enum {
  MHC_GROUP_GRAPH = 1,      /* capture the per-block sequence as a HIP graph on the first full
                               block and replay it for every later block                 */
  MHC_GROUP_AUTOTUNE = 2    /* on the first block, time the valid contraction tile shapes
                               (alternating, one launch at a time, best of four rounds) and
                               keep the largest tile unless another is more than 3 % faster
                               (cached per process for the same sizes)                     */
};

/* systems: n finalized contexts with the same device, stream, precision and
 * t_block > 1.  flags: MHC_GROUP_* bits.
 * Errors: INVALID_ARG, STATE (a context not finalized or per-step), OOM, HIP. */
mhc_status mhc_group_create(mhc_ctx *const *systems, int32_t n, int32_t flags, mhc_group **out);
mhc_status mhc_group_destroy(mhc_group *group);
const char *mhc_group_last_error(const mhc_group *group);

/* Push n_steps samples to every system: v[i], W[i] are system i's arrays in
 * the layout of mhc_push (host or device pointers, as on_device says).
 * Full blocks go through the grouped path; a trailing partial block is
 * pushed system by system.  Systems configured with check_finite have their
 * inputs checked first, as for mhc_push.
 * Errors: INVALID_ARG, NONFINITE (nothing pushed to any system), HIP. */
mhc_status mhc_group_push(mhc_group *group, int32_t n_steps, const float *const *v, const float *const *W,
                          int on_device);

/* Tile shape in use (0: 128 slots x 4 t-blocks, 1: 256 x 2, 2: 256 x 1), the
 * autotuner's best measured milliseconds per grouped contraction for each
 * shape ([3], -1 where not timed), and the number of tiles per launch. */
mhc_status mhc_group_info(mhc_group *group, int32_t *tile_shape, double *tuned_ms, int64_t *n_tiles);

/* HIP-event timing of the grouped contraction (graph replay is switched off
 * while timing is on); counters as for mhc_kernel_timing. */
mhc_status mhc_group_set_timing(mhc_group *group, int enable);
mhc_status mhc_group_kernel_timing(mhc_group *group, int64_t *launches, double *total_ms);

/* ---------------------------------------------------- spectral heat current
 * The SHC method (Sec. II.C), which needs no eigenvectors: the steady-state
 * virial-velocity correlation of Eq. 21,
 *   K^mu(tau) = < sum_i sum_nu W_i^{mu nu}(s) v_i^nu(s + tau) >,
 * with the virial at the time origin s and the velocity tau samples later,
 * averaged over the S - tau available origins (tau = 0 .. n_lags-1; K(0) is
 * the time average of the Eq. 10 current), accumulated in float64 on the
 * device (the float32 inputs' products are exact in float64; fixed summation
 * order, Neumaier compensation: bitwise reproducible), and its transform
 * (Eq. 22).  v and W have the layout of mhc_push.  A separate object, so it can
 * run beside an HNEMA/GKMA context on the same inputs (Sec. III.B). */
typedef struct mhc_shc mhc_shc;

/* n_atoms in [1, 2^26]; n_lags in [1, 4096]; t_block (steps per device
 * block) a multiple of 64 in [64, 1024].  hip_stream as for mhc_create.
 * Device memory: about (n_lags + t_block) * 3N * 12 bytes (virial ring) plus
 * t_block * 3N * 20 bytes (velocity rows and host-input staging).
 * Errors: INVALID_ARG, OOM, HIP (mhc_shc_last_error(NULL) tells which). */
mhc_status mhc_shc_create(int device, void *hip_stream, int64_t n_atoms, int32_t n_lags, int32_t t_block,
                          mhc_shc **out);
mhc_status mhc_shc_destroy(mhc_shc *shc);
const char *mhc_shc_last_error(const mhc_shc *shc);

/* Append n_steps samples: v [n_steps][N][3], W [n_steps][N][3][3] float32
 * (host pointers copied before return when on_device = 0; device pointers
 * read by work queued on the stream when on_device = 1, as for mhc_push).
 * Errors: INVALID_ARG, HIP (sticky). */
mhc_status mhc_shc_push(mhc_shc *shc, int32_t n_steps, const float *v, const float *W, int on_device);

/* K [n_lags][3] (float64, Eq. 21 as above; lags with no origin are 0) and the
 * number of samples since the last reset.  Synchronizes.  Errors: INVALID_ARG, HIP. */
mhc_status mhc_shc_read(mhc_shc *shc, double *K, int64_t *n_samples);

/* Eq. 22 on the sampled lags: K is extended evenly, K(-t) = K(t), and the
 * integral over [-(n-1) dt, (n-1) dt] taken by the trapezoid rule,
 *   Kw[w][mu] = dt sum_tau c_tau K[tau][mu] cos(omega[w] tau dt),
 * c_0 = c_{n-1} = 1, c_tau = 2 otherwise, times the Hann window
 * (1 + cos(pi tau / (n-1))) / 2 when window = 1.  omega [n_omega] in radians
 * per unit of dt; n_omega in [1, 2^24].  kappa(omega) = 2 Kw / (V T F_e)
 * (Eq. 23) is left to the caller.  Synchronizes.  Errors: INVALID_ARG, OOM, HIP. */
mhc_status mhc_shc_spectrum(mhc_shc *shc, int32_t n_omega, const double *omega, double dt, int32_t window,
                            double *Kw);

/* Eq. 21 split by the direction nu of the atoms' motion (Sec. II, remark
 * after Eq. 10; closing remark of Sec. II.C), always accumulated at no extra
 * cost (K above is its sum over nu):
 *   K [n_lags][3][3]  K^{mu nu}(tau) = < sum_i W_i^{mu nu}(s) v_i^nu(s + tau) >,
 *                     indices [tau][mu][nu].
 * Synchronizes.  Errors: INVALID_ARG, HIP. */
mhc_status mhc_shc_read_dir(mhc_shc *shc, double *K, int64_t *n_samples);

/* The transform of mhc_shc_spectrum applied to each of the nine split
 * components: Kw [n_omega][3][3], indices [w][mu][nu].  Arguments and errors
 * as for mhc_shc_spectrum. */
mhc_status mhc_shc_spectrum_dir(mhc_shc *shc, int32_t n_omega, const double *omega, double dt, int32_t window,
                                double *Kw);

/* Clear the sums and the sample count (the next push starts a new run). */
mhc_status mhc_shc_reset(mhc_shc *shc);

/* Accumulator state (float64 sums and compensations, the virial history the
 * next blocks correlate against, the sample count), as for mhc_save_state:
 * with buf == NULL *len is set to the size needed (about
 * (n_lags + t_block) * 3N * 12 bytes); mhc_shc_load_state restores a buffer
 * saved from an object with the same n_atoms, n_lags and t_block, after which
 * pushes continue the run exactly.  Errors: INVALID_ARG (size / format
 * mismatch), HIP. */
mhc_status mhc_shc_save_state(mhc_shc *shc, void *buf, size_t *len);
mhc_status mhc_shc_load_state(mhc_shc *shc, const void *buf, size_t len);
mhc_status mhc_shc_synchronize(mhc_shc *shc);

/* HIP-event timing of the virial-velocity product kernel of pushed blocks,
 * as for mhc_set_timing / mhc_kernel_timing.  enable: 0 off, k >= 1 events
 * around every k-th block from this call on (1: each); launches counts the
 * blocks timed.  INVALID_ARG for enable < 0. */
mhc_status mhc_shc_set_timing(mhc_shc *shc, int enable);
mhc_status mhc_shc_kernel_timing(mhc_shc *shc, int64_t *launches, double *total_ms);

/* Grouped SHC: several independent systems (the paper averages its spectra
 * over many independent runs, Sec. III.A) advanced together.  Systems whose
 * own block launch is short share one launch per kernel and block (launch
 * overhead and an underfilled GPU dominate them alone); systems large enough
 * to fill the GPU keep their own launches (fused, they lose cache reuse).
 * systems: n distinct SHC objects (1..4096) with the same device, stream and
 * t_block; their sizes and lag counts may differ.  The group borrows them
 * (destroy it before them); each keeps working on its own (reads, resets,
 * single pushes) between grouped pushes.
 * Errors: INVALID_ARG, OOM, HIP (mhc_shc_group_last_error(NULL) tells which). */
typedef struct mhc_shc_group mhc_shc_group;
mhc_status mhc_shc_group_create(mhc_shc *const *systems, int32_t n, mhc_shc_group **out);
mhc_status mhc_shc_group_destroy(mhc_shc_group *group);
const char *mhc_shc_group_last_error(const mhc_shc_group *group);

/* Push n_steps samples to every system: v[i], W[i] are system i's arrays in
 * the layout of mhc_shc_push, device pointers (on_device = 1: read on the
 * stream, the call returns before the GPU finishes) or host (0: staged,
 * returns when the copies are done).  Each system's sums are the same bits as
 * pushing its samples alone.
 * Errors: INVALID_ARG, HIP (sticky for the group). */
mhc_status mhc_shc_group_push(mhc_shc_group *group, int32_t n_steps, const float *const *v, const float *const *W,
                              int on_device);

/* ------------------------------------------------------ per-atom virial
 * The inputs of the modal current, from positions (Sec. II.A): for a
 * many-body potential written as site energies U = sum_i U_i, with U_i a
 * function of the vectors r_ij = r_j - r_i (Eq. 3) to atom i's neighbours,
 *   F_i        = sum_j (dU_i/dr_ij - dU_j/dr_ji)                 (Eq. 4)
 *   W_i^{mu nu} = sum_{j != i} r_ij^mu (dU_j/dr_ji)^nu            (Eq. 8)
 *   J_i        = W_i v_i                                          (Eq. 10)
 *   F_i^ext    = E_i F_e + F_e . W_i, (F_e . W_i)^nu = sum_mu F_e^mu W_i^{mu nu}
 *                                                                 (Eq. 12)
 * with E_i = U_i + m_i |v_i|^2 / 2 the total energy of atom i.  W_i is not
 * symmetric for a many-body potential; its sum over atoms is the total virial
 * of Eq. 5.  The potential is Tersoff's bond-order form (Phys. Rev. B 38, 9902
 * (1988); the paper's Si potential, Sec. III.A):
 *   U_i     = 1/2 sum_j f_C(r_ij) [A exp(-lambda1 r_ij) - b_ij B exp(-lambda2 r_ij)]
 *   b_ij    = (1 + beta^n zeta_ij^n)^(-1/(2n))
 *   zeta_ij = sum_{k != i,j} f_C(r_ik) g(cos theta_ijk) exp(lambda3^m (r_ij - r_ik)^m)
 *   g(x)    = gamma (1 + c^2/d^2 - c^2 / (d^2 + (x - h)^2))
 *   f_C(r)  = 1 (r < R - D), 1/2 - 1/2 sin(pi/2 (r - R)/D) (|r - R| <= D), 0 beyond.
 * Everything is float64 on the device, in a fixed summation order (bitwise
 * repeatable).  Units: A, eV, amu, fs (kinetic energy converted with
 * 1 amu A^2/fs^2 = 103.6427 eV); F_e in 1/A.  Periodic orthorhombic box,
 * minimum image. */
typedef struct mhc_virial mhc_virial;

typedef struct {
  double A, B;            /* eV                                    */
  double lambda1, lambda2;/* 1/A                                   */
  double lambda3;         /* 1/A (0 switches the exponential off)  */
  int32_t m;              /* exponent of the lambda3 term: 1 or 3  */
  int32_t reserved;       /* must be zero                          */
  double beta, n, c, d, h, gamma;
  double R, D;            /* cutoff centre and half-width, A       */
} mhc_tersoff_params;

/* n_atoms in [1, 2^26]; mass_amu [N] host array (> 0); box [3] host array of
 * the orthorhombic box edges, each larger than 2 (R + D + skin); max_neighbors
 * in [1, 64] (atoms within R + D + skin); skin >= 0 widens the neighbour lists
 * so that they stay valid while atoms move less than skin / 2 (pairs beyond
 * R + D contribute exactly zero).  hip_stream as for mhc_create.
 * Device memory: about N (3 max_neighbors + 2) doubles and N (2 max_neighbors
 * + 3) ints, plus at most 3 (8N + 64) ints of cells.
 * Errors: INVALID_ARG, OOM, HIP (mhc_virial_last_error(NULL)). */
mhc_status mhc_virial_create(int device, void *hip_stream, int64_t n_atoms, const double *mass_amu,
                             const double *box, const mhc_tersoff_params *params, int32_t max_neighbors,
                             double skin, mhc_virial **out);
mhc_status mhc_virial_destroy(mhc_virial *v);
const char *mhc_virial_last_error(const mhc_virial *v);

/* Build the neighbour lists from pos [N][3] (device, A; any periodic image):
 * every j != i with |r_ij| < R + D + skin, in ascending j.  Synchronizes.
 * *max_found (if not NULL) receives the largest neighbour count.
 * Errors: INVALID_ARG (an atom has more than max_neighbors neighbours, or the
 * lists are not symmetric, which non-finite positions cause; the lists are
 * then invalid until the next successful call), HIP. */
mhc_status mhc_virial_neighbors(mhc_virial *v, const double *pos, int32_t *max_found);

/* Copy the lists to the host: counts [N] and lists [N][max_neighbors]
 * (entries past an atom's count are -1); either may be NULL.
 * Errors: STATE (no valid lists), HIP. */
mhc_status mhc_virial_read_neighbors(mhc_virial *v, int32_t *counts, int32_t *lists);

/* One evaluation at positions pos [N][3] (device), with the current lists:
 * outputs are device arrays, each optional (NULL skips it):
 *   U    [N]        site energies U_i (eV)
 *   F    [N][3]     forces (Eq. 4 summed, eV/A)
 *   W    [N][3][3]  per-atom virial W_i^{mu nu} (Eq. 8, eV), float64
 *   W32  [N][3][3]  the same rounded to float32: one step of the W input of
 *                   mhc_push / mhc_shc_push
 *   Fext [N][3]     HNEMD driving force (Eq. 12, eV/A) for fe [3] (host, 1/A;
 *                   NULL: zero); vel [N][3] (device, A/fs) gives the kinetic
 *                   part of E_i (NULL: E_i = U_i).
 * Queued on the stream (returns before the GPU finishes).
 * Errors: INVALID_ARG, STATE (no valid lists), HIP. */
mhc_status mhc_virial_compute(mhc_virial *v, const double *pos, const double *vel, const double *fe, double *U,
                              double *F, double *W, float *W32, double *Fext);
mhc_status mhc_virial_synchronize(mhc_virial *v);

/* NVE molecular dynamics with these forces, fused with the per-step inputs of
 * the modal push (the paper's NVE production runs use a 1 fs time step,
 * Sec. III.A; it names no integrator, and velocity Verlet is used): n_steps
 * steps of dt fs on pos [N][3] (A) and vel [N][3] (A/fs), device float64
 * arrays updated in place (positions wrapped into the box).  One step, with
 * a = F / (m KE) in A/fs^2 (KE = 103.6427 eV per amu A^2/fs^2):
 *   v += dt/2 a(x);  x += dt v;  v += dt/2 a(x).
 * The force at the entry positions is evaluated first.  The neighbour lists
 * are rebuilt before the force of every step whose number (1-based) is a
 * multiple of rebuild (0: never; the lists in use must then stay valid, i.e.
 * no atom moves more than skin / 2 from where they were built); the first
 * call needs lists (mhc_virial_neighbors).  After step s (0-based) the
 * step's velocities and per-atom virials rounded to float32 go to
 * v32 + 3 N s and W32 + 9 N s (device; either may be NULL): the v and W
 * inputs of mhc_push / mhc_shc_push for that step, so n_steps MD steps fill
 * a block of n_steps steps.  The last forces go to F (device [N][3], NULL:
 * skip).  No thermostat and no driving force act (the HNEMD force of Eq. 12
 * is an output of mhc_virial_compute).
 * Lists built with a skin hold many pairs beyond R + D; the force kernels
 * then run on bond lists instead: the listed pairs inside R + D + delta
 * (delta = the smaller of the skin and 0.5 A) at their build, rebuilt on the
 * device whenever an atom has moved more than delta / 2 since (so they hold
 * every pair inside R + D), and at every list rebuild.  Their slots per atom
 * are the largest count found at the last list build plus two; an atom with
 * more makes the call fail with INVALID_ARG at its end, and the call's
 * results are then not valid (rebuild the lists more often).
 * Queued on the stream, except that every rebuild synchronizes, and so does
 * the end of a call that used bond lists (to read their overflow flag).
 * Errors: INVALID_ARG (NULL pos or vel, n_steps or rebuild < 0, dt not finite
 * and positive, a rebuild finding too many neighbours, more bonds on an atom
 * than bond slots), STATE (no valid lists), HIP. */
mhc_status mhc_virial_md(mhc_virial *v, double *pos, double *vel, double dt, int32_t n_steps, int32_t rebuild,
                         float *v32, float *W32, double *F);

/* NVT molecular dynamics with the HNEMD driving force, the protocol of the
 * paper's HNEMA and SHC runs (Sec. III.A: a Nose-Hoover thermostat; the
 * driving force F_ext = E_i F_e + F_e . W_i of Eq. 12 on every atom, E_i with
 * the velocities at the force evaluation).  One thermostat variable xi (1/fs)
 * with mass Q = 3N k_B T tau^2 and its time integral eta; each step is
 *   xi += dt/2 G;  v *= exp(-xi dt/2);  eta += dt/2 xi;
 *   velocity-Verlet step with force F + F_ext;
 *   v *= exp(-xi dt/2);  eta += dt/2 xi;  xi += dt/2 G,
 * G = (2K - 3N k_B T) / Q with the kinetic energy K at that point (summed on
 * the device in a fixed order).  Without a drive, K + U + Q xi^2/2 +
 * 3N k_B T eta is conserved.
 *   fe [3]         driving force parameter (host, 1/A; NULL: none)
 *   temperature    set temperature (K, > 0); tau: thermostat time (fs, > 0)
 *   thermostat [2] (host, in/out) xi and eta: read at entry, written at the
 *                  end ({0, 0} to start a run)
 * Everything else (positions, velocities, lists, bond lists, v32, W32, F,
 * rebuilds) as for mhc_virial_md; the call synchronizes at its end.
 * Errors: those of mhc_virial_md; INVALID_ARG also for a temperature or tau
 * that is not finite and positive, a NULL or non-finite thermostat, a
 * non-finite fe. */
mhc_status mhc_virial_md_nvt(mhc_virial *v, double *pos, double *vel, double dt, int32_t n_steps, int32_t rebuild,
                             const double *fe, double temperature, double tau, double *thermostat, float *v32,
                             float *W32, double *F);

/* HIP-event timing of evaluations (mhc_virial_compute, and every force
 * evaluation of mhc_virial_md / _md_nvt), as mhc_set_timing /
 * mhc_kernel_timing: the summed milliseconds of the per-atom site kernel (bond
 * orders, site energies, partials) and of the gather kernel (forces, W,
 * F_ext) apart, and in launches the number of evaluations timed.  enable: 0
 * off, k >= 1 events around every k-th evaluation from this call on (1: each;
 * at a few thousand atoms an evaluation takes about as long as recording its
 * events, so k > 1 keeps them from slowing what they time).  INVALID_ARG for
 * enable < 0. */
mhc_status mhc_virial_set_timing(mhc_virial *v, int enable);
mhc_status mhc_virial_kernel_timing(mhc_virial *v, int64_t *launches, double *site_ms, double *gather_ms);

#ifdef __cplusplus
}
#endif
#endif /* MHC_H */
