// Host side of libmodalhc: the C ABI declared in include/mhc.h.
//
// Responsibilities: argument validation, the load/configure/finalize state
// machine, the bin-sorted slot order of the modes, device memory, and the
// per-block launch sequence
//   input prep -> contraction (per-step or T-batched) -> bin reduce /
//   float64 accumulate -> (GKMA) correlation update.
// No arithmetic of the method runs here; every step is a HIP kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mhc.h"
#include "mhc_common.h"
#include "mhc_prep_group.h"
#include "mhc_back_group.h"

using namespace mhc;

// Scratch of mhc_push_noalloc: the T-batched contraction's partial tiles (two
// 256-thread x 256-float tiles per compute unit, for up to 256 CUs) followed
// by the split schedule's arrival counters (one int per CU).  One copy per
// device, held until the process ends.  Host code never passes this name to a
// kernel (on the host it is only a stand-in for the symbol); it uses the
// device address from hipGetSymbolAddress instead.
#define MHC_NOALLOC_MAX_CU 256
#define MHC_NOALLOC_WS_FLOATS ((size_t)MHC_NOALLOC_MAX_CU * 2 * 256 * 256)
#define MHC_NOALLOC_SCRATCH_BYTES (MHC_NOALLOC_WS_FLOATS * 4 + (size_t)MHC_NOALLOC_MAX_CU * 4)
static __device__ __align__(256) unsigned char scratch[MHC_NOALLOC_SCRATCH_BYTES];

// Clears the arrival counters in the scratch before a push: a kernel rather
// than a memset, so that the call can be captured in a HIP graph.
__global__ void k_zero_ints(int* __restrict__ p, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = 0;
}

namespace {

thread_local std::string g_create_error;

// Device address of `scratch` on each device, looked up once per device with
// that device current.
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;

hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_addr[device] = p;
  *out = p;
  return hipSuccess;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct mhc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  mhc_status sticky = MHC_OK;

  // system
  bool has_system = false;
  int64_t N = 0, K = 0, M = 0;
  std::vector<double> mass, freq;
  // bins
  bool has_bins = false;
  int32_t nb = 0;
  std::vector<int32_t> bins;
  // configuration
  bool configured = false;
  mhc_run_config cfg{};
  // loading
  bool rows_started = false, finalized = false;
  int64_t K_pad = 0, M_used = 0, M_pad = 0;
  // > 0: the direction split as one contraction, K direction-major with
  // thirds of n3 dofs (T-batched contexts)
  int64_t n3 = 0;
  std::vector<int32_t> slot_of_mode, bin_off;
  std::vector<uint8_t> row_loaded;

  // device memory
  std::vector<DevBuf> allocs;
  void* dE = nullptr;
  double* d_rows = nullptr;   // staging for host eigenvector rows
  int64_t rows_cap = 0;
  int32_t* d_slot = nullptr;
  float* d_sqrtm = nullptr;
  float* d_isqrtm = nullptr;
  int32_t* d_bin_off = nullptr;
  int32_t* d_slot_bin = nullptr;  // GKMA: bin of each slot (-1: padding)
  double* d_seg_part = nullptr;   // GKMA: segment rows of the bin reduction
  int n_seg = 0;
  float* d_rowscale = nullptr;  // e4m3: per-slot scale of E
  float* d_colscale = nullptr;  // e4m3: per-(channel, step) scale of the activations
  float* d_colpart = nullptr;   // e4m3: per-atom-chunk maxima behind d_colscale

  // per-block work buffers
  int chunk = 0;       // steps per processed block
  int t_pad = 0;       // columns of the B operand
  int n_atom_chunks = 0;
  void* dB = nullptr;
  float* dJ = nullptr;
  double* d_jt = nullptr;
  double* d_jtot = nullptr;
  float* d_v = nullptr;
  float* d_W = nullptr;
  // host-pointer pushes: a second staging set and a copy stream, so that the
  // PCIe copy of one block overlaps the kernels of the previous one
  float* d_v2 = nullptr;
  float* d_W2 = nullptr;
  hipStream_t copy_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_copied[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
  double *d_hsum = nullptr, *d_hcomp = nullptr, *d_tsum = nullptr, *d_tcomp = nullptr;
  int n_dir = 1;                 // 3 with the motion-direction split
  int64_t j_region = 0;          // one contraction split: floats of each direction's modal currents in dJ
  double* d_jd = nullptr;        // split Eq. 10 partials of the current pass
  double* d_jdtot = nullptr;     // split Eq. 10 per-step totals
  double *d_tdsum = nullptr, *d_tdcomp = nullptr;   // [dir][mu] time sums of the split totals
  bool cross = false;            // bin-bin cross-correlations
  double* d_bring = nullptr;     // cross: history of the binned currents [nb][ring_len][3]
  double *d_xsum = nullptr, *d_xcomp = nullptr;     // cross sums [nb (second bin)][R3][3][L]
  double* dX = nullptr;
  double* d_ring = nullptr;
  int64_t ring_len = 0;
  int64_t R3 = 0;
  double *d_csum = nullptr, *d_ccomp = nullptr;
  double* d_out = nullptr;
  float* d_ws = nullptr;      // partial tiles of the split and stream-K schedules
  int* d_tile_cnt = nullptr;  // arrival counters of the split schedule (zero between launches)
  int* d_flag = nullptr;      // non-finite flag of the device-input check
  int last_sched = 0;         // schedule the last batched contraction used (MHC_SCHED_*; 0 = none yet)
  int64_t ws_floats = 0;
  int n_cu = 256;
  int64_t n_samples = 0;
  int last_block = 0;
  // GKMA: the binned series of several blocks is kept in X (x_cap columns)
  // and correlated in one update; X holds steps [x_base, x_base + x_fill),
  // the last block starting at column x_last
  int64_t x_cap = 0, x_base = 0, x_fill = 0, x_last = 0;
  double* d_psum = nullptr;      // reads: correlation of the buffered steps (sum + compensation)

  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;   // pairs
  size_t ev_used = 0;
  int64_t bytes = 0;
};

namespace {

mhc_status fail(mhc_ctx* c, mhc_status st, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (st == MHC_ERR_HIP) c->sticky = MHC_ERR_HIP;
  }
  return st;
}

mhc_status hip_fail(mhc_ctx* c, hipError_t e, const char* where) {
  return fail(c, MHC_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, where)                                   \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, (where));   \
  } while (0)

mhc_status enter(mhc_ctx* c) {
  if (!c) return MHC_ERR_INVALID_ARG;
  if (c->sticky != MHC_OK) return c->sticky;
  c->err.clear();
  return MHC_OK;
}

// Allocate device memory owned by the context.  On failure nothing is kept.
mhc_status dev_alloc(mhc_ctx* ctx, size_t bytes, void** out, const char* what) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, MHC_ERR_OOM, std::string("device allocation failed: ") + what + " (" +
                                      std::to_string(bytes) + " bytes)");
  }
  ctx->allocs.push_back({p, bytes});
  ctx->bytes += (int64_t)bytes;
  *out = p;
  return MHC_OK;
}

// Free the allocations made since allocs.size() was `mark` (a load step that
// failed part-way leaves the context as it was).
void rollback_allocs(mhc_ctx* c, size_t mark) {
  while (c->allocs.size() > mark) {
    (void)hipFree(c->allocs.back().p);
    c->bytes -= (int64_t)c->allocs.back().bytes;
    c->allocs.pop_back();
  }
}

void free_all(mhc_ctx* c) {
  for (auto& a : c->allocs) (void)hipFree(a.p);
  c->allocs.clear();
  c->bytes = 0;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

bool all_finite(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

bool all_finite_f(const float* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

bool uniform_bins(int64_t n_modes, const double* f, int32_t nb, double lo, double hi, int32_t* out) {
  if (n_modes < 1 || !f || !out || nb < 1 || nb > (1 << 20)) return false;
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo)) return false;
  const double d = (hi - lo) / nb;
  for (int64_t n = 0; n < n_modes; ++n) {
    const double x = f[n];
    if (!(x >= lo && x <= hi)) {
      out[n] = -1;
      continue;
    }
    double b = std::floor((x - lo) / d + 1e-9);
    out[n] = (int32_t)std::min<double>(b, (double)(nb - 1));
  }
  return true;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

int mhc_abi_version(void) { return MHC_ABI_VERSION; }

const char* mhc_status_string(mhc_status s) {
  // a C caller may pass any int: read the bits as an int (loading an
  // out-of-range value as the enum type is undefined in C++)
  int v = 0;
  std::memcpy(&v, &s, sizeof v < sizeof s ? sizeof v : sizeof s);
  switch (v) {
    case MHC_OK: return "MHC_OK";
    case MHC_ERR_INVALID_ARG: return "MHC_ERR_INVALID_ARG";
    case MHC_ERR_STATE: return "MHC_ERR_STATE";
    case MHC_ERR_OOM: return "MHC_ERR_OOM";
    case MHC_ERR_HIP: return "MHC_ERR_HIP";
    case MHC_ERR_UNSUPPORTED: return "MHC_ERR_UNSUPPORTED";
    case MHC_ERR_NONFINITE: return "MHC_ERR_NONFINITE";
  }
  return "MHC_ERR_UNKNOWN";
}

const char* mhc_last_error(const mhc_ctx* ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->err.c_str();
}

mhc_status mhc_bins_uniform(int64_t n_modes, const double* freq_thz, int32_t n_bins, double f_lo, double f_hi,
                            int32_t* out_bins) {
  return uniform_bins(n_modes, freq_thz, n_bins, f_lo, f_hi, out_bins) ? MHC_OK : MHC_ERR_INVALID_ARG;
}

mhc_status mhc_create(int device, void* hip_stream, mhc_ctx** out) {
  g_create_error.clear();
  if (!out) {
    g_create_error = "out is NULL";
    return MHC_ERR_INVALID_ARG;
  }
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) {
    (void)hipGetLastError();
    g_create_error = std::string("no HIP device: ") + (e != hipSuccess ? hipGetErrorString(e) : "count = 0");
    return MHC_ERR_HIP;
  }
  if (device < 0 || device >= n) {
    g_create_error = "device index out of range";
    return MHC_ERR_INVALID_ARG;
  }
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
    return MHC_ERR_HIP;
  }
  mhc_ctx* c = new (std::nothrow) mhc_ctx();
  if (!c) {
    g_create_error = "host allocation failed";
    return MHC_ERR_OOM;
  }
  c->device = device;
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreate(&c->stream);   // blocking: ordered with the null stream
    if (e != hipSuccess) {
      g_create_error = std::string("hipStreamCreate: ") + hipGetErrorString(e);
      delete c;
      return MHC_ERR_HIP;
    }
    c->own_stream = true;
  }
  *out = c;
  return MHC_OK;
}

mhc_status mhc_destroy(mhc_ctx* ctx) {
  if (!ctx) return MHC_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->copy_stream) (void)hipStreamSynchronize(ctx->copy_stream);
  free_all(ctx);
  for (auto e : ctx->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : {ctx->ev_start, ctx->ev_copied[0], ctx->ev_copied[1], ctx->ev_free[0], ctx->ev_free[1]})
    if (e) (void)hipEventDestroy(e);
  if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return MHC_OK;
}

mhc_status mhc_load_system(mhc_ctx* ctx, int64_t n_atoms, const double* mass_amu, int64_t n_modes,
                           const double* freq_thz) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (ctx->has_system) return fail(ctx, MHC_ERR_STATE, "system already loaded");
  if (n_atoms < 1 || n_atoms > (int64_t(1) << 26)) return fail(ctx, MHC_ERR_INVALID_ARG, "n_atoms out of range");
  if (n_modes < 1 || n_modes > 3 * n_atoms) return fail(ctx, MHC_ERR_INVALID_ARG, "n_modes must be in [1, 3N]");
  if (!mass_amu || !freq_thz) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL mass or frequency array");
  for (int64_t i = 0; i < n_atoms; ++i)
    if (!std::isfinite(mass_amu[i]) || !(mass_amu[i] > 0.0))
      return fail(ctx, MHC_ERR_INVALID_ARG, "masses must be finite and > 0");
  if (!all_finite(freq_thz, n_modes)) return fail(ctx, MHC_ERR_INVALID_ARG, "non-finite frequency");
  ctx->N = n_atoms;
  ctx->K = 3 * n_atoms;
  ctx->M = n_modes;
  ctx->mass.assign(mass_amu, mass_amu + n_atoms);
  ctx->freq.assign(freq_thz, freq_thz + n_modes);
  ctx->has_system = true;
  return MHC_OK;
}

static mhc_status set_bins_impl(mhc_ctx* ctx, int32_t nb, std::vector<int32_t>&& b) {
  ctx->nb = nb;
  ctx->bins = std::move(b);
  ctx->has_bins = true;
  return MHC_OK;
}

mhc_status mhc_set_bins(mhc_ctx* ctx, int32_t n_bins, const int32_t* bin_of_mode) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->has_system || ctx->rows_started) return fail(ctx, MHC_ERR_STATE, "set_bins needs a system and no rows yet");
  if (n_bins < 1 || n_bins > (1 << 20)) return fail(ctx, MHC_ERR_INVALID_ARG, "n_bins out of range");
  if (!bin_of_mode) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL bin map");
  for (int64_t n = 0; n < ctx->M; ++n)
    if (bin_of_mode[n] < -1 || bin_of_mode[n] >= n_bins) return fail(ctx, MHC_ERR_INVALID_ARG, "bin id out of range");
  return set_bins_impl(ctx, n_bins, std::vector<int32_t>(bin_of_mode, bin_of_mode + ctx->M));
}

mhc_status mhc_set_bins_uniform(mhc_ctx* ctx, int32_t n_bins, double f_lo, double f_hi) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->has_system || ctx->rows_started) return fail(ctx, MHC_ERR_STATE, "set_bins needs a system and no rows yet");
  std::vector<int32_t> b(ctx->M);
  if (!uniform_bins(ctx->M, ctx->freq.data(), n_bins, f_lo, f_hi, b.data()))
    return fail(ctx, MHC_ERR_INVALID_ARG, "bad bin count or range");
  return set_bins_impl(ctx, n_bins, std::move(b));
}

mhc_status mhc_configure(mhc_ctx* ctx, const mhc_run_config* cfg) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->has_system || ctx->rows_started) return fail(ctx, MHC_ERR_STATE, "configure needs a system and no rows yet");
  if (!cfg) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL config");
  if (cfg->methods < 1 || cfg->methods > 15 || !(cfg->methods & (MHC_HNEMA | MHC_GKMA)))
    return fail(ctx, MHC_ERR_INVALID_ARG, "methods must be HNEMA, GKMA or both, optionally with DIRECTIONAL or CROSS");
  if ((cfg->methods & MHC_CROSS) && !(cfg->methods & MHC_GKMA))
    return fail(ctx, MHC_ERR_INVALID_ARG, "CROSS needs GKMA");
  if ((cfg->methods & MHC_CROSS) && (cfg->methods & MHC_DIRECTIONAL))
    return fail(ctx, MHC_ERR_UNSUPPORTED, "CROSS together with DIRECTIONAL is not implemented");
  if (cfg->precision < MHC_PREC_FP32 || cfg->precision > MHC_PREC_FP8X3)
    return fail(ctx, MHC_ERR_INVALID_ARG, "unknown precision");
  if (cfg->t_block != 1 && (cfg->t_block < 32 || cfg->t_block > 512 || cfg->t_block % 32))
    return fail(ctx, MHC_ERR_INVALID_ARG, "t_block must be 1 or a multiple of 32 in [32, 512]");
  if (cfg->t_block == 1 && cfg->precision != MHC_PREC_FP32)
    return fail(ctx, MHC_ERR_UNSUPPORTED, "the per-step path (t_block = 1) is FP32 only");
  if ((cfg->methods & MHC_GKMA) && (cfg->corr_len < 1 || cfg->corr_len > 65536))
    return fail(ctx, MHC_ERR_INVALID_ARG, "corr_len must be in [1, 65536]");
  if ((cfg->methods & MHC_GKMA) && !(std::isfinite(cfg->dt) && cfg->dt > 0.0))
    return fail(ctx, MHC_ERR_INVALID_ARG, "dt must be finite and > 0");
  if (cfg->check_finite != 0 && cfg->check_finite != 1) return fail(ctx, MHC_ERR_INVALID_ARG, "check_finite is 0 or 1");
  if (cfg->schedule < MHC_SCHED_AUTO || cfg->schedule > MHC_SCHED_SPLIT)
    return fail(ctx, MHC_ERR_INVALID_ARG, "unknown schedule");
  if (cfg->reserved[0] || cfg->reserved[1])
    return fail(ctx, MHC_ERR_INVALID_ARG, "reserved fields must be zero");
  ctx->cfg = *cfg;
  ctx->configured = true;
  return MHC_OK;
}

// Build the bin-sorted slot order and allocate the basis on the first row load.
static mhc_status start_rows_impl(mhc_ctx* ctx);
static mhc_status start_rows(mhc_ctx* ctx) {
  const size_t mark = ctx->allocs.size();
  const mhc_status st = start_rows_impl(ctx);
  if (st) rollback_allocs(ctx, mark);
  return st;
}

static mhc_status start_rows_impl(mhc_ctx* ctx) {
  const int64_t M = ctx->M, nb = ctx->nb;
  std::vector<int64_t> count(nb + 1, 0);
  for (int64_t n = 0; n < M; ++n)
    if (ctx->bins[n] >= 0) count[ctx->bins[n] + 1]++;
  std::vector<int32_t> off(nb + 1, 0);
  for (int64_t b = 0; b < nb; ++b) off[b + 1] = (int32_t)(off[b] + count[b + 1]);
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  std::vector<int32_t> slot(M, -1);
  for (int64_t n = 0; n < M; ++n) {     // stable: modes keep their order inside a bin
    const int32_t b = ctx->bins[n];
    if (b >= 0) slot[n] = fill[b]++;
  }
  const int64_t M_used = off[nb];
  // input prep writes whole 32-atom (96-dof) groups, so cover them; the
  // one-contraction direction split orders K direction-major, each third a
  // whole number of 32-dof stages
  const auto& cf = ctx->cfg;
  const bool dir1 = (cf.methods & MHC_DIRECTIONAL) && cf.t_block > 1;
  const int64_t n3 = dir1 ? round_up(ctx->N, K_ALIGN) : 0;
  const int64_t K_pad = dir1 ? 3 * n3
                             : round_up(3 * round_up(ctx->N, ATOMS_PER_PREP),
                                        ctx->cfg.t_block == 1 ? K_ALIGN_GEMV : K_ALIGN);
  const int64_t M_pad = round_up(std::max<int64_t>(M_used, 1), M_ALIGN);
  // bytes per element: fp32 or bf16 hi + lo 4, e4m3 hi + lo 2, e4m3 1
  const int prec = ctx->cfg.precision;
  const size_t bpe = prec == MHC_PREC_FP8 ? 1 : (prec == MHC_PREC_FP8X3 ? 2 : 4);
  const size_t e_bytes = (size_t)M_pad * (size_t)K_pad * bpe;
  void* dE = nullptr;
  mhc_status st = dev_alloc(ctx, e_bytes, &dE, "eigenvectors");
  if (st) return st;
  HIP_TRY(hipMemsetAsync(dE, 0, e_bytes, ctx->stream), "zero basis");
  if (prec == MHC_PREC_FP8 || prec == MHC_PREC_FP8X3) {
    void* prs = nullptr;
    if ((st = dev_alloc(ctx, (size_t)M_pad * 4, &prs, "row scales"))) return st;
    HIP_TRY(hipMemsetAsync(prs, 0, (size_t)M_pad * 4, ctx->stream), "zero row scales");
    ctx->d_rowscale = reinterpret_cast<float*>(prs);
  }
  // staging for host rows (about 64 MiB) and slot ids
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(M, (int64_t(64) << 20) / (8 * ctx->K)));
  void* drows = nullptr;
  void* dslot = nullptr;
  if ((st = dev_alloc(ctx, (size_t)cap * ctx->K * 8, &drows, "row staging"))) return st;
  if ((st = dev_alloc(ctx, (size_t)std::max<int64_t>(cap, 1 << 16) * 4, &dslot, "row slots"))) return st;
  ctx->dE = dE;
  ctx->d_rows = reinterpret_cast<double*>(drows);
  ctx->rows_cap = cap;
  ctx->d_slot = reinterpret_cast<int32_t*>(dslot);
  ctx->slot_of_mode = std::move(slot);
  ctx->bin_off = std::move(off);
  ctx->M_used = M_used;
  ctx->K_pad = K_pad;
  ctx->n3 = n3;
  ctx->M_pad = M_pad;
  ctx->row_loaded.assign(M, 0);
  ctx->rows_started = true;
  return MHC_OK;
}

mhc_status mhc_load_eigvec_rows(mhc_ctx* ctx, int64_t mode0, int64_t n_rows, const double* rows, int on_device) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->has_system || !ctx->has_bins || !ctx->configured || ctx->finalized)
    return fail(ctx, MHC_ERR_STATE, "eigenvector rows need system, bins and configuration, before finalize");
  if (mode0 < 0 || n_rows < 0 || mode0 + n_rows > ctx->M) return fail(ctx, MHC_ERR_INVALID_ARG, "row range outside [0, M)");
  if (n_rows == 0) return MHC_OK;
  if (!rows) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL rows");
  if (on_device != 0 && on_device != 1) return fail(ctx, MHC_ERR_INVALID_ARG, "on_device is 0 or 1");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  if (!ctx->rows_started) {
    if ((st = start_rows(ctx))) return st;
  }
  const int prec = ctx->cfg.precision;
  const int64_t step = on_device ? std::min<int64_t>(n_rows, 1 << 16) : ctx->rows_cap;
  std::vector<int32_t> slots;
  for (int64_t r0 = 0; r0 < n_rows; r0 += step) {
    const int64_t nr = std::min(step, n_rows - r0);
    slots.resize(nr);
    for (int64_t r = 0; r < nr; ++r) slots[r] = ctx->slot_of_mode[mode0 + r0 + r];
    HIP_TRY(hipMemcpyAsync(ctx->d_slot, slots.data(), nr * 4, hipMemcpyHostToDevice, ctx->stream), "copy slots");
    const double* src = rows + r0 * ctx->K;
    if (!on_device) {
      HIP_TRY(hipMemcpyAsync(ctx->d_rows, src, (size_t)nr * ctx->K * 8, hipMemcpyHostToDevice, ctx->stream),
              "copy rows");
      src = ctx->d_rows;
    }
    if (prec == MHC_PREC_FP8 || prec == MHC_PREC_FP8X3)
      HIP_TRY(launch_basis_store_fp8(ctx->stream, prec == MHC_PREC_FP8X3, src, nr, ctx->K, ctx->d_slot, ctx->dE,
                                     ctx->K_pad, ctx->d_rowscale, ctx->n3),
              "basis store");
    else
      HIP_TRY(launch_basis_store(ctx->stream, prec, src, nr, ctx->K, ctx->d_slot, ctx->dE, ctx->K_pad,
                                 ctx->cfg.t_block == 1 ? 1 : 0, ctx->n3),
              "basis store");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "basis store sync");
  }
  for (int64_t r = 0; r < n_rows; ++r) ctx->row_loaded[mode0 + r] = 1;
  return MHC_OK;
}

static int t_pad_of(const mhc_run_config& c) { return c.t_block == 1 ? 256 : c.t_block; }

// HNEMA accumulator doubles: bin sums and compensations [dir][nb][3], the
// Eq. 10 total and its compensation [3], and with the split the split totals
// and compensations [dir][3].
static size_t hn_doubles(int64_t nb, int nd) { return (size_t)2 * nd * nb * 3 + 6 + (nd > 1 ? 18 : 0); }

// GKMA correlation doubles (sums and compensations of every direction pass).
static size_t gk_doubles(const mhc_ctx* c) { return (size_t)2 * c->n_dir * c->cfg.corr_len * c->R3 * 3; }

// Cross-correlation doubles (sums and compensations) and bin-history doubles.
static size_t cross_doubles(const mhc_ctx* c) {
  return c->cross ? (size_t)2 * c->nb * c->R3 * 3 * c->cfg.corr_len : 0;
}
static size_t bring_doubles(const mhc_ctx* c) { return c->cross ? (size_t)c->nb * c->ring_len * 3 : 0; }

static mhc_status finalize_impl(mhc_ctx* ctx);

mhc_status mhc_finalize(mhc_ctx* ctx) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->rows_started || ctx->finalized) return fail(ctx, MHC_ERR_STATE, "finalize needs loaded rows, once");
  const size_t mark = ctx->allocs.size();
  st = finalize_impl(ctx);
  if (st) {                             // a failed finalize keeps nothing (it may be retried)
    rollback_allocs(ctx, mark);
    ctx->finalized = false;
  }
  return st;
}

static mhc_status finalize_impl(mhc_ctx* ctx) {
  mhc_status st;
  for (int64_t n = 0; n < ctx->M; ++n)
    if (ctx->slot_of_mode[n] >= 0 && !ctx->row_loaded[n])
      return fail(ctx, MHC_ERR_STATE, "eigenvector row " + std::to_string(n) + " was not loaded");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  const auto& c = ctx->cfg;
  const bool gk = c.methods & MHC_GKMA;
  const bool hn = c.methods & MHC_HNEMA;
  const int chunk = t_pad_of(c);
  const int t_pad = chunk;
  const int64_t N = ctx->N, K_pad = ctx->K_pad, M_pad = ctx->M_pad, nb = ctx->nb;
  const int n_ac = (int)((N + ATOMS_PER_PREP - 1) / ATOMS_PER_PREP);
  const int64_t n_parts = (c.t_block == 1) ? chunk : std::max(1, t_pad / 32);
  size_t j_bytes = (size_t)n_parts * M_pad * 3 * 4;
  if (gk) j_bytes = std::max(j_bytes, (size_t)3 * M_pad * t_pad * 4);
  ctx->j_region = ctx->n3 ? (int64_t)(j_bytes / 4) : 0;
  if (ctx->n3) j_bytes *= 3;          // one region per direction
  const int64_t R3 = 3 * (nb + 1);
  const int L = gk ? c.corr_len : 0;
  void *pB, *pJ, *pjt, *pv, *pW, *psm, *pism, *poff, *pacc, *pout;
  if ((st = dev_alloc(ctx, (size_t)16 * t_pad * K_pad, &pB, "B operand"))) return st;
  if ((st = dev_alloc(ctx, j_bytes, &pJ, "modal currents"))) return st;
  if ((st = dev_alloc(ctx, (size_t)t_pad * n_ac * 3 * 8, &pjt, "total-current partials"))) return st;
  void* pjtot = nullptr;
  if ((st = dev_alloc(ctx, (size_t)t_pad * 3 * 8, &pjtot, "total current"))) return st;
  if ((st = dev_alloc(ctx, (size_t)chunk * N * 3 * 4, &pv, "velocity staging"))) return st;
  if ((st = dev_alloc(ctx, (size_t)chunk * N * 9 * 4, &pW, "virial staging"))) return st;
  if ((st = dev_alloc(ctx, (size_t)N * 4, &psm, "sqrt m"))) return st;
  if ((st = dev_alloc(ctx, (size_t)N * 4, &pism, "1/sqrt m"))) return st;
  if ((st = dev_alloc(ctx, (size_t)(nb + 1) * 4, &poff, "bin offsets"))) return st;
  if (c.precision == MHC_PREC_FP8 || c.precision == MHC_PREC_FP8X3) {
    void* pcs = nullptr;
    if ((st = dev_alloc(ctx, (size_t)4 * t_pad * 4, &pcs, "column scales"))) return st;
    ctx->d_colscale = reinterpret_cast<float*>(pcs);
    const int64_t n_cc = (N + COLSCALE_ATOMS - 1) / COLSCALE_ATOMS;
    void* pcp = nullptr;
    if ((st = dev_alloc(ctx, (size_t)n_cc * 4 * t_pad * 4, &pcp, "column maxima"))) return st;
    ctx->d_colpart = reinterpret_cast<float*>(pcp);
  }
  const int nd = (c.methods & MHC_DIRECTIONAL) ? 3 : 1;
  ctx->n_dir = nd;
  const size_t acc_doubles = hn_doubles(nb, nd);
  if ((st = dev_alloc(ctx, acc_doubles * 8, &pacc, "HNEMA sums"))) return st;
  size_t out_doubles = (size_t)nd * nb * 3 + 12;
  if (nd > 1) {
    void *pjd, *pjdt;
    const size_t jd_bytes = (size_t)(ctx->n3 ? 3 : 1) * t_pad * n_ac * 3 * 8;   // [nu][t][chunk][mu]
    if ((st = dev_alloc(ctx, jd_bytes, &pjd, "split total partials"))) return st;
    if ((st = dev_alloc(ctx, (size_t)t_pad * 3 * 8, &pjdt, "split total current"))) return st;
    HIP_TRY(hipMemsetAsync(pjd, 0, jd_bytes, ctx->stream), "zero split partials");
    ctx->d_jd = reinterpret_cast<double*>(pjd);
    ctx->d_jdtot = reinterpret_cast<double*>(pjdt);
  }
  if (gk) {
    void *pX, *pring, *pc;
    // Blocks of binned currents folded into one correlation update, so that
    // the float64 read-modify-write of the correlation sums happens once per
    // fold; the matrix-core accumulators sum the fold's steps uncompensated
    // (at most 1024 steps).  One block per update with the direction split
    // (its passes share the series buffer) and with cross-correlations (their
    // bin history would grow with the fold).
    const int fold = (nd == 1 && !(c.methods & MHC_CROSS)) ? std::max(1, std::min(16, 1024 / t_pad)) : 1;
    const int64_t x_cap = (int64_t)fold * t_pad;
    const int64_t ring_len = (int64_t)L - 1 + x_cap;
    if ((st = dev_alloc(ctx, (size_t)R3 * x_cap * 8, &pX, "binned series"))) return st;
    if ((st = dev_alloc(ctx, (size_t)ring_len * 3 * 8, &pring, "history ring"))) return st;
    if ((st = dev_alloc(ctx, (size_t)2 * nd * L * R3 * 3 * 8, &pc, "correlation sums"))) return st;
    ctx->dX = reinterpret_cast<double*>(pX);
    ctx->d_ring = reinterpret_cast<double*>(pring);
    ctx->ring_len = ring_len;
    ctx->x_cap = x_cap;
    if (fold > 1) {   // reads add the buffered steps' correlation from scratch sums
      void* pp = nullptr;
      if ((st = dev_alloc(ctx, (size_t)2 * L * R3 * 3 * 8, &pp, "pending correlation sums"))) return st;
      ctx->d_psum = reinterpret_cast<double*>(pp);
    }
    ctx->d_csum = reinterpret_cast<double*>(pc);
    ctx->d_ccomp = ctx->d_csum + (size_t)nd * L * R3 * 3;
    out_doubles = std::max(out_doubles, (size_t)2 * L * R3 * 3);
    HIP_TRY(hipMemsetAsync(pX, 0, (size_t)R3 * x_cap * 8, ctx->stream), "zero series");
    HIP_TRY(hipMemsetAsync(pring, 0, (size_t)ring_len * 3 * 8, ctx->stream), "zero ring");
    // segment pass of the bin reduction: bin of every slot, float64 segment rows
    const int64_t n_seg = (M_pad + REDUCE_SEG - 1) / REDUCE_SEG;
    std::vector<int32_t> sbin(M_pad, -1);
    for (int64_t b = 0; b < nb; ++b)
      for (int64_t q = ctx->bin_off[b]; q < ctx->bin_off[b + 1]; ++q) sbin[q] = (int32_t)b;
    void *psb, *psp;
    if ((st = dev_alloc(ctx, (size_t)M_pad * 4, &psb, "slot bins"))) return st;
    if ((st = dev_alloc(ctx, (size_t)3 * (n_seg + nb) * t_pad * 8, &psp, "segment sums"))) return st;
    HIP_TRY(hipMemcpyAsync(psb, sbin.data(), (size_t)M_pad * 4, hipMemcpyHostToDevice, ctx->stream), "copy slot bins");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "slot bins sync");
    ctx->d_slot_bin = reinterpret_cast<int32_t*>(psb);
    ctx->d_seg_part = reinterpret_cast<double*>(psp);
    ctx->n_seg = (int)n_seg;
    if (c.methods & MHC_CROSS) {
      if (nb > 65535) return fail(ctx, MHC_ERR_INVALID_ARG, "CROSS allows at most 65535 bins");
      void *pbr, *px;
      const size_t br = (size_t)nb * ring_len * 3 * 8;
      const size_t xs = (size_t)2 * nb * R3 * 3 * L * 8;
      if ((st = dev_alloc(ctx, br, &pbr, "bin history ring"))) return st;
      if ((st = dev_alloc(ctx, xs, &px, "cross-correlation sums"))) return st;
      HIP_TRY(hipMemsetAsync(pbr, 0, br, ctx->stream), "zero bin ring");
      ctx->cross = true;
      ctx->d_bring = reinterpret_cast<double*>(pbr);
      ctx->d_xsum = reinterpret_cast<double*>(px);
      ctx->d_xcomp = ctx->d_xsum + (size_t)nb * R3 * 3 * L;
    }
  }
  if ((st = dev_alloc(ctx, out_doubles * 8, &pout, "read-out"))) return st;
  void* pflag = nullptr;
  if ((st = dev_alloc(ctx, 16, &pflag, "non-finite flag"))) return st;
  ctx->d_flag = reinterpret_cast<int*>(pflag);
  if (c.t_block > 1) {
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, ctx->device), "device properties");
    ctx->n_cu = std::max(1, prop.multiProcessorCount);
    // per CU: two partial tiles of 256 threads x 256 accumulator floats
    ctx->ws_floats = (int64_t)ctx->n_cu * 2 * 256 * 256;
    void* pws = nullptr;
    if ((st = dev_alloc(ctx, (size_t)ctx->ws_floats * 4, &pws, "contraction workspace"))) return st;
    ctx->d_ws = reinterpret_cast<float*>(pws);
    void* pcnt = nullptr;
    if ((st = dev_alloc(ctx, (size_t)ctx->n_cu * 4, &pcnt, "split counters"))) return st;
    HIP_TRY(hipMemsetAsync(pcnt, 0, (size_t)ctx->n_cu * 4, ctx->stream), "zero split counters");
    ctx->d_tile_cnt = reinterpret_cast<int*>(pcnt);
  }
  // masses
  std::vector<float> sm(N), ism(N);
  for (int64_t i = 0; i < N; ++i) {
    const double r = std::sqrt(ctx->mass[i]);
    sm[i] = (float)r;
    ism[i] = (float)(1.0 / r);
  }
  HIP_TRY(hipMemcpyAsync(psm, sm.data(), N * 4, hipMemcpyHostToDevice, ctx->stream), "copy sqrt m");
  HIP_TRY(hipMemcpyAsync(pism, ism.data(), N * 4, hipMemcpyHostToDevice, ctx->stream), "copy 1/sqrt m");
  HIP_TRY(hipMemcpyAsync(poff, ctx->bin_off.data(), (nb + 1) * 4, hipMemcpyHostToDevice, ctx->stream), "copy bins");
  HIP_TRY(hipMemsetAsync(pB, 0, (size_t)16 * t_pad * K_pad, ctx->stream), "zero B");
  HIP_TRY(hipMemsetAsync(pJ, 0, j_bytes, ctx->stream), "zero J");
  HIP_TRY(hipMemsetAsync(pjt, 0, (size_t)t_pad * n_ac * 3 * 8, ctx->stream), "zero partials");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "finalize sync");

  ctx->chunk = chunk;
  ctx->t_pad = t_pad;
  ctx->n_atom_chunks = n_ac;
  ctx->dB = pB;
  ctx->dJ = reinterpret_cast<float*>(pJ);
  ctx->d_jt = reinterpret_cast<double*>(pjt);
  ctx->d_jtot = reinterpret_cast<double*>(pjtot);
  ctx->d_v = reinterpret_cast<float*>(pv);
  ctx->d_W = reinterpret_cast<float*>(pW);
  ctx->d_sqrtm = reinterpret_cast<float*>(psm);
  ctx->d_isqrtm = reinterpret_cast<float*>(pism);
  ctx->d_bin_off = reinterpret_cast<int32_t*>(poff);
  double* acc = reinterpret_cast<double*>(pacc);
  ctx->d_hsum = hn ? acc : nullptr;
  ctx->d_hcomp = hn ? acc + nd * nb * 3 : nullptr;
  ctx->d_tsum = hn ? acc + 2 * nd * nb * 3 : nullptr;
  ctx->d_tcomp = hn ? acc + 2 * nd * nb * 3 + 3 : nullptr;
  ctx->d_tdsum = (hn && nd > 1) ? acc + 2 * nd * nb * 3 + 6 : nullptr;
  ctx->d_tdcomp = (hn && nd > 1) ? acc + 2 * nd * nb * 3 + 15 : nullptr;
  ctx->R3 = R3;
  ctx->d_out = reinterpret_cast<double*>(pout);
  ctx->finalized = true;
  return mhc_reset(ctx);
}

mhc_status mhc_reset(mhc_ctx* ctx) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized) return fail(ctx, MHC_ERR_STATE, "reset needs a finalized context");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  const int64_t nb = ctx->nb;
  if (ctx->d_hsum) HIP_TRY(hipMemsetAsync(ctx->d_hsum, 0, hn_doubles(nb, ctx->n_dir) * 8, ctx->stream), "zero sums");
  if (ctx->d_csum) HIP_TRY(hipMemsetAsync(ctx->d_csum, 0, gk_doubles(ctx) * 8, ctx->stream), "zero corr");
  if (ctx->d_ring) HIP_TRY(hipMemsetAsync(ctx->d_ring, 0, (size_t)ctx->ring_len * 3 * 8, ctx->stream), "zero ring");
  if (ctx->cross) {
    HIP_TRY(hipMemsetAsync(ctx->d_xsum, 0, cross_doubles(ctx) * 8, ctx->stream), "zero cross");
    HIP_TRY(hipMemsetAsync(ctx->d_bring, 0, bring_doubles(ctx) * 8, ctx->stream), "zero bin ring");
  }
  ctx->n_samples = 0;
  ctx->last_block = 0;
  ctx->x_base = ctx->x_fill = ctx->x_last = 0;
  return MHC_OK;
}

// Front of a block: activation scales (e4m3), B operand, per-chunk Eq. 10 partials.
// With tab != NULL the input pointers are read from device memory (tab[0] =
// v, tab[1] = W) when the kernels run.
static mhc_status block_front(mhc_ctx* ctx, const float* v, const float* W, int t_count,
                              const float* const* tab = nullptr, int dir = -1) {
  const auto& c = ctx->cfg;
  if (ctx->n3 && dir < 0) dir = DIR_ALL;   // one-contraction split: every direction in one operand
  if (ctx->d_colscale)
    HIP_TRY(launch_col_scale(ctx->stream, v, W, ctx->d_sqrtm, ctx->d_isqrtm, ctx->N, t_count, ctx->t_pad,
                             ctx->d_colpart, tab, dir == DIR_ALL ? -1 : dir),   // whole columns serve every third
            "column scales");
  HIP_TRY(launch_input_prep(ctx->stream, c.precision, c.t_block == 1 ? 1 : 0, v, W, ctx->d_sqrtm, ctx->d_isqrtm,
                            ctx->N, t_count, ctx->t_pad, ctx->dB, ctx->K_pad, ctx->d_jt, ctx->d_colscale,
                            ctx->d_colpart, tab, dir, ctx->d_jd),
          "input prep");
  return MHC_OK;
}

// Correlation update of the count buffered GKMA steps starting at global step
// t0 (X columns 0 .. count - 1) into the sums (sum, comp), by default the
// context's own.
static mhc_status corr_update(mhc_ctx* ctx, int64_t t0, int64_t count, double* sum = nullptr,
                              double* comp = nullptr) {
  const int L = ctx->cfg.corr_len;
  HIP_TRY(launch_corr(ctx->stream, ctx->dX, ctx->x_cap, (int)count, ctx->R3, L, ctx->d_ring, ctx->ring_len, t0,
                      sum ? sum : ctx->d_csum, comp ? comp : ctx->d_ccomp, nullptr),
          "correlation");
  if (sum) return MHC_OK;
  if (ctx->cross)   // every binned row against the history of every bin b2 (grid z = b2)
    HIP_TRY(launch_corr(ctx->stream, ctx->dX, ctx->x_cap, (int)count, ctx->R3, L, ctx->d_bring, ctx->ring_len, t0,
                        ctx->d_xsum, ctx->d_xcomp, nullptr, nullptr, (int)ctx->nb, ctx->ring_len * 3,
                        ctx->R3 * 3 * L),
            "cross-correlation");
  return MHC_OK;
}


// Where a block's binned series goes in X, and whether the correlation update
// runs after it (the number of buffered steps to correlate, 0 for none); the
// host keeps this account for the single pushes and for the group's table.
static void fold_step(mhc_ctx* ctx, int t_count, int64_t* xoff, int64_t* tbuf) {
  *xoff = ctx->x_fill;
  ctx->x_last = ctx->x_fill;
  ctx->x_fill += t_count;
  *tbuf = 0;
  if (ctx->x_fill + ctx->t_pad > ctx->x_cap) {   // no room for another full block
    *tbuf = ctx->x_fill;
    ctx->x_base += ctx->x_fill;
    ctx->x_fill = 0;
  }
}

// Back of a block: per-step totals, bins + float64 accumulation, GKMA update.
// With t0_dev the block's first step index is read from device memory when
// the kernels run (the group's input table), so a captured graph can be
// replayed block after block; so are the block's column in X (xoff_dev) and
// the correlation update's step count (tbuf_dev).
// With the motion-direction split, pass dir in {0, 1, 2} accumulates into its
// own slice of the bin sums and correlation sums; the whole Eq. 10 total is
// summed in pass 0 only (every pass rewrites the same GKMA history entries).
static mhc_status block_back(mhc_ctx* ctx, int t_count, int n_parts, const int64_t* t0_dev, int dir = -1,
                             const int64_t* xoff_dev = nullptr, const int64_t* tbuf_dev = nullptr) {
  const auto& c = ctx->cfg;
  const bool gk = c.methods & MHC_GKMA;
  const int64_t ld = ctx->t_pad;
  const int d = dir < 0 ? 0 : dir;
  // the one-contraction split leaves every direction's currents and split
  // partials in their own regions; the pass-per-direction form reuses one
  const bool one = ctx->n3 > 0 && dir >= 0;
  HIP_TRY(launch_total(ctx->stream, ctx->d_jt, ctx->n_atom_chunks, t_count, ctx->d_jtot), "total current");
  if (dir >= 0 && ctx->d_tdsum)
    HIP_TRY(launch_total(ctx->stream, ctx->d_jd + (one ? (int64_t)d * ctx->t_pad * ctx->n_atom_chunks * 3 : 0),
                         ctx->n_atom_chunks, t_count, ctx->d_jdtot),
            "split total current");
  ReduceArgs a{};
  a.in = ctx->dJ + (one ? d * ctx->j_region : 0);
  a.layout_g = gk ? 1 : 0;
  a.n_parts = n_parts;
  a.M_pad = ctx->M_pad;
  a.ld = ld;
  a.t_count = t_count;
  a.bin_off = ctx->d_bin_off;
  a.slot_bin = ctx->d_slot_bin;
  a.seg_part = ctx->d_seg_part;
  a.n_seg = ctx->n_seg;
  a.nb = ctx->nb;
  a.jtot = ctx->d_jtot;
  a.hsum = ctx->d_hsum ? ctx->d_hsum + (int64_t)d * ctx->nb * 3 : nullptr;
  a.hcomp = ctx->d_hcomp ? ctx->d_hcomp + (int64_t)d * ctx->nb * 3 : nullptr;
  a.tsum = d == 0 ? ctx->d_tsum : nullptr;
  a.tcomp = d == 0 ? ctx->d_tcomp : nullptr;
  if (dir >= 0 && ctx->d_tdsum) {
    a.jdtot = ctx->d_jdtot;
    a.tdsum = ctx->d_tdsum + 3 * dir;
    a.tdcomp = ctx->d_tdcomp + 3 * dir;
  }
  a.X = gk ? ctx->dX : nullptr;
  a.bring = ctx->d_bring;
  a.ring = ctx->d_ring;
  a.ring_len = ctx->ring_len;
  a.t0 = ctx->n_samples;
  a.t0_dev = t0_dev;
  a.ldx = gk ? ctx->x_cap : ld;
  int64_t xoff = 0, tbuf = 0;
  if (gk && dir < 0 && !t0_dev) fold_step(ctx, t_count, &xoff, &tbuf);
  a.xoff = xoff;
  a.xoff_dev = t0_dev ? xoff_dev : nullptr;
  HIP_TRY(launch_reduce(ctx->stream, a), "bin reduce");
  if (!gk) return MHC_OK;
  if (dir >= 0) {
    // direction passes: one update per pass over this block (X holds one block)
    const size_t off = (size_t)d * c.corr_len * ctx->R3 * 3;
    HIP_TRY(launch_corr(ctx->stream, ctx->dX, ctx->x_cap, t_count, ctx->R3, c.corr_len, ctx->d_ring, ctx->ring_len,
                        ctx->n_samples, ctx->d_csum + off, ctx->d_ccomp + off, t0_dev),
            "correlation");
  } else if (t0_dev) {
    // grouped: the block table says how many buffered steps to correlate now
    HIP_TRY(launch_corr(ctx->stream, ctx->dX, ctx->x_cap, t_count, ctx->R3, c.corr_len, ctx->d_ring, ctx->ring_len,
                        0, ctx->d_csum, ctx->d_ccomp, t0_dev, tbuf_dev),
            "correlation");
    if (ctx->cross)
      HIP_TRY(launch_corr(ctx->stream, ctx->dX, ctx->x_cap, t_count, ctx->R3, c.corr_len, ctx->d_bring,
                          ctx->ring_len, 0, ctx->d_xsum, ctx->d_xcomp, t0_dev, tbuf_dev, (int)ctx->nb,
                          ctx->ring_len * 3, ctx->R3 * 3 * c.corr_len),
              "cross-correlation");
  } else if (tbuf > 0) {
    // the tbuf buffered steps ending with this block (fold_step has moved
    // x_base past them)
    return corr_update(ctx, ctx->x_base - tbuf, tbuf);
  }
  return MHC_OK;
}

static mhc_status timing_begin(mhc_ctx* ctx, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (!ctx->timing) return MHC_OK;
  if (ctx->ev_used + 2 > ctx->ev.size()) {
    for (int q = 0; q < 2; ++q) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e), "event create");
      ctx->ev.push_back(e);
    }
  }
  *e0 = ctx->ev[ctx->ev_used];
  *e1 = ctx->ev[ctx->ev_used + 1];
  ctx->ev_used += 2;
  HIP_TRY(hipEventRecord(*e0, ctx->stream), "event record");
  return MHC_OK;
}

// Workspace of the T-batched contraction: partial tiles of the split and
// stream-K schedules and the split's arrival counters (zero between launches).
struct Workspace {
  float* ws = nullptr;
  int64_t ws_floats = 0;
  int* cnt = nullptr;
};

static Workspace ctx_workspace(const mhc_ctx* ctx) { return {ctx->d_ws, ctx->ws_floats, ctx->d_tile_cnt}; }

// One block of t_count steps: front, contraction, back; with the
// motion-direction split, one such pass per direction (the contraction is
// the same kernel on the masked operand).  timed = false skips the event
// timing (which creates events on first use).
static mhc_status run_block(mhc_ctx* ctx, const float* v, const float* W, int t_count, const Workspace& wk,
                            bool timed = true) {
  const auto& c = ctx->cfg;
  const bool gk = c.methods & MHC_GKMA;
  mhc_status st;
  if (ctx->n3) {
    // direction split in one contraction: one operand with every direction,
    // one launch, then the back end once per direction on its own region
    if ((st = block_front(ctx, v, W, t_count))) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed && (st = timing_begin(ctx, &e0, &e1))) return st;
    int n_parts = 0;
    HIP_TRY(launch_gemm_dir(ctx->stream, c.precision, ctx->dE, ctx->dB, ctx->M_pad, ctx->n3, ctx->t_pad / 32, ctx->dJ,
                            ctx->j_region, gk ? 1 : 0, &n_parts, wk.ws, wk.ws_floats, ctx->n_cu, ctx->d_rowscale,
                            ctx->d_colscale),
            "direction-split contraction");
    ctx->last_sched = MHC_SCHED_TILES;
    if (e1) HIP_TRY(hipEventRecord(e1, ctx->stream), "event record");
    for (int d = 0; d < 3; ++d)
      if ((st = block_back(ctx, t_count, n_parts, nullptr, d))) return st;
    ctx->n_samples += t_count;
    ctx->last_block = t_count;
    return MHC_OK;
  }
  for (int d = 0; d < ctx->n_dir; ++d) {
    const int dir = ctx->n_dir > 1 ? d : -1;
    if ((st = block_front(ctx, v, W, t_count, nullptr, dir))) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed && (st = timing_begin(ctx, &e0, &e1))) return st;
    int n_parts = 0;
    if (c.t_block == 1) {
      HIP_TRY(launch_gemv_f32(ctx->stream, reinterpret_cast<const float*>(ctx->dE),
                              reinterpret_cast<const float*>(ctx->dB), t_count, ctx->M_pad, ctx->K_pad, ctx->dJ,
                              gk ? 1 : 0, ctx->t_pad),
              "per-step contraction");
      n_parts = t_count;
    } else {
      HIP_TRY(launch_gemm(ctx->stream, c.precision, ctx->dE, ctx->dB, ctx->M_pad, ctx->K_pad, ctx->t_pad / 32,
                          ctx->dJ, gk ? 1 : 0, &n_parts, wk.ws, wk.ws_floats, wk.cnt, ctx->n_cu, c.schedule,
                          ctx->d_rowscale, ctx->d_colscale, &ctx->last_sched),
              "batched contraction");
    }
    if (e1) HIP_TRY(hipEventRecord(e1, ctx->stream), "event record");
    if ((st = block_back(ctx, t_count, n_parts, nullptr, dir))) return st;
  }
  ctx->n_samples += t_count;
  ctx->last_block = t_count;
  return MHC_OK;
}

// Second input staging set, copy stream and events of host-pointer pushes,
// created on the first such push; each piece once, so that a push after a
// failed one completes the set without leaking what was already made.
static mhc_status staging_set2(mhc_ctx* ctx) {
  mhc_status st;
  void* p = nullptr;
  if (!ctx->d_v2) {
    if ((st = dev_alloc(ctx, (size_t)ctx->chunk * ctx->N * 3 * 4, &p, "velocity staging 2"))) return st;
    ctx->d_v2 = reinterpret_cast<float*>(p);
  }
  if (!ctx->d_W2) {
    if ((st = dev_alloc(ctx, (size_t)ctx->chunk * ctx->N * 9 * 4, &p, "virial staging 2"))) return st;
    ctx->d_W2 = reinterpret_cast<float*>(p);
  }
  return MHC_OK;
}

static mhc_status host_staging(mhc_ctx* ctx) {
  if (ctx->copy_stream) return MHC_OK;
  mhc_status st;
  if ((st = staging_set2(ctx))) return st;
  for (hipEvent_t* e : {&ctx->ev_start, &ctx->ev_copied[0], &ctx->ev_copied[1], &ctx->ev_free[0], &ctx->ev_free[1]})
    if (!*e) HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming), "event create");
  hipStream_t cs = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "copy stream");
  ctx->copy_stream = cs;
  return MHC_OK;
}

// check_finite on device inputs: a scan kernel sets the context's flag, which
// is read back before anything of the push is queued (this synchronizes).
static mhc_status device_inputs_finite(mhc_ctx* ctx, const float* v, const float* W, int64_t n_steps, bool* ok) {
  HIP_TRY(launch_fill_i32(ctx->stream, ctx->d_flag, 1, 0), "clear flag");
  HIP_TRY(launch_nonfinite(ctx->stream, v, n_steps * ctx->N * 3, ctx->d_flag), "non-finite scan");
  HIP_TRY(launch_nonfinite(ctx->stream, W, n_steps * ctx->N * 9, ctx->d_flag), "non-finite scan");
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "read flag");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "non-finite check sync");
  *ok = flag == 0;
  return MHC_OK;
}

mhc_status mhc_push(mhc_ctx* ctx, int32_t n_steps, const float* v, const float* W, int on_device) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized) return fail(ctx, MHC_ERR_STATE, "push needs a finalized context");
  if (n_steps < 0) return fail(ctx, MHC_ERR_INVALID_ARG, "n_steps < 0");
  if (on_device != 0 && on_device != 1) return fail(ctx, MHC_ERR_INVALID_ARG, "on_device is 0 or 1");
  if (n_steps == 0) return MHC_OK;
  if (!v || !W) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL v or W");
  const int64_t N = ctx->N;
  if (!on_device && ctx->cfg.check_finite) {
    if (!all_finite_f(v, (int64_t)n_steps * N * 3) || !all_finite_f(W, (int64_t)n_steps * N * 9))
      return fail(ctx, MHC_ERR_NONFINITE, "non-finite velocity or virial");
  }
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  if (on_device && ctx->cfg.check_finite) {
    bool ok = false;
    if ((st = device_inputs_finite(ctx, v, W, n_steps, &ok))) return st;
    if (!ok) return fail(ctx, MHC_ERR_NONFINITE, "non-finite velocity or virial (device input)");
  }
  if (on_device) {
    for (int32_t s0 = 0; s0 < n_steps; s0 += ctx->chunk) {
      const int tc = std::min(ctx->chunk, n_steps - s0);
      if ((st = run_block(ctx, v + (int64_t)s0 * N * 3, W + (int64_t)s0 * N * 9, tc, ctx_workspace(ctx))))
        return st;
    }
    return MHC_OK;
  }
  if (n_steps <= ctx->chunk) {
    // one block: copy and kernels in order on the context stream
    HIP_TRY(hipMemcpyAsync(ctx->d_v, v, (size_t)n_steps * N * 3 * 4, hipMemcpyHostToDevice, ctx->stream), "copy v");
    HIP_TRY(hipMemcpyAsync(ctx->d_W, W, (size_t)n_steps * N * 9 * 4, hipMemcpyHostToDevice, ctx->stream), "copy W");
    if ((st = run_block(ctx, ctx->d_v, ctx->d_W, n_steps, ctx_workspace(ctx)))) return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream), "push sync");
    return MHC_OK;
  }
  // Several blocks of host inputs: block k is copied into staging set k % 2
  // on the copy stream while block k - 1 runs.  The copy stream first waits for all work queued
  // on the context stream (which may still read the staging sets, e.g. a
  // grouped push), then each copy waits for the block that last used its set.
  if ((st = host_staging(ctx))) return st;
  HIP_TRY(hipEventRecord(ctx->ev_start, ctx->stream), "event record");
  HIP_TRY(hipStreamWaitEvent(ctx->copy_stream, ctx->ev_start, 0), "stream wait");
  float* const sv[2] = {ctx->d_v, ctx->d_v2};
  float* const sW[2] = {ctx->d_W, ctx->d_W2};
  int k = 0;
  for (int32_t s0 = 0; s0 < n_steps; s0 += ctx->chunk, ++k) {
    const int tc = std::min(ctx->chunk, n_steps - s0);
    const int b = k & 1;
    if (k >= 2) HIP_TRY(hipStreamWaitEvent(ctx->copy_stream, ctx->ev_free[b], 0), "stream wait");
    HIP_TRY(hipMemcpyAsync(sv[b], v + (int64_t)s0 * N * 3, (size_t)tc * N * 3 * 4, hipMemcpyHostToDevice,
                           ctx->copy_stream), "copy v");
    HIP_TRY(hipMemcpyAsync(sW[b], W + (int64_t)s0 * N * 9, (size_t)tc * N * 9 * 4, hipMemcpyHostToDevice,
                           ctx->copy_stream), "copy W");
    HIP_TRY(hipEventRecord(ctx->ev_copied[b], ctx->copy_stream), "event record");
    HIP_TRY(hipStreamWaitEvent(ctx->stream, ctx->ev_copied[b], 0), "stream wait");
    if ((st = run_block(ctx, sv[b], sW[b], tc, ctx_workspace(ctx)))) {
      (void)hipStreamSynchronize(ctx->copy_stream);     // the caller may reuse v and W on return
      return st;
    }
    HIP_TRY(hipEventRecord(ctx->ev_free[b], ctx->stream), "event record");
  }
  // every copy precedes a kernel the context stream waited for
  HIP_TRY(hipStreamSynchronize(ctx->stream), "push sync");
  return MHC_OK;
}

mhc_status mhc_push_noalloc(mhc_ctx* ctx, int32_t n_steps, const float* v, const float* W) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized) return fail(ctx, MHC_ERR_STATE, "push needs a finalized context");
  if (n_steps < 0) return fail(ctx, MHC_ERR_INVALID_ARG, "n_steps < 0");
  if (n_steps == 0) return MHC_OK;
  if (!v || !W) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL v or W");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  Workspace wk{};
  if (ctx->cfg.t_block > 1) {
    // the same workspace size the context's own push uses, so that both take
    // the same work split and give the same bits
    if (ctx->n_cu > MHC_NOALLOC_MAX_CU)
      return fail(ctx, MHC_ERR_UNSUPPORTED,
                  "mhc_push_noalloc: the device has " + std::to_string(ctx->n_cu) +
                      " compute units; its scratch holds the contraction workspace of at most " +
                      std::to_string(MHC_NOALLOC_MAX_CU) + " (" + std::to_string(MHC_NOALLOC_SCRATCH_BYTES) +
                      " bytes)");
    void* base = nullptr;
    HIP_TRY(scratch_address(ctx->device, &base), "hipGetSymbolAddress(scratch)");
    wk.ws = reinterpret_cast<float*>(base);
    wk.ws_floats = (int64_t)ctx->n_cu * 2 * 256 * 256;
    wk.cnt = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(base) + MHC_NOALLOC_WS_FLOATS * 4);
    // the scratch keeps whatever the last call on this device left in it
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(MHC_NOALLOC_MAX_CU), 0, ctx->stream, wk.cnt, MHC_NOALLOC_MAX_CU);
    HIP_TRY(hipGetLastError(), "clear scratch counters");
  }
  const int64_t N = ctx->N;
  for (int32_t s0 = 0; s0 < n_steps; s0 += ctx->chunk) {
    const int tc = std::min(ctx->chunk, n_steps - s0);
    if ((st = run_block(ctx, v + (int64_t)s0 * N * 3, W + (int64_t)s0 * N * 9, tc, wk, false))) return st;
  }
  return MHC_OK;
}

mhc_status mhc_synchronize(mhc_ctx* ctx) {
  mhc_status st = enter(ctx);
  if (st) return st;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "synchronize");
  return MHC_OK;
}

// Finished HNEMA averages on the host: h[0 .. nd*nb*3) = bin averages
// [dir][b][mu], then the Eq. 10 total [3], then (split) the split totals [dir][mu].
static mhc_status hnema_finished(mhc_ctx* ctx, std::vector<double>& h) {
  const int nd = ctx->n_dir;
  const int64_t n = (int64_t)nd * ctx->nb * 3;
  HIP_TRY(launch_hnema_finish(ctx->stream, ctx->d_hsum, ctx->d_hcomp, n, ctx->n_samples, ctx->d_out), "finish");
  HIP_TRY(launch_hnema_finish(ctx->stream, ctx->d_tsum, ctx->d_tcomp, 3, ctx->n_samples, ctx->d_out + n), "finish");
  if (nd > 1)
    HIP_TRY(launch_hnema_finish(ctx->stream, ctx->d_tdsum, ctx->d_tdcomp, 9, ctx->n_samples, ctx->d_out + n + 3),
            "finish");
  h.resize(n + 3 + (nd > 1 ? 9 : 0));
  HIP_TRY(hipMemcpyAsync(h.data(), ctx->d_out, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream), "read");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "read sync");
  return MHC_OK;
}

mhc_status mhc_read_hnema(mhc_ctx* ctx, double* avg, double* total_avg, int64_t* n_samples) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized || !(ctx->cfg.methods & MHC_HNEMA)) return fail(ctx, MHC_ERR_STATE, "HNEMA not enabled");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<double> h;
  if ((st = hnema_finished(ctx, h))) return st;
  const int64_t n = ctx->nb * 3;
  const int nd = ctx->n_dir;
  if (avg) {
    // the whole current is the sum of the direction slices, in direction order
    for (int64_t e = 0; e < n; ++e) {
      double a = h[e];
      for (int d = 1; d < nd; ++d) a += h[(size_t)d * n + e];
      avg[e] = a;
    }
  }
  if (total_avg) std::memcpy(total_avg, h.data() + (size_t)nd * n, 24);
  if (n_samples) *n_samples = ctx->n_samples;
  return MHC_OK;
}

mhc_status mhc_read_hnema_dir(mhc_ctx* ctx, double* avg, double* total_avg, int64_t* n_samples) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized || !(ctx->cfg.methods & MHC_HNEMA) || ctx->n_dir == 1)
    return fail(ctx, MHC_ERR_STATE, "HNEMA with the direction split not enabled");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<double> h;
  if ((st = hnema_finished(ctx, h))) return st;
  const int64_t nb = ctx->nb, n = nb * 3;
  if (avg)
    for (int d = 0; d < 3; ++d)
      for (int64_t b = 0; b < nb; ++b)
        for (int mu = 0; mu < 3; ++mu) avg[(b * 3 + mu) * 3 + d] = h[(size_t)d * n + b * 3 + mu];
  if (total_avg)
    for (int d = 0; d < 3; ++d)
      for (int mu = 0; mu < 3; ++mu) total_avg[mu * 3 + d] = h[(size_t)3 * n + 3 + d * 3 + mu];
  if (n_samples) *n_samples = ctx->n_samples;
  return MHC_OK;
}

// Finished correlation and running integral of direction pass d on the host:
// h[0 .. per) = corr[tau][r][nu], h[per .. 2 per) = integral, r = 3 b + mu.
static mhc_status gkma_finished(mhc_ctx* ctx, int d, std::vector<double>& h) {
  const int L = ctx->cfg.corr_len;
  const size_t per = (size_t)L * ctx->R3 * 3;
  const double *psum = nullptr, *pcomp = nullptr;
  if (ctx->x_fill > 0) {
    // steps still buffered for a later update: their contribution goes into
    // scratch sums that the read adds, so a read leaves the running sums (and
    // the order of later updates) as they were
    HIP_TRY(hipMemsetAsync(ctx->d_psum, 0, 2 * per * 8, ctx->stream), "zero pending sums");
    mhc_status st = corr_update(ctx, ctx->x_base, ctx->x_fill, ctx->d_psum, ctx->d_psum + per);
    if (st) return st;
    psum = ctx->d_psum;
    pcomp = ctx->d_psum + per;
  }
  HIP_TRY(launch_corr_finish(ctx->stream, ctx->d_csum + d * per, ctx->d_ccomp + d * per, psum, pcomp, ctx->R3, L,
                             ctx->n_samples, ctx->cfg.dt, ctx->d_out, ctx->d_out + per),
          "finish");
  h.resize(2 * per);
  HIP_TRY(hipMemcpyAsync(h.data(), ctx->d_out, 2 * per * 8, hipMemcpyDeviceToHost, ctx->stream), "read");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "read sync");
  return MHC_OK;
}

mhc_status mhc_read_gkma(mhc_ctx* ctx, double* corr, double* integral, double* hcacf, int64_t* n_samples) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized || !(ctx->cfg.methods & MHC_GKMA)) return fail(ctx, MHC_ERR_STATE, "GKMA not enabled");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  const int L = ctx->cfg.corr_len;
  const int64_t R3 = ctx->R3, nb = ctx->nb;
  const size_t per = (size_t)L * R3 * 3;
  std::vector<double> h, acc;
  for (int d = 0; d < ctx->n_dir; ++d) {
    if ((st = gkma_finished(ctx, d, h))) return st;
    if (d == 0) {
      acc = h;
    } else {   // the whole current is the sum of the direction slices, in direction order
      for (size_t e = 0; e < 2 * per; ++e) acc[e] += h[e];
    }
  }
  for (int tau = 0; tau < L; ++tau) {
    const double* src = acc.data() + (size_t)tau * R3 * 3;
    if (corr) std::memcpy(corr + (size_t)tau * nb * 9, src, nb * 9 * 8);
    if (integral) std::memcpy(integral + (size_t)tau * nb * 9, acc.data() + per + (size_t)tau * R3 * 3, nb * 9 * 8);
  }
  if (hcacf) {   // the total current's rows are the same in every pass: take pass 0
    if (ctx->n_dir > 1 && (st = gkma_finished(ctx, 0, h))) return st;
    const std::vector<double>& h0 = ctx->n_dir > 1 ? h : acc;
    for (int tau = 0; tau < L; ++tau) std::memcpy(hcacf + (size_t)tau * 9, h0.data() + (size_t)tau * R3 * 3 + nb * 9, 9 * 8);
  }
  if (n_samples) *n_samples = ctx->n_samples;
  return MHC_OK;
}

mhc_status mhc_read_gkma_dir(mhc_ctx* ctx, double* corr, double* integral, int64_t* n_samples) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized || !(ctx->cfg.methods & MHC_GKMA) || ctx->n_dir == 1)
    return fail(ctx, MHC_ERR_STATE, "GKMA with the direction split not enabled");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  const int L = ctx->cfg.corr_len;
  const int64_t R3 = ctx->R3, nb = ctx->nb;
  const size_t per = (size_t)L * R3 * 3;
  std::vector<double> h;
  for (int d = 0; d < 3; ++d) {
    if ((st = gkma_finished(ctx, d, h))) return st;
    for (int tau = 0; tau < L; ++tau)
      for (int64_t b = 0; b < nb; ++b)
        for (int mu = 0; mu < 3; ++mu)
          for (int m2 = 0; m2 < 3; ++m2) {
            const size_t src = ((size_t)tau * R3 + b * 3 + mu) * 3 + m2;
            const size_t dst = ((((size_t)tau * nb + b) * 3 + mu) * 3 + d) * 3 + m2;
            if (corr) corr[dst] = h[src];
            if (integral) integral[dst] = h[per + src];
          }
  }
  if (n_samples) *n_samples = ctx->n_samples;
  return MHC_OK;
}

mhc_status mhc_read_gkma_cross(mhc_ctx* ctx, double* corr, double* integral, int64_t* n_samples) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized || !ctx->cross) return fail(ctx, MHC_ERR_STATE, "cross-correlations not enabled");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  const int L = ctx->cfg.corr_len;
  const int64_t R3 = ctx->R3, nb = ctx->nb;
  const size_t per = (size_t)L * R3 * 3;
  std::vector<double> h(2 * per);
  for (int64_t b2 = 0; b2 < nb; ++b2) {
    HIP_TRY(launch_corr_finish(ctx->stream, ctx->d_xsum + b2 * per, ctx->d_xcomp + b2 * per, nullptr, nullptr, R3, L,
                               ctx->n_samples, ctx->cfg.dt, ctx->d_out, ctx->d_out + per),
            "finish");
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->d_out, 2 * per * 8, hipMemcpyDeviceToHost, ctx->stream), "read");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "read sync");
    for (int tau = 0; tau < L; ++tau)
      for (int64_t b = 0; b < nb; ++b)
        for (int mu = 0; mu < 3; ++mu)
          for (int nu = 0; nu < 3; ++nu) {
            const size_t src = ((size_t)tau * R3 + b * 3 + mu) * 3 + nu;
            const size_t dst = ((((size_t)tau * nb + b) * nb + b2) * 3 + mu) * 3 + nu;
            if (corr) corr[dst] = h[src];
            if (integral) integral[dst] = h[per + src];
          }
  }
  if (n_samples) *n_samples = ctx->n_samples;
  return MHC_OK;
}

mhc_status mhc_read_block_currents(mhc_ctx* ctx, int32_t t_count, double* jb) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized || !(ctx->cfg.methods & MHC_GKMA)) return fail(ctx, MHC_ERR_STATE, "GKMA not enabled");
  if (ctx->n_dir > 1) return fail(ctx, MHC_ERR_UNSUPPORTED, "block currents are not kept with the direction split");
  if (t_count < 0 || t_count > ctx->last_block) return fail(ctx, MHC_ERR_INVALID_ARG, "t_count exceeds the last block");
  if (t_count == 0) return MHC_OK;
  if (!jb) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL output");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  const int64_t nb = ctx->nb, ld = ctx->x_cap;
  std::vector<double> h((size_t)3 * nb * ld);
  HIP_TRY(hipMemcpyAsync(h.data(), ctx->dX, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream), "read");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "read sync");
  const int64_t first = ctx->x_last + ctx->last_block - t_count;   // the last block starts at column x_last
  for (int t = 0; t < t_count; ++t)
    for (int64_t b = 0; b < nb; ++b)
      for (int mu = 0; mu < 3; ++mu) jb[((size_t)t * nb + b) * 3 + mu] = h[(size_t)(b * 3 + mu) * ld + first + t];
  return MHC_OK;
}

// ------------------------------------------------------------ save / load
namespace {
struct StateHeader {
  uint64_t magic;
  int64_t N, M, nb, L, ring_len, R3, n_samples;
  int32_t methods, precision, t_block, last_block;
  int64_t x_cap, x_fill;   // GKMA: steps buffered for a later correlation update
};
constexpr uint64_t kMagic = 0x4D48435354415432ull;  // "MHCSTAT2"
}  // namespace

// Bytes of a saved state with x_fill buffered GKMA steps (their binned series
// rows, R3 x x_fill doubles, follow the other sections).
static size_t state_bytes(const mhc_ctx* c, int64_t x_fill) {
  size_t n = sizeof(StateHeader);
  if (c->d_hsum) n += hn_doubles(c->nb, c->n_dir) * 8;
  if (c->d_csum) n += gk_doubles(c) * 8 + (size_t)c->ring_len * 3 * 8 + (size_t)c->R3 * x_fill * 8;
  n += (cross_doubles(c) + bring_doubles(c)) * 8;
  return n;
}

mhc_status mhc_save_state(mhc_ctx* ctx, void* buf, size_t* len) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized) return fail(ctx, MHC_ERR_STATE, "save needs a finalized context");
  if (!len) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL len");
  const size_t need = state_bytes(ctx, ctx->x_fill);
  if (!buf) {
    *len = need;
    return MHC_OK;
  }
  if (*len < need) return fail(ctx, MHC_ERR_INVALID_ARG, "buffer too small");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  StateHeader hd{kMagic, ctx->N, ctx->M, ctx->nb, ctx->cfg.corr_len, ctx->ring_len, ctx->R3, ctx->n_samples,
                 ctx->cfg.methods, ctx->cfg.precision, ctx->cfg.t_block, ctx->last_block, ctx->x_cap, ctx->x_fill};
  char* p = reinterpret_cast<char*>(buf);
  std::memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  if (ctx->d_hsum) {
    const size_t n = hn_doubles(ctx->nb, ctx->n_dir) * 8;
    HIP_TRY(hipMemcpyAsync(p, ctx->d_hsum, n, hipMemcpyDeviceToHost, ctx->stream), "save");
    p += n;
  }
  if (ctx->d_csum) {
    const size_t n = gk_doubles(ctx) * 8;
    HIP_TRY(hipMemcpyAsync(p, ctx->d_csum, n, hipMemcpyDeviceToHost, ctx->stream), "save");
    p += n;
    const size_t r = (size_t)ctx->ring_len * 3 * 8;
    HIP_TRY(hipMemcpyAsync(p, ctx->d_ring, r, hipMemcpyDeviceToHost, ctx->stream), "save");
    p += r;
  }
  if (ctx->cross) {
    const size_t x = cross_doubles(ctx) * 8, br = bring_doubles(ctx) * 8;
    HIP_TRY(hipMemcpyAsync(p, ctx->d_xsum, x, hipMemcpyDeviceToHost, ctx->stream), "save");
    p += x;
    HIP_TRY(hipMemcpyAsync(p, ctx->d_bring, br, hipMemcpyDeviceToHost, ctx->stream), "save");
    p += br;
  }
  if (ctx->d_csum && ctx->x_fill > 0) {   // the buffered steps' binned series, rows of x_fill
    HIP_TRY(hipMemcpy2DAsync(p, (size_t)ctx->x_fill * 8, ctx->dX, (size_t)ctx->x_cap * 8, (size_t)ctx->x_fill * 8,
                             (size_t)ctx->R3, hipMemcpyDeviceToHost, ctx->stream),
            "save");
    p += (size_t)ctx->R3 * ctx->x_fill * 8;
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream), "save sync");
  *len = need;
  return MHC_OK;
}

mhc_status mhc_load_state(mhc_ctx* ctx, const void* buf, size_t len) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!ctx->finalized) return fail(ctx, MHC_ERR_STATE, "load needs a finalized context");
  if (!buf || len < sizeof(StateHeader)) return fail(ctx, MHC_ERR_INVALID_ARG, "state size mismatch");
  StateHeader hd;
  std::memcpy(&hd, buf, sizeof hd);
  if (hd.magic != kMagic || hd.N != ctx->N || hd.M != ctx->M || hd.nb != ctx->nb || hd.L != ctx->cfg.corr_len ||
      hd.ring_len != ctx->ring_len || hd.R3 != ctx->R3 || hd.methods != ctx->cfg.methods || hd.n_samples < 0 ||
      hd.x_cap != ctx->x_cap || hd.x_fill < 0 || hd.x_fill > ctx->x_cap || hd.x_fill > hd.n_samples ||
      (!ctx->d_csum && hd.x_fill != 0))
    return fail(ctx, MHC_ERR_INVALID_ARG, "state from a different system or configuration");
  if (len != state_bytes(ctx, hd.x_fill)) return fail(ctx, MHC_ERR_INVALID_ARG, "state size mismatch");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  const char* p = reinterpret_cast<const char*>(buf) + sizeof hd;
  if (ctx->d_hsum) {
    const size_t n = hn_doubles(ctx->nb, ctx->n_dir) * 8;
    HIP_TRY(hipMemcpyAsync(ctx->d_hsum, p, n, hipMemcpyHostToDevice, ctx->stream), "load");
    p += n;
  }
  if (ctx->d_csum) {
    const size_t n = gk_doubles(ctx) * 8;
    HIP_TRY(hipMemcpyAsync(ctx->d_csum, p, n, hipMemcpyHostToDevice, ctx->stream), "load");
    p += n;
    const size_t r = (size_t)ctx->ring_len * 3 * 8;
    HIP_TRY(hipMemcpyAsync(ctx->d_ring, p, r, hipMemcpyHostToDevice, ctx->stream), "load");
    p += r;
  }
  if (ctx->cross) {
    const size_t x = cross_doubles(ctx) * 8, br = bring_doubles(ctx) * 8;
    HIP_TRY(hipMemcpyAsync(ctx->d_xsum, p, x, hipMemcpyHostToDevice, ctx->stream), "load");
    p += x;
    HIP_TRY(hipMemcpyAsync(ctx->d_bring, p, br, hipMemcpyHostToDevice, ctx->stream), "load");
    p += br;
  }
  if (hd.x_fill > 0)
    HIP_TRY(hipMemcpy2DAsync(ctx->dX, (size_t)ctx->x_cap * 8, p, (size_t)hd.x_fill * 8, (size_t)hd.x_fill * 8,
                             (size_t)ctx->R3, hipMemcpyHostToDevice, ctx->stream),
            "load");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "load sync");
  ctx->n_samples = hd.n_samples;
  ctx->last_block = 0;
  ctx->x_fill = hd.x_fill;
  ctx->x_base = hd.n_samples - hd.x_fill;
  ctx->x_last = 0;
  return MHC_OK;
}

// ------------------------------------------------------------ diagnostics
mhc_status mhc_set_timing(mhc_ctx* ctx, int enable) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (enable != 0 && enable != 1) return fail(ctx, MHC_ERR_INVALID_ARG, "enable is 0 or 1");
  ctx->timing = enable == 1;
  return MHC_OK;
}

mhc_status mhc_kernel_timing(mhc_ctx* ctx, int64_t* launches, double* total_ms) {
  mhc_status st = enter(ctx);
  if (st) return st;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "timing sync");
  double tot = 0.0;
  for (size_t q = 0; q + 1 < ctx->ev_used; q += 2) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[q], ctx->ev[q + 1]), "elapsed");
    tot += ms;
  }
  if (launches) *launches = (int64_t)(ctx->ev_used / 2);
  if (total_ms) *total_ms = tot;
  ctx->ev_used = 0;
  return MHC_OK;
}

mhc_status mhc_device_bytes(mhc_ctx* ctx, int64_t* bytes) {
  mhc_status st = enter(ctx);
  if (st) return st;
  if (!bytes) return fail(ctx, MHC_ERR_INVALID_ARG, "NULL bytes");
  *bytes = ctx->bytes;
  return MHC_OK;
}

mhc_status mhc_last_schedule(mhc_ctx* ctx, int32_t* schedule) {
  if (!ctx || !schedule) return MHC_ERR_INVALID_ARG;
  *schedule = ctx->last_sched;
  return MHC_OK;
}

}  // extern "C"

// ================================================================= groups
// Several systems pushed together: per block, the fronts of all systems, one
// persistent contraction over all their tiles (largest first), and the
// backs of all systems, optionally captured once as a HIP graph and replayed.
constexpr int TAB_RING = 8;   // pinned input-table slots of a group
constexpr int TAB_W = 5;      // table words per system
constexpr int NAUX = 4;       // side streams of a group (the device has 4 hardware queues per process)

struct mhc_group {
  std::vector<mhc_ctx*> sys;
  int device = 0;
  hipStream_t stream = nullptr;
  int prec = 0, t_block = 0, ntb = 0, shape = 0;
  bool use_graph = false, autotune = false, tuned = false;
  double tuned_ms[3] = {-1.0, -1.0, -1.0};
  int n_cu = 256;
  std::vector<DevBuf> allocs;
  GemmGeom* d_geom = nullptr;
  GroupTile* d_tiles = nullptr;
  int* d_counter = nullptr;
  int n_tiles = 0;
  std::vector<int> n_parts;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string err;
  // Block table: words TAB_W i + 0 .. 4 = v, W, the first step index of
  // system i for the block the queued work will process, the block's column
  // in the system's GKMA series buffer and the number of buffered steps the
  // correlation update correlates after the block (0: none).  Each block's
  // table is written to its own pinned ring slot, copied to the device in
  // stream order, and the slot is reused only after that copy has completed
  // (event).
  uint64_t* d_tab = nullptr;
  uint64_t* h_tab = nullptr;                // [TAB_RING][TAB_W n]
  // The input prep of all systems runs as one launch (two for e4m3: the
  // column maxima first) over per-system descriptors that read v and W
  // through the block table.
  PrepDesc* d_prep = nullptr;
  int n_wg_cs = 0, n_wg_prep = 0;
  // The back end of all systems likewise (four launches) unless a system
  // keeps cross-correlations, which fan out per system as before.
  bool back_grouped = false;
  BackGroup back{};
  void* d_back = nullptr;           // BackDesc[n], ReduceArgs[n], int wg0[3][n]
  // Per-system front and back kernels fan out over NAUX streams (joined
  // before and after the shared contraction), so small systems' kernels run
  // side by side instead of one after another.
  hipStream_t aux[NAUX] = {};
  std::vector<int> aux_of;      // side stream of each system (balanced by estimated cost)
  hipEvent_t fork_ev = nullptr, join_ev[NAUX] = {};
  hipEvent_t tab_ev[TAB_RING] = {};
  bool tab_busy[TAB_RING] = {};
  // host-input pushes of several blocks: copies of block k go to staging set
  // k % 2 of every system on this stream while block k - 1 runs
  hipStream_t copy_stream = nullptr;
  hipEvent_t cp_start = nullptr, cp_done[2] = {nullptr, nullptr}, cp_free[2] = {nullptr, nullptr};
  int tab_pos = 0;
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
};

namespace {

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;   // (precision, T, system sizes) -> tile shape

mhc_status gfail(mhc_group* g, mhc_status st, const std::string& msg) {
  g->err = msg;
  return st;
}

#define GHIP_TRY(call, where)                                                                  \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return gfail(g, MHC_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e_)); \
  } while (0)

std::string tune_key(const mhc_group* g) {
  std::vector<int64_t> n;
  for (auto* c : g->sys) n.push_back(c->M_pad * 1000003 + c->K_pad);
  std::sort(n.begin(), n.end());
  std::string k = std::to_string(g->prec) + "/" + std::to_string(g->t_block);
  for (auto x : n) k += "/" + std::to_string(x);
  return k;
}

// Descriptors and the largest-first tile queue for the current shape.
// Descriptors of the grouped back end (the reduction's part count depends on
// the tile shape, so they are rebuilt with the queue).
mhc_status build_back(mhc_group* g) {
  if (!g->back_grouped) return MHC_OK;
  const int n = (int)g->sys.size();
  const int T = g->t_block;
  const int TT = T <= 64 ? 64 : (T <= 128 ? 128 : 256);
  const int G = 256 / TT;
  std::vector<BackDesc> bd(n);
  std::vector<ReduceArgs> ra(n);
  std::vector<int> w(3 * n);
  int64_t ws = 0, wr = 0, wc = 0;
  for (int i = 0; i < n; ++i) {
    mhc_ctx* c = g->sys[i];
    const bool gk = c->cfg.methods & MHC_GKMA;
    const int64_t* t0_dev = reinterpret_cast<const int64_t*>(g->d_tab + TAB_W * i + 2);
    const int64_t* xoff_dev = reinterpret_cast<const int64_t*>(g->d_tab + TAB_W * i + 3);
    const int64_t* tbuf_dev = reinterpret_cast<const int64_t*>(g->d_tab + TAB_W * i + 4);
    ReduceArgs& a = ra[i];
    a = ReduceArgs{};
    a.in = c->dJ;
    a.layout_g = gk ? 1 : 0;
    a.n_parts = g->n_parts[i];
    a.M_pad = c->M_pad;
    a.ld = c->t_pad;
    a.t_count = T;
    a.bin_off = c->d_bin_off;
    a.slot_bin = c->d_slot_bin;
    a.seg_part = c->d_seg_part;
    a.n_seg = c->n_seg;
    a.nb = c->nb;
    a.jtot = c->d_jtot;
    a.hsum = c->d_hsum;
    a.hcomp = c->d_hcomp;
    a.tsum = c->d_tsum;
    a.tcomp = c->d_tcomp;
    a.X = gk ? c->dX : nullptr;
    a.ring = c->d_ring;
    a.ring_len = c->ring_len;
    a.t0_dev = t0_dev;
    a.ldx = gk ? c->x_cap : c->t_pad;
    a.xoff_dev = gk ? xoff_dev : nullptr;
    BackDesc& d = bd[i];
    d.jt_part = c->d_jt;
    d.n_chunks = c->n_atom_chunks;
    d.jtot = c->d_jtot;
    d.X = c->dX;
    d.ldx = c->x_cap;
    d.R3 = c->R3;
    d.L = gk ? c->cfg.corr_len : 0;
    d.ring = c->d_ring;
    d.ring_len = c->ring_len;
    d.csum = c->d_csum;
    d.ccomp = c->d_ccomp;
    d.t0_dev = t0_dev;
    d.tbuf_dev = tbuf_dev;
    d.n_rt = gk ? (int)((c->R3 + 63) / 64) : 0;
    w[i] = (int)ws;
    w[n + i] = (int)wr;
    w[2 * n + i] = (int)wc;
    if (gk && c->n_seg > 0) ws += (c->n_seg + G - 1) / G;
    wr += c->nb + 1;
    if (gk) wc += (int64_t)d.n_rt * ((d.L + 63) / 64);
  }
  if (ws > INT32_MAX || wr > INT32_MAX || wc > INT32_MAX) return gfail(g, MHC_ERR_INVALID_ARG, "group too large");
  char* base = static_cast<char*>(g->d_back);
  const size_t o_red = (size_t)n * sizeof(BackDesc), o_w = o_red + (size_t)n * sizeof(ReduceArgs);
  GHIP_TRY(hipMemcpy(base, bd.data(), o_red, hipMemcpyHostToDevice), "back descriptors");
  GHIP_TRY(hipMemcpy(base + o_red, ra.data(), (size_t)n * sizeof(ReduceArgs), hipMemcpyHostToDevice),
           "reduce descriptors");
  GHIP_TRY(hipMemcpy(base + o_w, w.data(), w.size() * sizeof(int), hipMemcpyHostToDevice), "back offsets");
  const int* wd = reinterpret_cast<const int*>(base + o_w);
  g->back.d = reinterpret_cast<const BackDesc*>(base);
  g->back.red = reinterpret_cast<const ReduceArgs*>(base + o_red);
  g->back.wg0_seg = wd;
  g->back.wg0_red = wd + n;
  g->back.wg0_corr = wd + 2 * n;
  g->back.n_wg_seg = (int)ws;
  g->back.n_wg_red = (int)wr;
  g->back.n_wg_corr = (int)wc;
  return MHC_OK;
}

mhc_status build_queue(mhc_group* g) {
  const int n = (int)g->sys.size();
  std::vector<GemmGeom> geom(n);
  std::vector<GroupTile> tiles;
  std::vector<std::pair<int64_t, int>> order;
  g->n_parts.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    mhc_ctx* c = g->sys[i];
    int n_m = 0;
    gemm_geom(g->prec, g->shape, c->dE, c->dB, c->dJ, c->M_pad, c->K_pad, g->ntb,
              (c->cfg.methods & MHC_GKMA) ? 1 : 0, c->d_rowscale, c->d_colscale, &geom[i], &n_m);
    g->n_parts[i] = geom[i].n_ntiles;
    if (c->n3) {   // direction split as one contraction
      geom[i].s3 = (int)(c->n3 / stage_dofs_of(g->prec));
      geom[i].region = c->j_region;
      geom[i].ws = c->d_ws;
    }
    order.push_back({c->K_pad, i});
  }
  std::stable_sort(order.begin(), order.end(), [](auto a, auto b) { return a.first > b.first; });
  for (auto& o : order) {
    const int i = o.second;
    const int nt = (int)(g->sys[i]->M_pad / gemm_shape_rows(g->shape)) * geom[i].n_ntiles;
    for (int t = 0; t < nt; ++t) tiles.push_back({i, t});
  }
  g->n_tiles = (int)tiles.size();
  GHIP_TRY(hipMemcpyAsync(g->d_geom, geom.data(), n * sizeof(GemmGeom), hipMemcpyHostToDevice, g->stream), "geom");
  GHIP_TRY(hipMemcpyAsync(g->d_tiles, tiles.data(), tiles.size() * sizeof(GroupTile), hipMemcpyHostToDevice,
                          g->stream),
           "tiles");
  GHIP_TRY(hipStreamSynchronize(g->stream), "queue sync");
  return build_back(g);
}

mhc_status group_contract(mhc_group* g) {
  GHIP_TRY(launch_fill_i32(g->stream, g->d_counter, 1, 0), "queue reset");
  bool with_dir = false;
  for (auto* c : g->sys) with_dir |= c->n3 > 0;
  GHIP_TRY(launch_gemm_group(g->stream, g->prec, g->shape, g->d_geom, g->d_tiles, g->n_tiles, g->d_counter,
                             std::min(g->n_cu, g->n_tiles), with_dir),
           "grouped contraction");
  return MHC_OK;
}

// Run fn(i) for every system with the system's work queued on side stream
// i % NAUX, forked from and joined back into the group stream.
template <class F>
mhc_status fan_out(mhc_group* g, F&& fn) {
  GHIP_TRY(hipEventRecord(g->fork_ev, g->stream), "fork");
  for (int k = 0; k < NAUX; ++k) GHIP_TRY(hipStreamWaitEvent(g->aux[k], g->fork_ev, 0), "fork wait");
  mhc_status st = MHC_OK;
  for (size_t i = 0; i < g->sys.size() && !st; ++i) {
    mhc_ctx* c = g->sys[i];
    hipStream_t own = c->stream;
    c->stream = g->aux[g->aux_of[i]];
    st = fn(i);
    c->stream = own;
  }
  for (int k = 0; k < NAUX; ++k) {
    GHIP_TRY(hipEventRecord(g->join_ev[k], g->aux[k]), "join");
    GHIP_TRY(hipStreamWaitEvent(g->stream, g->join_ev[k], 0), "join wait");
  }
  return st;
}

// The whole block (inputs named by the block table).
mhc_status group_block(mhc_group* g, bool timed) {
  mhc_status st;
  GHIP_TRY(launch_prep_group(g->stream, g->prec, g->d_prep, (int)g->sys.size(), g->t_block, g->n_wg_cs,
                             g->n_wg_prep),
           "grouped input prep");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    while (g->ev_used + 2 > g->ev.size()) {
      hipEvent_t e;
      GHIP_TRY(hipEventCreate(&e), "event create");
      g->ev.push_back(e);
    }
    e0 = g->ev[g->ev_used];
    e1 = g->ev[g->ev_used + 1];
    g->ev_used += 2;
    GHIP_TRY(hipEventRecord(e0, g->stream), "event record");
  }
  if ((st = group_contract(g))) return st;
  if (timed) GHIP_TRY(hipEventRecord(e1, g->stream), "event record");
  if (g->back_grouped) {
    GHIP_TRY(launch_back_group(g->stream, g->back, (int)g->sys.size(), g->t_block), "grouped back end");
    return MHC_OK;
  }
  return fan_out(g, [&](size_t i) {
    mhc_ctx* c = g->sys[i];
    const int64_t* w = reinterpret_cast<const int64_t*>(g->d_tab + TAB_W * i);
    mhc_status s2 = MHC_OK;
    if (c->n_dir > 1) {   // the three directions' regions, one after the other
      for (int d = 0; d < 3 && !s2; ++d) s2 = block_back(c, g->t_block, g->n_parts[i], w + 2, d, w + 3, w + 4);
    } else {
      s2 = block_back(c, g->t_block, g->n_parts[i], w + 2, -1, w + 3, w + 4);
    }
    return s2 ? gfail(g, s2, c->err) : MHC_OK;
  });
}

// Time every valid tile shape on the staged block and keep the fastest.
// The shapes are timed alternately, one launch per event pair after a host
// synchronisation, over several rounds, and each keeps its best launch:
// back-to-back launches of one shape hold the chip at its sustained power
// limit, where the shapes come out nearly equal, while a push leaves the
// front and back kernels between contractions.  The preferred shape (the
// lowest valid index, the largest tile) is kept unless another one is more
// than 3 % faster.
mhc_status autotune(mhc_group* g) {
  const std::string key = tune_key(g);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      g->shape = it->second;
      g->tuned = true;
      return build_queue(g);
    }
  }
  for (size_t i = 0; i < g->sys.size(); ++i) {
    mhc_ctx* c = g->sys[i];
    mhc_status st =
        block_front(c, nullptr, nullptr, g->t_block, reinterpret_cast<const float* const*>(g->d_tab + TAB_W * i));
    if (st) return gfail(g, st, c->err);
  }
  std::vector<int> shapes;
  for (int shape = 0; shape < 3; ++shape)
    if (gemm_shape_valid(shape, g->ntb)) shapes.push_back(shape);
  hipEvent_t a, b;
  GHIP_TRY(hipEventCreate(&a), "event");
  GHIP_TRY(hipEventCreate(&b), "event");
  constexpr int ROUNDS = 4;                 // timed rounds after one warm-up round
  double best_of[3] = {1e300, 1e300, 1e300};
  for (int r = 0; r <= ROUNDS; ++r) {
    for (int shape : shapes) {
      g->shape = shape;
      mhc_status st = build_queue(g);       // synchronizes the stream
      if (st) return st;
      GHIP_TRY(hipEventRecord(a, g->stream), "event");
      if ((st = group_contract(g))) return st;
      GHIP_TRY(hipEventRecord(b, g->stream), "event");
      GHIP_TRY(hipEventSynchronize(b), "event sync");
      float ms = 0.f;
      GHIP_TRY(hipEventElapsedTime(&ms, a, b), "elapsed");
      if (r > 0) best_of[shape] = std::min(best_of[shape], (double)ms);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  int best = shapes.empty() ? 0 : shapes[0];
  for (int shape : shapes) {
    g->tuned_ms[shape] = best_of[shape];
    if (best_of[shape] < 0.97 * best_of[best]) best = shape;
  }
  g->shape = best;
  g->tuned = true;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  return build_queue(g);
}

}  // namespace

extern "C" {

mhc_status mhc_group_create(mhc_ctx* const* systems, int32_t n, int32_t flags, mhc_group** out) {
  if (!out) return MHC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!systems || n < 1 || n > 4096) return MHC_ERR_INVALID_ARG;
  if (flags & ~(MHC_GROUP_GRAPH | MHC_GROUP_AUTOTUNE)) return MHC_ERR_INVALID_ARG;
  mhc_ctx* c0 = systems[0];
  for (int i = 0; i < n; ++i) {
    mhc_ctx* c = systems[i];
    if (!c) return MHC_ERR_INVALID_ARG;
    if (c->sticky) return c->sticky;
    if (!c->finalized || c->cfg.t_block == 1) return MHC_ERR_STATE;
    // grouped pushes run one contraction per block: the direction split in
    // its one-contraction form (every T-batched context has it)
    if (c->n_dir > 1 && !c->n3) return MHC_ERR_UNSUPPORTED;
    if (c->device != c0->device || c->stream != c0->stream || c->cfg.precision != c0->cfg.precision ||
        c->cfg.t_block != c0->cfg.t_block)
      return MHC_ERR_INVALID_ARG;
    for (int j = 0; j < i; ++j)
      if (systems[j] == c) return MHC_ERR_INVALID_ARG;
  }
  mhc_group* g = new (std::nothrow) mhc_group();
  if (!g) return MHC_ERR_OOM;
  g->sys.assign(systems, systems + n);
  g->device = c0->device;
  g->stream = c0->stream;
  g->prec = c0->cfg.precision;
  g->t_block = c0->cfg.t_block;
  g->ntb = g->t_block / 32;
  g->use_graph = flags & MHC_GROUP_GRAPH;
  g->autotune = flags & MHC_GROUP_AUTOTUNE;
  g->n_cu = c0->n_cu;
  g->shape = (g->ntb % 4 == 0) ? 0 : (g->ntb % 2 == 0 ? 1 : 2);
  {
    // longest-processing-time assignment of systems to side streams; a
    // system's front and back work scales with its modes, GKMA's correlation
    // update with its bins x lags
    std::vector<std::pair<double, int>> cost;
    for (int i = 0; i < n; ++i) {
      const mhc_ctx* c = systems[i];
      double w = (double)c->M_pad;
      if (c->cfg.methods & MHC_GKMA) w += 3.0 * (c->nb + 1) * c->cfg.corr_len * 3.0 / g->t_block;
      cost.push_back({w, i});
    }
    std::stable_sort(cost.begin(), cost.end(), [](auto a, auto b) { return a.first > b.first; });
    double load[NAUX] = {};
    g->aux_of.assign(n, 0);
    for (auto& ci : cost) {
      int k = (int)(std::min_element(load, load + NAUX) - load);
      g->aux_of[ci.second] = k;
      load[k] += ci.first;
    }
  }
  auto cleanup = [&](mhc_status st) {
    for (auto& a : g->allocs) (void)hipFree(a.p);
    if (g->h_tab) (void)hipHostFree(g->h_tab);
    for (auto e : g->tab_ev)
      if (e) (void)hipEventDestroy(e);
    if (g->fork_ev) (void)hipEventDestroy(g->fork_ev);
    for (int k = 0; k < NAUX; ++k) {
      if (g->join_ev[k]) (void)hipEventDestroy(g->join_ev[k]);
      if (g->aux[k]) (void)hipStreamDestroy(g->aux[k]);
    }
    delete g;
    return st;
  };
  if (hipSetDevice(g->device) != hipSuccess) return cleanup(MHC_ERR_HIP);
  int64_t max_tiles = 0;
  for (auto* c : g->sys) max_tiles += (c->M_pad / 128) * g->ntb;   // upper bound over shapes
  void *pg = nullptr, *pt = nullptr, *pc = nullptr;
  if (hipMalloc(&pg, n * sizeof(GemmGeom)) != hipSuccess) return cleanup(MHC_ERR_OOM);
  g->allocs.push_back({pg, n * sizeof(GemmGeom)});
  if (hipMalloc(&pt, max_tiles * sizeof(GroupTile)) != hipSuccess) return cleanup(MHC_ERR_OOM);
  g->allocs.push_back({pt, (size_t)max_tiles * sizeof(GroupTile)});
  if (hipMalloc(&pc, 256) != hipSuccess) return cleanup(MHC_ERR_OOM);
  g->allocs.push_back({pc, 256});
  void* ptab = nullptr;
  if (hipMalloc(&ptab, TAB_W * n * sizeof(uint64_t)) != hipSuccess) return cleanup(MHC_ERR_OOM);
  g->allocs.push_back({ptab, TAB_W * n * sizeof(uint64_t)});
  g->d_tab = reinterpret_cast<uint64_t*>(ptab);
  if (hipHostMalloc(reinterpret_cast<void**>(&g->h_tab), TAB_RING * TAB_W * n * sizeof(uint64_t), 0) != hipSuccess)
    return cleanup(MHC_ERR_OOM);
  for (int k = 0; k < TAB_RING; ++k)
    if (hipEventCreateWithFlags(&g->tab_ev[k], hipEventDisableTiming) != hipSuccess) return cleanup(MHC_ERR_HIP);
  if (hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming) != hipSuccess) return cleanup(MHC_ERR_HIP);
  for (int k = 0; k < NAUX; ++k) {
    if (hipStreamCreateWithFlags(&g->aux[k], hipStreamNonBlocking) != hipSuccess) return cleanup(MHC_ERR_HIP);
    if (hipEventCreateWithFlags(&g->join_ev[k], hipEventDisableTiming) != hipSuccess) return cleanup(MHC_ERR_HIP);
  }
  g->d_geom = reinterpret_cast<GemmGeom*>(pg);
  g->d_tiles = reinterpret_cast<GroupTile*>(pt);
  g->d_counter = reinterpret_cast<int*>(pc);
  {
    std::vector<PrepDesc> pd(n);
    int64_t wcs = 0, wpr = 0;
    for (int i = 0; i < n; ++i) {
      mhc_ctx* c = g->sys[i];
      PrepDesc& d = pd[i];
      d.sqrt_m = c->d_sqrtm;
      d.inv_sqrt_m = c->d_isqrtm;
      d.N = c->N;
      d.t_pad = c->t_pad;
      d.n_chunks = c->n_atom_chunks;
      d.B = c->dB;
      d.K_pad = c->K_pad;
      d.jt_part = c->d_jt;
      d.col_scale = c->d_colscale;
      d.col_part = c->d_colpart;
      d.tab = reinterpret_cast<const float* const*>(g->d_tab + TAB_W * i);
      d.dir = c->n3 ? DIR_ALL : -1;
      d.jd_part = c->n3 ? c->d_jd : nullptr;
      d.wg0_cs = (int)wcs;
      d.wg0_prep = (int)wpr;
      wcs += (int64_t)c->t_pad * ((c->N + COLSCALE_ATOMS - 1) / COLSCALE_ATOMS);
      wpr += (int64_t)c->n_atom_chunks * ((c->t_pad + 31) / 32);
    }
    if (wcs > INT32_MAX || wpr > INT32_MAX) return cleanup(MHC_ERR_INVALID_ARG);
    g->n_wg_cs = (int)wcs;
    g->n_wg_prep = (int)wpr;
    void* pp = nullptr;
    if (hipMalloc(&pp, n * sizeof(PrepDesc)) != hipSuccess) return cleanup(MHC_ERR_OOM);
    g->allocs.push_back({pp, n * sizeof(PrepDesc)});
    g->d_prep = reinterpret_cast<PrepDesc*>(pp);
    if (hipMemcpy(pp, pd.data(), n * sizeof(PrepDesc), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(MHC_ERR_HIP);
  }
  g->back_grouped = true;
  for (auto* c : g->sys)
    if (c->cross || c->n_dir > 1) g->back_grouped = false;
  if (g->back_grouped) {
    const size_t bytes = (size_t)n * (sizeof(BackDesc) + sizeof(ReduceArgs) + 3 * sizeof(int));
    void* pb = nullptr;
    if (hipMalloc(&pb, bytes) != hipSuccess) return cleanup(MHC_ERR_OOM);
    g->allocs.push_back({pb, bytes});
    g->d_back = pb;
  }
  if (build_queue(g) != MHC_OK) return cleanup(MHC_ERR_HIP);
  *out = g;
  return MHC_OK;
}

mhc_status mhc_group_destroy(mhc_group* g) {
  if (!g) return MHC_OK;
  (void)hipSetDevice(g->device);
  (void)hipStreamSynchronize(g->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (auto e : g->ev) (void)hipEventDestroy(e);
  for (auto& a : g->allocs) (void)hipFree(a.p);
  if (g->h_tab) (void)hipHostFree(g->h_tab);
  for (auto e : g->tab_ev)
    if (e) (void)hipEventDestroy(e);
  if (g->fork_ev) (void)hipEventDestroy(g->fork_ev);
  for (int k = 0; k < NAUX; ++k) {
    if (g->aux[k]) (void)hipStreamSynchronize(g->aux[k]);
    if (g->join_ev[k]) (void)hipEventDestroy(g->join_ev[k]);
    if (g->aux[k]) (void)hipStreamDestroy(g->aux[k]);
  }
  if (g->copy_stream) {
    (void)hipStreamSynchronize(g->copy_stream);
    (void)hipStreamDestroy(g->copy_stream);
  }
  for (hipEvent_t e : {g->cp_start, g->cp_done[0], g->cp_done[1], g->cp_free[0], g->cp_free[1]})
    if (e) (void)hipEventDestroy(e);
  delete g;
  return MHC_OK;
}

const char* mhc_group_last_error(const mhc_group* g) { return g ? g->err.c_str() : ""; }

mhc_status mhc_group_push(mhc_group* g, int32_t n_steps, const float* const* v, const float* const* W,
                          int on_device) {
  if (!g) return MHC_ERR_INVALID_ARG;
  g->err.clear();
  if (n_steps < 0 || (on_device != 0 && on_device != 1)) return gfail(g, MHC_ERR_INVALID_ARG, "bad arguments");
  if (n_steps == 0) return MHC_OK;
  if (!v || !W) return gfail(g, MHC_ERR_INVALID_ARG, "NULL pointer arrays");
  const int n = (int)g->sys.size();
  for (int i = 0; i < n; ++i) {
    if (!v[i] || !W[i]) return gfail(g, MHC_ERR_INVALID_ARG, "NULL input pointer");
    if (g->sys[i]->sticky) return gfail(g, g->sys[i]->sticky, "system " + std::to_string(i) + " has a HIP error");
  }
  GHIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  // check_finite of the member contexts, before anything is queued
  for (int i = 0; i < n; ++i) {
    mhc_ctx* c = g->sys[i];
    if (!c->cfg.check_finite) continue;
    bool ok = true;
    if (!on_device) {
      ok = all_finite_f(v[i], (int64_t)n_steps * c->N * 3) && all_finite_f(W[i], (int64_t)n_steps * c->N * 9);
    } else {
      mhc_status st = device_inputs_finite(c, v[i], W[i], n_steps, &ok);
      if (st) return gfail(g, st, c->err);
    }
    if (!ok)
      return gfail(g, MHC_ERR_NONFINITE, "non-finite velocity or virial of system " + std::to_string(i));
  }
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const int T = g->t_block;
  // host inputs of two or more full blocks: copies on the copy stream into
  // alternating staging sets, overlapped with the previous block's kernels
  // (the copy stream first waits for everything queued on the group stream,
  // then each copy for the block that last read its set)
  const bool overlap = !on_device && n_steps >= 2 * T;
  if (overlap) {
    for (auto* c : g->sys) {
      mhc_status st = staging_set2(c);
      if (st) return gfail(g, st, c->err);
    }
    for (hipEvent_t* e : {&g->cp_start, &g->cp_done[0], &g->cp_done[1], &g->cp_free[0], &g->cp_free[1]})
      if (!*e) GHIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming), "event create");
    if (!g->copy_stream) {
      hipStream_t cs = nullptr;
      GHIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "copy stream");
      g->copy_stream = cs;
    }
    GHIP_TRY(hipEventRecord(g->cp_start, g->stream), "event record");
    GHIP_TRY(hipStreamWaitEvent(g->copy_stream, g->cp_start, 0), "stream wait");
  }
  int32_t s0 = 0;
  for (int blk = 0; s0 + T <= n_steps; s0 += T, ++blk) {
    // device inputs are read in place; host inputs go through the staging buffers
    const int b = blk & 1;
    if (overlap && blk >= 2) GHIP_TRY(hipStreamWaitEvent(g->copy_stream, g->cp_free[b], 0), "stream wait");
    const int k = g->tab_pos;
    g->tab_pos = (g->tab_pos + 1) % TAB_RING;
    if (g->tab_busy[k]) GHIP_TRY(hipEventSynchronize(g->tab_ev[k]), "input table slot");
    uint64_t* tab = g->h_tab + (size_t)k * TAB_W * n;
    for (int i = 0; i < n; ++i) {
      mhc_ctx* c = g->sys[i];
      const float* vi = v[i] + (int64_t)s0 * c->N * 3;
      const float* Wi = W[i] + (int64_t)s0 * c->N * 9;
      if (!on_device) {
        float* sv = (overlap && b) ? c->d_v2 : c->d_v;
        float* sW = (overlap && b) ? c->d_W2 : c->d_W;
        hipStream_t cs = overlap ? g->copy_stream : g->stream;
        GHIP_TRY(hipMemcpyAsync(sv, vi, (size_t)T * c->N * 3 * 4, hipMemcpyHostToDevice, cs), "v");
        GHIP_TRY(hipMemcpyAsync(sW, Wi, (size_t)T * c->N * 9 * 4, hipMemcpyHostToDevice, cs), "W");
        vi = sv;
        Wi = sW;
      }
      tab[TAB_W * i] = reinterpret_cast<uint64_t>(vi);
      tab[TAB_W * i + 1] = reinterpret_cast<uint64_t>(Wi);
      tab[TAB_W * i + 2] = (uint64_t)c->n_samples;
      int64_t xoff = 0, tbuf = 0;
      if (c->cfg.methods & MHC_GKMA) fold_step(c, T, &xoff, &tbuf);
      tab[TAB_W * i + 3] = (uint64_t)xoff;
      tab[TAB_W * i + 4] = (uint64_t)tbuf;
    }
    if (overlap) {
      GHIP_TRY(hipEventRecord(g->cp_done[b], g->copy_stream), "event record");
      GHIP_TRY(hipStreamWaitEvent(g->stream, g->cp_done[b], 0), "stream wait");
    }
    GHIP_TRY(hipMemcpyAsync(g->d_tab, tab, TAB_W * n * sizeof(uint64_t), hipMemcpyHostToDevice, g->stream),
             "block table");
    GHIP_TRY(hipEventRecord(g->tab_ev[k], g->stream), "input table event");
    g->tab_busy[k] = true;
    if (g->autotune && !g->tuned) {
      mhc_status st = autotune(g);
      if (st) {
        if (overlap) (void)hipStreamSynchronize(g->copy_stream);   // the caller may reuse v and W on return
        return st;
      }
    }
    mhc_status st;
    if (g->use_graph && !g->timing) {
      if (!g->exec) {
        GHIP_TRY(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed), "begin capture");
        st = group_block(g, false);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(g->stream, &graph);
        if (st) {
          if (graph) (void)hipGraphDestroy(graph);
          if (overlap) (void)hipStreamSynchronize(g->copy_stream);
          return st;
        }
        GHIP_TRY(e, "end capture");
        g->graph = graph;
        GHIP_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "instantiate");
      }
      GHIP_TRY(hipGraphLaunch(g->exec, g->stream), "graph launch");
    } else {
      if ((st = group_block(g, g->timing))) {
        if (overlap) (void)hipStreamSynchronize(g->copy_stream);
        return st;
      }
    }
    if (overlap) GHIP_TRY(hipEventRecord(g->cp_free[b], g->stream), "event record");
    for (auto* c : g->sys) {
      c->n_samples += T;
      c->last_block = T;
    }
  }
  // trailing partial block: each system on its own
  if (s0 < n_steps) {
    const int tc = n_steps - s0;
    for (int i = 0; i < n; ++i) {
      mhc_ctx* c = g->sys[i];
      GHIP_TRY(hipMemcpyAsync(c->d_v, v[i] + (int64_t)s0 * c->N * 3, (size_t)tc * c->N * 3 * 4, kind, g->stream), "v");
      GHIP_TRY(hipMemcpyAsync(c->d_W, W[i] + (int64_t)s0 * c->N * 9, (size_t)tc * c->N * 9 * 4, kind, g->stream), "W");
      mhc_status st = run_block(c, c->d_v, c->d_W, tc, ctx_workspace(c));
      if (st) return gfail(g, st, c->err);
    }
  }
  if (!on_device) GHIP_TRY(hipStreamSynchronize(g->stream), "push sync");
  return MHC_OK;
}

mhc_status mhc_group_info(mhc_group* g, int32_t* tile_shape, double* tuned_ms, int64_t* n_tiles) {
  if (!g) return MHC_ERR_INVALID_ARG;
  if (tile_shape) *tile_shape = g->shape;
  if (tuned_ms)
    for (int i = 0; i < 3; ++i) tuned_ms[i] = g->tuned_ms[i];
  if (n_tiles) *n_tiles = g->n_tiles;
  return MHC_OK;
}

mhc_status mhc_group_set_timing(mhc_group* g, int enable) {
  if (!g || (enable != 0 && enable != 1)) return MHC_ERR_INVALID_ARG;
  g->timing = enable == 1;
  return MHC_OK;
}

mhc_status mhc_group_kernel_timing(mhc_group* g, int64_t* launches, double* total_ms) {
  if (!g) return MHC_ERR_INVALID_ARG;
  GHIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  GHIP_TRY(hipStreamSynchronize(g->stream), "timing sync");
  double tot = 0.0;
  for (size_t q = 0; q + 1 < g->ev_used; q += 2) {
    float ms = 0.f;
    GHIP_TRY(hipEventElapsedTime(&ms, g->ev[q], g->ev[q + 1]), "elapsed");
    tot += ms;
  }
  if (launches) *launches = (int64_t)(g->ev_used / 2);
  if (total_ms) *total_ms = tot;
  g->ev_used = 0;
  return MHC_OK;
}

}  // extern "C"
