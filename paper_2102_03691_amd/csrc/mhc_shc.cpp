// Host side of the spectral-heat-current entry points (mhc_shc_*, include/mhc.h).
//
// Per pushed block of at most T steps: the block's virials go into the ring
// of past virials and its velocities into a staging copy, both with
// direction-major dof columns (nu * Np + i), then the virial-velocity
// products of the block's steps against the last n_lags origins are formed
// and added to the float64 sums of each motion direction.  No arithmetic of
// the method runs here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mhc.h"
#include "mhc_common.h"

using namespace mhc;

struct mhc_shc {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  mhc_status sticky = MHC_OK;
  int64_t N = 0, N3 = 0, Np = 0, ld = 0;
  int n_lags = 0, T = 0;
  int64_t ring_len = 0;
  int64_t dk = 0;
  int n_kcs = 0;                       // dof ranges per direction segment
  int64_t cost = 0;                    // estimated product-launch time of a full block, in chunk-times
  int64_t S = 0;                       // samples pushed since the last reset
  std::vector<void*> allocs;
  float* ring = nullptr;               // [ring_len][3 mu][ld = 3 Np]
  float* vt = nullptr;                 // [T][ld] velocities, direction-major
  float* sv = nullptr;                 // host-input staging [T][N][3]
  float* sW = nullptr;                 // [T][N][9]
  // host pushes of several blocks: a second staging set and a copy stream,
  // so that one block's PCIe copy overlaps the previous block's kernels
  float* sv2 = nullptr;
  float* sW2 = nullptr;
  hipStream_t copy_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_copied[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
  double* part = nullptr;              // [3 n_kcs][T/64][n_lags_pad][3]
  double* ksum = nullptr;              // [3 nu][n_lags][3 mu] x 2 (sum, compensation)
  double* kout = nullptr;              // [n_lags][3] then [n_lags][3][3] read-out
  double* omega = nullptr;             // spectrum frequencies (grown on demand)
  double* kw = nullptr;                // [n_omega][3]
  int omega_cap = 0;
  int timing_every = 0;                // events around every timing_every-th block (0: none)
  int64_t n_timed_seen = 0;            // blocks since timing was set
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
};

namespace {

thread_local std::string g_shc_create_error;

mhc_status sfail(mhc_shc* c, mhc_status st, const std::string& msg) {
  c->err = msg;
  return st;
}

mhc_status shc_hip_fail(mhc_shc* c, hipError_t e, const char* where) {
  (void)hipGetLastError();
  c->sticky = MHC_ERR_HIP;
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return MHC_ERR_HIP;
}

#define SHIP_TRY(call, where)                                   \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return shc_hip_fail(c, e_, (where));  \
  } while (0)

mhc_status senter(mhc_shc* c) {
  if (!c) return MHC_ERR_INVALID_ARG;
  if (c->sticky != MHC_OK) return c->sticky;
  c->err.clear();
  if (hipSetDevice(c->device) != hipSuccess) return shc_hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
  return MHC_OK;
}

mhc_status salloc(mhc_shc* c, size_t bytes, void** out, const char* what) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return sfail(c, MHC_ERR_OOM, std::string("device allocation failed: ") + what);
  }
  c->allocs.push_back(p);
  *out = p;
  return MHC_OK;
}

void sfree(mhc_shc* c) {
  if (c->copy_stream) {
    (void)hipStreamSynchronize(c->copy_stream);
    (void)hipStreamDestroy(c->copy_stream);
    c->copy_stream = nullptr;
  }
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  for (auto e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  for (hipEvent_t* e : {&c->ev_start, &c->ev_copied[0], &c->ev_copied[1], &c->ev_free[0], &c->ev_free[1]})
    if (*e) {
      (void)hipEventDestroy(*e);
      *e = nullptr;
    }
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  c->stream = nullptr;
}

// lags of the product work-groups are padded to 128
int lags_pad(int n) { return (n + 127) / 128 * 128; }

// One block of t_count <= T steps whose inputs are device pointers.
mhc_status shc_block(mhc_shc* c, const float* v, const float* W, int t_count) {
  SHIP_TRY(launch_shc_ring(c->stream, W, v, t_count, c->N, c->Np, c->ring, c->ring_len, c->ld, c->S, c->vt),
           "virial ring");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing_every > 0 && c->n_timed_seen++ % c->timing_every == 0) {
    while (c->ev_used + 2 > c->ev.size()) {
      hipEvent_t e;
      SHIP_TRY(hipEventCreate(&e), "event create");
      c->ev.push_back(e);
    }
    e0 = c->ev[c->ev_used];
    e1 = c->ev[c->ev_used + 1];
    c->ev_used += 2;
    SHIP_TRY(hipEventRecord(e0, c->stream), "event record");
  }
  SHIP_TRY(launch_shc_products(c->stream, c->vt, c->ring, c->ring_len, c->ld, c->N, c->Np, t_count, c->S,
                               c->n_lags, c->dk, c->n_kcs, c->part),
           "virial-velocity products");
  if (e1) SHIP_TRY(hipEventRecord(e1, c->stream), "event record");
  SHIP_TRY(launch_shc_accum(c->stream, c->part, t_count, c->n_lags, c->n_kcs, c->ksum, c->ksum + 9 * c->n_lags),
           "partial sums");
  c->S += t_count;
  return MHC_OK;
}

}  // namespace

extern "C" {

mhc_status mhc_shc_create(int device, void* hip_stream, int64_t n_atoms, int32_t n_lags, int32_t t_block,
                          mhc_shc** out) {
  if (!out) return MHC_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_atoms < 1 || n_atoms > (int64_t(1) << 26) || n_lags < 1 || n_lags > 4096 || t_block < 64 ||
      t_block > 1024 || t_block % 64)
    return MHC_ERR_INVALID_ARG;
  mhc_shc* c = new (std::nothrow) mhc_shc();
  if (!c) return MHC_ERR_OOM;
  c->device = device;
  auto bail = [&](mhc_status st, const char* what) {
    g_shc_create_error = what;
    sfree(c);
    delete c;
    return st;
  };
  if (hipSetDevice(device) != hipSuccess) return bail(MHC_ERR_HIP, "hipSetDevice");
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) return bail(MHC_ERR_HIP, "hipStreamCreate");
    c->own_stream = true;
  }
  int n_cu = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) n_cu = std::max(1, prop.multiProcessorCount);
  c->N = n_atoms;
  c->N3 = 3 * n_atoms;
  c->Np = (n_atoms + 31) / 32 * 32;
  c->ld = 3 * c->Np;
  c->n_lags = n_lags;
  c->T = t_block;
  c->ring_len = (int64_t)n_lags - 1 + t_block;
  // Split each direction's N dofs into n_kcs ranges of dk.  A product
  // work-group (64 steps x 128 lags x one virial component) takes half a CU
  // (half its registers and LDS), so a full block takes
  // ceil(3 n_kcs tiles / (2 n_cu)) rounds of dk / 32 chunks each, plus a
  // fixed cost per work-group (staging, the diagonal sums: about two chunks);
  // pick the split with the least such time, the fewer work-groups on a tie.
  const int64_t tiles = (int64_t)3 * (t_block / 64) * (lags_pad(n_lags) / 128);
  const int64_t max_kc = c->Np / 32;
  int64_t best = -1, best_cost = 0;
  for (int64_t kc = 1; kc <= max_kc; ++kc) {
    const int64_t dk = ((c->N + kc - 1) / kc + 31) / 32 * 32;
    const int64_t n = (c->N + dk - 1) / dk;
    if (n != kc) continue;
    const int64_t rounds = (3 * n * tiles + 2 * n_cu - 1) / (2 * n_cu);
    const int64_t cost = rounds * (dk / 32 + 2);
    if (best < 0 || cost < best_cost) {
      best = kc;
      best_cost = cost;
    }
  }
  c->dk = ((c->N + best - 1) / best + 31) / 32 * 32;
  c->n_kcs = (int)((c->N + c->dk - 1) / c->dk);
  c->cost = best_cost;
  void *pr, *pvt, *pv, *pW, *pp, *ps, *po;
  const size_t ring_bytes = (size_t)c->ring_len * 3 * c->ld * 4;
  const size_t vt_bytes = (size_t)t_block * c->ld * 4;
  if (salloc(c, ring_bytes, &pr, "virial ring") || salloc(c, vt_bytes, &pvt, "velocity rows") ||
      salloc(c, (size_t)t_block * c->N3 * 4, &pv, "velocity staging") ||
      salloc(c, (size_t)t_block * c->N3 * 3 * 4, &pW, "virial staging") ||
      salloc(c, (size_t)3 * c->n_kcs * (t_block / 64) * lags_pad(n_lags) * 3 * 8, &pp, "partials") ||
      salloc(c, (size_t)n_lags * 9 * 2 * 8, &ps, "sums") || salloc(c, (size_t)n_lags * 12 * 8, &po, "read-out"))
    return bail(MHC_ERR_OOM, "device allocation failed");
  c->ring = static_cast<float*>(pr);
  c->vt = static_cast<float*>(pvt);
  c->sv = static_cast<float*>(pv);
  c->sW = static_cast<float*>(pW);
  c->part = static_cast<double*>(pp);
  c->ksum = static_cast<double*>(ps);
  c->kout = static_cast<double*>(po);
  // the pad columns of the ring and the velocity rows stay zero for good
  if (hipMemsetAsync(c->ring, 0, ring_bytes, c->stream) != hipSuccess ||
      hipMemsetAsync(c->vt, 0, vt_bytes, c->stream) != hipSuccess ||
      hipMemsetAsync(c->ksum, 0, (size_t)n_lags * 9 * 2 * 8, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(MHC_ERR_HIP, "initial clear");
  *out = c;
  return MHC_OK;
}

mhc_status mhc_shc_destroy(mhc_shc* c) {
  if (!c) return MHC_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  sfree(c);
  delete c;
  return MHC_OK;
}

const char* mhc_shc_last_error(const mhc_shc* c) { return c ? c->err.c_str() : g_shc_create_error.c_str(); }

// Second staging set, copy stream and events of host pushes, created on the
// first push of several blocks; each piece once.
static mhc_status shc_host_staging(mhc_shc* c) {
  if (c->copy_stream) return MHC_OK;
  mhc_status st;
  void* p = nullptr;
  if (!c->sv2) {
    if ((st = salloc(c, (size_t)c->T * c->N3 * 4, &p, "velocity staging 2"))) return st;
    c->sv2 = static_cast<float*>(p);
  }
  if (!c->sW2) {
    if ((st = salloc(c, (size_t)c->T * c->N3 * 12, &p, "virial staging 2"))) return st;
    c->sW2 = static_cast<float*>(p);
  }
  for (hipEvent_t* e : {&c->ev_start, &c->ev_copied[0], &c->ev_copied[1], &c->ev_free[0], &c->ev_free[1]})
    if (!*e) SHIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming), "event create");
  hipStream_t cs = nullptr;
  SHIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "copy stream");
  c->copy_stream = cs;
  return MHC_OK;
}

mhc_status mhc_shc_push(mhc_shc* c, int32_t n_steps, const float* v, const float* W, int on_device) {
  mhc_status st = senter(c);
  if (st) return st;
  if (n_steps < 0 || (on_device != 0 && on_device != 1)) return sfail(c, MHC_ERR_INVALID_ARG, "bad arguments");
  if (n_steps == 0) return MHC_OK;
  if (!v || !W) return sfail(c, MHC_ERR_INVALID_ARG, "NULL input");
  if (on_device) {
    for (int32_t s0 = 0; s0 < n_steps; s0 += c->T) {
      const int tc = std::min<int32_t>(c->T, n_steps - s0);
      if ((st = shc_block(c, v + (int64_t)s0 * c->N3, W + (int64_t)s0 * c->N3 * 3, tc))) return st;
    }
    return MHC_OK;
  }
  if (n_steps <= c->T) {
    // one block: copy and kernels in order on the stream
    SHIP_TRY(hipMemcpyAsync(c->sv, v, (size_t)n_steps * c->N3 * 4, hipMemcpyHostToDevice, c->stream), "copy v");
    SHIP_TRY(hipMemcpyAsync(c->sW, W, (size_t)n_steps * c->N3 * 12, hipMemcpyHostToDevice, c->stream), "copy W");
    if ((st = shc_block(c, c->sv, c->sW, n_steps))) return st;
    SHIP_TRY(hipStreamSynchronize(c->stream), "push sync");
    return MHC_OK;
  }
  // Several blocks: block k is copied into staging set k % 2 on the copy
  // stream while block k - 1 runs; the copy stream first waits for the work
  // already queued on the stream, then each copy for the block that last
  // read its set.
  if ((st = shc_host_staging(c))) return st;
  SHIP_TRY(hipEventRecord(c->ev_start, c->stream), "event record");
  SHIP_TRY(hipStreamWaitEvent(c->copy_stream, c->ev_start, 0), "stream wait");
  float* const sv[2] = {c->sv, c->sv2};
  float* const sW[2] = {c->sW, c->sW2};
  int k = 0;
  for (int32_t s0 = 0; s0 < n_steps; s0 += c->T, ++k) {
    const int tc = std::min<int32_t>(c->T, n_steps - s0);
    const int b = k & 1;
    if (k >= 2) SHIP_TRY(hipStreamWaitEvent(c->copy_stream, c->ev_free[b], 0), "stream wait");
    SHIP_TRY(hipMemcpyAsync(sv[b], v + (int64_t)s0 * c->N3, (size_t)tc * c->N3 * 4, hipMemcpyHostToDevice,
                            c->copy_stream), "copy v");
    SHIP_TRY(hipMemcpyAsync(sW[b], W + (int64_t)s0 * c->N3 * 3, (size_t)tc * c->N3 * 12, hipMemcpyHostToDevice,
                            c->copy_stream), "copy W");
    SHIP_TRY(hipEventRecord(c->ev_copied[b], c->copy_stream), "event record");
    SHIP_TRY(hipStreamWaitEvent(c->stream, c->ev_copied[b], 0), "stream wait");
    if ((st = shc_block(c, sv[b], sW[b], tc))) {
      (void)hipStreamSynchronize(c->copy_stream);     // the caller may reuse v and W on return
      return st;
    }
    SHIP_TRY(hipEventRecord(c->ev_free[b], c->stream), "event record");
  }
  // every copy precedes a kernel the stream waited for
  SHIP_TRY(hipStreamSynchronize(c->stream), "push sync");
  return MHC_OK;
}

static mhc_status shc_read(mhc_shc* c, double* K, int64_t* n_samples, int split) {
  mhc_status st = senter(c);
  if (st) return st;
  if (!K) return sfail(c, MHC_ERR_INVALID_ARG, "NULL output");
  const size_t n = (size_t)c->n_lags * 3;
  SHIP_TRY(launch_shc_finish(c->stream, c->ksum, c->ksum + 9 * c->n_lags, c->n_lags, c->S, c->kout, c->kout + n),
           "finish");
  SHIP_TRY(hipMemcpyAsync(K, c->kout + (split ? n : 0), (split ? 3 : 1) * n * 8, hipMemcpyDeviceToHost, c->stream),
           "copy K");
  SHIP_TRY(hipStreamSynchronize(c->stream), "read sync");
  if (n_samples) *n_samples = c->S;
  return MHC_OK;
}

mhc_status mhc_shc_read(mhc_shc* c, double* K, int64_t* n_samples) { return shc_read(c, K, n_samples, 0); }

mhc_status mhc_shc_read_dir(mhc_shc* c, double* K, int64_t* n_samples) { return shc_read(c, K, n_samples, 1); }

static mhc_status shc_spectrum(mhc_shc* c, int32_t n_omega, const double* omega, double dt, int32_t window,
                               double* Kw, int split) {
  mhc_status st = senter(c);
  if (st) return st;
  if (n_omega < 1 || n_omega > (1 << 24) || !omega || !Kw || !(std::isfinite(dt) && dt > 0.0) ||
      (window != 0 && window != 1))
    return sfail(c, MHC_ERR_INVALID_ARG, "bad arguments");
  for (int32_t w = 0; w < n_omega; ++w)
    if (!std::isfinite(omega[w])) return sfail(c, MHC_ERR_INVALID_ARG, "non-finite frequency");
  if (n_omega > c->omega_cap) {
    void *po, *pk;
    if ((st = salloc(c, (size_t)n_omega * 8, &po, "frequencies"))) return st;
    if ((st = salloc(c, (size_t)n_omega * 9 * 8, &pk, "spectrum"))) return st;
    c->omega = static_cast<double*>(po);
    c->kw = static_cast<double*>(pk);
    c->omega_cap = n_omega;
  }
  SHIP_TRY(hipMemcpyAsync(c->omega, omega, (size_t)n_omega * 8, hipMemcpyHostToDevice, c->stream), "copy omega");
  const size_t n = (size_t)c->n_lags * 3;
  const int nc = split ? 9 : 3;
  SHIP_TRY(launch_shc_finish(c->stream, c->ksum, c->ksum + 9 * c->n_lags, c->n_lags, c->S, c->kout, c->kout + n),
           "finish");
  SHIP_TRY(launch_shc_spectrum(c->stream, c->kout + (split ? n : 0), c->n_lags, nc, c->omega, n_omega, dt, window,
                               c->kw),
           "spectrum");
  SHIP_TRY(hipMemcpyAsync(Kw, c->kw, (size_t)n_omega * nc * 8, hipMemcpyDeviceToHost, c->stream), "copy spectrum");
  SHIP_TRY(hipStreamSynchronize(c->stream), "spectrum sync");
  return MHC_OK;
}

mhc_status mhc_shc_spectrum(mhc_shc* c, int32_t n_omega, const double* omega, double dt, int32_t window,
                            double* Kw) {
  return shc_spectrum(c, n_omega, omega, dt, window, Kw, 0);
}

mhc_status mhc_shc_spectrum_dir(mhc_shc* c, int32_t n_omega, const double* omega, double dt, int32_t window,
                                double* Kw) {
  return shc_spectrum(c, n_omega, omega, dt, window, Kw, 1);
}

mhc_status mhc_shc_reset(mhc_shc* c) {
  mhc_status st = senter(c);
  if (st) return st;
  SHIP_TRY(hipMemsetAsync(c->ksum, 0, (size_t)c->n_lags * 9 * 2 * 8, c->stream), "clear sums");
  SHIP_TRY(hipStreamSynchronize(c->stream), "reset sync");
  c->S = 0;
  return MHC_OK;
}

// Saved state: a header, the float64 sums and compensations, then the virial
// ring (the history later blocks correlate against).
namespace {
struct ShcStateHeader {
  uint64_t magic;
  int64_t N, ring_len, ld, S;
  int32_t n_lags, T;
};
constexpr uint64_t kShcMagic = 0x4D48435348435331ull;  // "MHCSHCS1"
size_t shc_state_bytes(const mhc_shc* c) {
  return sizeof(ShcStateHeader) + (size_t)c->n_lags * 9 * 2 * 8 + (size_t)c->ring_len * 3 * c->ld * 4;
}
}  // namespace

mhc_status mhc_shc_save_state(mhc_shc* c, void* buf, size_t* len) {
  mhc_status st = senter(c);
  if (st) return st;
  if (!len) return sfail(c, MHC_ERR_INVALID_ARG, "NULL len");
  const size_t need = shc_state_bytes(c);
  if (!buf) {
    *len = need;
    return MHC_OK;
  }
  if (*len < need) return sfail(c, MHC_ERR_INVALID_ARG, "buffer too small");
  ShcStateHeader hd{kShcMagic, c->N, c->ring_len, c->ld, c->S, c->n_lags, c->T};
  char* p = static_cast<char*>(buf);
  std::memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  const size_t ks = (size_t)c->n_lags * 9 * 2 * 8;
  SHIP_TRY(hipMemcpyAsync(p, c->ksum, ks, hipMemcpyDeviceToHost, c->stream), "save sums");
  p += ks;
  SHIP_TRY(hipMemcpyAsync(p, c->ring, (size_t)c->ring_len * 3 * c->ld * 4, hipMemcpyDeviceToHost, c->stream),
           "save ring");
  SHIP_TRY(hipStreamSynchronize(c->stream), "save sync");
  *len = need;
  return MHC_OK;
}

mhc_status mhc_shc_load_state(mhc_shc* c, const void* buf, size_t len) {
  mhc_status st = senter(c);
  if (st) return st;
  if (!buf || len != shc_state_bytes(c)) return sfail(c, MHC_ERR_INVALID_ARG, "state size mismatch");
  ShcStateHeader hd;
  std::memcpy(&hd, buf, sizeof hd);
  if (hd.magic != kShcMagic || hd.N != c->N || hd.ring_len != c->ring_len || hd.ld != c->ld ||
      hd.n_lags != c->n_lags || hd.T != c->T || hd.S < 0)
    return sfail(c, MHC_ERR_INVALID_ARG, "state from a different configuration");
  const char* p = static_cast<const char*>(buf) + sizeof hd;
  const size_t ks = (size_t)c->n_lags * 9 * 2 * 8;
  SHIP_TRY(hipMemcpyAsync(c->ksum, p, ks, hipMemcpyHostToDevice, c->stream), "load sums");
  p += ks;
  SHIP_TRY(hipMemcpyAsync(c->ring, p, (size_t)c->ring_len * 3 * c->ld * 4, hipMemcpyHostToDevice, c->stream),
           "load ring");
  SHIP_TRY(hipStreamSynchronize(c->stream), "load sync");
  c->S = hd.S;
  return MHC_OK;
}

mhc_status mhc_shc_synchronize(mhc_shc* c) {
  mhc_status st = senter(c);
  if (st) return st;
  SHIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
  return MHC_OK;
}

mhc_status mhc_shc_set_timing(mhc_shc* c, int enable) {
  mhc_status st = senter(c);
  if (st) return st;
  if (enable < 0) return sfail(c, MHC_ERR_INVALID_ARG, "enable is 0 (off) or k >= 1 (every k-th block)");
  c->timing_every = enable;
  c->n_timed_seen = 0;
  c->ev_used = 0;
  return MHC_OK;
}

mhc_status mhc_shc_kernel_timing(mhc_shc* c, int64_t* launches, double* total_ms) {
  mhc_status st = senter(c);
  if (st) return st;
  if (!launches || !total_ms) return sfail(c, MHC_ERR_INVALID_ARG, "NULL output");
  SHIP_TRY(hipStreamSynchronize(c->stream), "timing sync");
  double tot = 0.0;
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.f;
    SHIP_TRY(hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]), "elapsed");
    tot += ms;
  }
  *launches = (int64_t)(c->ev_used / 2);
  *total_ms = tot;
  c->ev_used = 0;
  return MHC_OK;
}

}  // extern "C"

// ------------------------------------------------------------ grouped pushes
// Several SHC contexts advanced together.  Systems whose own product launch
// is short (at most SHC_FUSE_COST chunk-times: launch overhead and a partly
// idle GPU dominate) are fused: the ring, product and accumulation kernels
// of all of them concatenated into one grid each, driven by a table of
// per-system descriptors.  Larger systems fill the GPU by themselves and
// run their own launches, in order: fused into a long grid their work-groups
// would start staggered instead of together, and the ones that share ring
// rows would no longer read them at the same time (measured: 16 systems of
// 0.6k..8k atoms fused 2.97 ms per block against 2.13 ms one by one; 64
// systems of 0.2k..1k atoms 1.91 against 2.56 ms).  Each system's arithmetic
// and summation order are those of its own push, so the results are the
// same bits.  The descriptors of a block go through a ring of pinned
// host slots and device slots; a host slot is refilled only after the event
// recorded behind its previous copy (device slots are reused in stream
// order, after the kernels that read them).
struct mhc_shc_group {
  std::vector<mhc_shc*> sys;
  int device = 0;
  hipStream_t stream = nullptr;
  int T = 0;
  std::string err;
  mhc_status sticky = MHC_OK;
  static constexpr int SLOTS = 64;
  ShcBlockDesc* h_desc = nullptr;   // pinned [SLOTS][n]
  ShcBlockDesc* d_desc = nullptr;   // device [SLOTS][n]
  hipEvent_t ev[SLOTS] = {};
  bool ev_pending[SLOTS] = {};
  int64_t next = 0;
};

namespace {

thread_local std::string g_shc_group_create_error;

mhc_status gfail(mhc_shc_group* g, mhc_status st, const std::string& msg) {
  g->err = msg;
  if (st == MHC_ERR_HIP) g->sticky = MHC_ERR_HIP;
  return st;
}

#define GHIP_TRY(call, where)                                                                   \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      (void)hipGetLastError();                                                                  \
      return gfail(g, MHC_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e_));          \
    }                                                                                           \
  } while (0)

void gfree(mhc_shc_group* g) {
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  for (hipEvent_t& e : g->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  if (g->h_desc) (void)hipHostFree(g->h_desc);
  if (g->d_desc) (void)hipFree(g->d_desc);
  g->h_desc = nullptr;
  g->d_desc = nullptr;
}

constexpr int64_t SHC_FUSE_COST = 8;

// One block of t_count steps for every system; v[q], W[q] are device pointers
// to system q's block.
mhc_status group_block(mhc_shc_group* g, const float* const* v, const float* const* W, int t_count) {
  const int n_all = (int)g->sys.size();
  // the large systems: their own launches, as a single push makes them
  for (int q = 0; q < n_all; ++q) {
    mhc_shc* c = g->sys[q];
    if (c->cost <= SHC_FUSE_COST) continue;
    mhc_status st = shc_block(c, v[q], W[q], t_count);
    if (st) return gfail(g, st, "system " + std::to_string(q) + ": " + c->err);
  }
  std::vector<int> fused;
  for (int q = 0; q < n_all; ++q)
    if (g->sys[q]->cost <= SHC_FUSE_COST) fused.push_back(q);
  const int n = (int)fused.size();
  if (n == 0) return MHC_OK;
  const int slot = (int)(g->next++ % mhc_shc_group::SLOTS);
  if (g->ev_pending[slot]) GHIP_TRY(hipEventSynchronize(g->ev[slot]), "descriptor slot wait");
  ShcBlockDesc* h = g->h_desc + (int64_t)slot * n_all;
  int64_t rb = 0, wg = 0, ab = 0;
  for (int k = 0; k < n; ++k) {
    const int q = fused[k];
    const mhc_shc* c = g->sys[q];
    ShcBlockDesc& d = h[k];
    d = ShcBlockDesc{};
    d.W = W[q];
    d.v = v[q];
    d.ring = c->ring;
    d.vt = c->vt;
    d.part = c->part;
    d.ksum = c->ksum;
    d.kcomp = c->ksum + 9 * c->n_lags;
    d.N = c->N;
    d.Np = c->Np;
    d.ring_len = c->ring_len;
    d.ld = c->ld;
    d.s0 = c->S;
    d.dk = c->dk;
    d.t_count = t_count;
    d.n_kcs = c->n_kcs;
    d.n_ttiles = (t_count + 63) / 64;
    d.n_lags = c->n_lags;
    d.n_lags_pad = lags_pad(c->n_lags);
    d.ring_blk0 = rb;
    d.gram_wg0 = wg;
    d.acc_blk0 = ab;
    rb += (c->N + 255) / 256;
    wg += shc_gram_wgs(t_count, c->n_lags, c->n_kcs);
    ab += shc_accum_blocks(c->n_lags);
  }
  ShcBlockDesc* d = g->d_desc + (int64_t)slot * n_all;
  GHIP_TRY(hipMemcpyAsync(d, h, sizeof(ShcBlockDesc) * n, hipMemcpyHostToDevice, g->stream), "descriptor copy");
  GHIP_TRY(hipEventRecord(g->ev[slot], g->stream), "event record");
  g->ev_pending[slot] = true;
  GHIP_TRY(launch_shc_ring_group(g->stream, d, n, rb, t_count), "virial rings");
  GHIP_TRY(launch_shc_gram_group(g->stream, d, n, wg), "virial-velocity products");
  GHIP_TRY(launch_shc_accum_group(g->stream, d, n, ab), "partial sums");
  for (int q : fused) g->sys[q]->S += t_count;
  return MHC_OK;
}

}  // namespace

extern "C" {

mhc_status mhc_shc_group_create(mhc_shc* const* systems, int32_t n, mhc_shc_group** out) {
  if (!out) return MHC_ERR_INVALID_ARG;
  *out = nullptr;
  auto bad = [](mhc_status st, const char* why) {
    g_shc_group_create_error = why;
    return st;
  };
  if (!systems || n < 1 || n > 4096) return bad(MHC_ERR_INVALID_ARG, "need 1 to 4096 systems");
  for (int32_t q = 0; q < n; ++q) {
    if (!systems[q]) return bad(MHC_ERR_INVALID_ARG, "NULL system");
    if (systems[q]->sticky != MHC_OK) return bad(systems[q]->sticky, "a system has a sticky error");
    for (int32_t r = 0; r < q; ++r)
      if (systems[r] == systems[q]) return bad(MHC_ERR_INVALID_ARG, "a system appears twice");
    if (systems[q]->device != systems[0]->device || systems[q]->stream != systems[0]->stream ||
        systems[q]->T != systems[0]->T)
      return bad(MHC_ERR_INVALID_ARG, "the systems must share the device, the stream and t_block");
  }
  mhc_shc_group* g = new (std::nothrow) mhc_shc_group();
  if (!g) return bad(MHC_ERR_OOM, "host allocation failed");
  g->sys.assign(systems, systems + n);
  g->device = systems[0]->device;
  g->stream = systems[0]->stream;
  g->T = systems[0]->T;
  auto bail = [&](mhc_status st, const char* why) {
    g_shc_group_create_error = why;
    gfree(g);
    delete g;
    return st;
  };
  if (hipSetDevice(g->device) != hipSuccess) return bail(MHC_ERR_HIP, "hipSetDevice");
  const size_t bytes = sizeof(ShcBlockDesc) * mhc_shc_group::SLOTS * (size_t)n;
  if (hipHostMalloc((void**)&g->h_desc, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    g->h_desc = nullptr;
    return bail(MHC_ERR_OOM, "pinned descriptor allocation failed");
  }
  if (hipMalloc((void**)&g->d_desc, bytes) != hipSuccess) {
    (void)hipGetLastError();
    g->d_desc = nullptr;
    return bail(MHC_ERR_OOM, "device descriptor allocation failed");
  }
  for (hipEvent_t& e : g->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      e = nullptr;
      return bail(MHC_ERR_HIP, "event create");
    }
  *out = g;
  return MHC_OK;
}

mhc_status mhc_shc_group_destroy(mhc_shc_group* g) {
  if (!g) return MHC_OK;
  (void)hipSetDevice(g->device);
  gfree(g);
  delete g;
  return MHC_OK;
}

const char* mhc_shc_group_last_error(const mhc_shc_group* g) {
  return g ? g->err.c_str() : g_shc_group_create_error.c_str();
}

mhc_status mhc_shc_group_push(mhc_shc_group* g, int32_t n_steps, const float* const* v, const float* const* W,
                              int on_device) {
  if (!g) return MHC_ERR_INVALID_ARG;
  if (g->sticky != MHC_OK) return g->sticky;
  g->err.clear();
  if (n_steps < 0 || (on_device != 0 && on_device != 1)) return gfail(g, MHC_ERR_INVALID_ARG, "bad arguments");
  if (n_steps == 0) return MHC_OK;
  if (!v || !W) return gfail(g, MHC_ERR_INVALID_ARG, "NULL input arrays");
  const int n = (int)g->sys.size();
  for (int q = 0; q < n; ++q) {
    if (!v[q] || !W[q]) return gfail(g, MHC_ERR_INVALID_ARG, "NULL input of system " + std::to_string(q));
    if (g->sys[q]->sticky != MHC_OK)
      return gfail(g, g->sys[q]->sticky, "system " + std::to_string(q) + " has a sticky error");
  }
  GHIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  std::vector<const float*> bv(n), bW(n);
  for (int32_t s0 = 0; s0 < n_steps; s0 += g->T) {
    const int tc = std::min<int32_t>(g->T, n_steps - s0);
    for (int q = 0; q < n; ++q) {
      mhc_shc* c = g->sys[q];
      const float* pv = v[q] + (int64_t)s0 * c->N3;
      const float* pW = W[q] + (int64_t)s0 * c->N3 * 3;
      if (on_device) {
        bv[q] = pv;
        bW[q] = pW;
      } else {   // into the system's staging, behind the kernels that last read it
        GHIP_TRY(hipMemcpyAsync(c->sv, pv, (size_t)tc * c->N3 * 4, hipMemcpyHostToDevice, g->stream), "copy v");
        GHIP_TRY(hipMemcpyAsync(c->sW, pW, (size_t)tc * c->N3 * 12, hipMemcpyHostToDevice, g->stream), "copy W");
        bv[q] = c->sv;
        bW[q] = c->sW;
      }
    }
    mhc_status st = group_block(g, bv.data(), bW.data(), tc);
    if (st) return st;
  }
  if (!on_device) GHIP_TRY(hipStreamSynchronize(g->stream), "push sync");   // the caller may reuse v and W
  return MHC_OK;
}

}  // extern "C"
