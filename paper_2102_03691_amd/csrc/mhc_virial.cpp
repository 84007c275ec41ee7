// Host side of the per-atom virial object (mhc_virial_*, include/mhc.h):
// argument checks, device buffers, the cell grid of the neighbour search and
// the launch sequence.  Every step of the computation is a HIP kernel
// (k_tersoff.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/mhc.h"
#include "mhc_tersoff.h"

using namespace mhc;

namespace {

thread_local std::string g_virial_create_error;

// 1 amu (A/fs)^2 in eV: 1.66053906660e-27 kg * 1e10 m^2/s^2 / 1.602176634e-19 J
constexpr double KE_UNIT_EV = 1.66053906660e-27 * 1e10 / 1.602176634e-19;
// Boltzmann constant in eV/K (CODATA 2018, exact)
constexpr double K_B_EV = 8.617333262e-5;

}  // namespace

struct mhc_virial {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  mhc_status sticky = MHC_OK;

  int64_t N = 0;
  double box[3] = {0, 0, 0};
  TersoffParams tp{};
  double rc = 0.0;        // neighbour cutoff: R + D + skin
  int max_nb = 0;
  CellGrid cg{};
  bool lists_ok = false;

  std::vector<void*> allocs;
  double* d_mass = nullptr;
  NeighborBufs nb{};
  double *d_dd = nullptr, *d_U = nullptr;
  double* d_F = nullptr;  // forces of the molecular dynamics (mhc_virial_md)
  double* d_thermo = nullptr;   // Nose-Hoover state [4] (mhc_virial_md_nvt)
  double* d_kepart = nullptr;   // kinetic-energy partials (per 64 atoms, or per gather work-group)
  // Bond lists of the molecular dynamics when the lists carry a skin: the
  // pairs inside R + D + delta (delta = bond_skin, the smaller of the skin and
  // 0.5 A), rebuilt on the device whenever an atom has moved more than
  // delta / 2 since their last build (so they hold every pair inside R + D),
  // with max_b slots (the largest count at the last list build plus 2) and
  // lpa_b lanes per atom (compact: fewer lanes than the lists need).
  // bb.flags[0..2] accumulate over one mhc_virial_md call; bb.need = flags + 8.
  BondBufs bb{};
  double bond_skin = 0.0;
  int max_b = 0, lpa_b = 4;
  bool compact = false;
  int lpa = 4;            // lanes per atom of the evaluation kernels (from the largest neighbour count)

  int timing_every = 0;    // events around every timing_every-th evaluation (0: none)
  int64_t n_evals = 0;     // evaluations since timing was set
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
};

namespace {

mhc_status vfail(mhc_virial* v, mhc_status st, const std::string& msg) {
  if (v) {
    v->err = msg;
    if (st == MHC_ERR_HIP) v->sticky = MHC_ERR_HIP;
  }
  return st;
}

#define VHIP_TRY(call, where)                                                               \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return vfail(v, MHC_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Three events around the site and gather kernels of every timing_every-th
// evaluation (none for the others, or with timing off).
mhc_status timing_events(mhc_virial* v, hipEvent_t e[3]) {
  if (v->timing_every <= 0 || v->n_evals++ % v->timing_every != 0) return MHC_OK;
  if (v->ev_used + 3 > v->ev.size())
    for (int q = 0; q < 3; ++q) {
      hipEvent_t ev;
      VHIP_TRY(hipEventCreate(&ev), "event create");
      v->ev.push_back(ev);
    }
  for (int q = 0; q < 3; ++q) e[q] = v->ev[v->ev_used + q];
  v->ev_used += 3;
  return MHC_OK;
}

// Squared pair distance beyond which the site kernel writes zero partials
// (R + D), widened by one part in 10^12 so that rounding in the gather
// kernel's own distance never drops a pair the site kernel kept.
double rcut2_of(const mhc_virial* v) {
  const double rc = (v->tp.R + v->tp.D) * (1.0 + 1e-12);
  return rc * rc;
}

// Bond slots and lanes of the molecular dynamics from the largest count of
// pairs inside R + D + bond_skin at the list build (found), and whether it
// uses bond lists at all (only with skin lists, and with fewer lanes).
void plan_bonds(mhc_virial* v, int found) {
  v->compact = false;
  if (!(v->rc > (v->tp.R + v->tp.D) * (1.0 + 1e-9))) return;   // no skin: the lists are the bonds
  v->max_b = std::min(v->max_nb, found + 2);
  v->lpa_b = tersoff_lanes(v->max_b);
  v->compact = v->lpa_b < v->lpa;
}

mhc_status venter(mhc_virial* v) {
  if (!v) return MHC_ERR_INVALID_ARG;
  if (v->sticky != MHC_OK) return v->sticky;
  v->err.clear();
  return MHC_OK;
}

void vfree(mhc_virial* v) {
  for (void* p : v->allocs) (void)hipFree(p);
  v->allocs.clear();
}

template <class T>
bool valloc(mhc_virial* v, size_t count, T** out) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  v->allocs.push_back(p);
  *out = reinterpret_cast<T*>(p);
  return true;
}

bool finite_params(const mhc_tersoff_params* p) {
  const double x[] = {p->A, p->B, p->lambda1, p->lambda2, p->lambda3, p->beta, p->n, p->c, p->d, p->h, p->gamma,
                      p->R, p->D};
  for (double a : x)
    if (!std::isfinite(a)) return false;
  return true;
}

// Cells per axis: floor(box / cutoff) (so a cell is at least the cutoff wide),
// 1 where that is below 3; the total kept below 8N + 64 by halving the
// largest count (cells only get wider).
CellGrid make_grid(const double box[3], double rc, int64_t N) {
  CellGrid g{};
  for (int a = 0; a < 3; ++a) {
    g.box[a] = box[a];
    g.ibox[a] = 1.0 / box[a];
    const double c = std::floor(box[a] / rc);
    int n = c > 1024.0 ? 1024 : (int)c;
    g.nc[a] = n < 3 ? 1 : n;
  }
  const int64_t cap = 8 * N + 64;
  while ((int64_t)g.nc[0] * g.nc[1] * g.nc[2] > cap) {
    int a = 0;
    for (int b = 1; b < 3; ++b)
      if (g.nc[b] > g.nc[a]) a = b;
    const int n = g.nc[a] / 2;
    g.nc[a] = n < 3 ? 1 : n;
  }
  return g;
}

}  // namespace

extern "C" {

mhc_status mhc_virial_create(int device, void* hip_stream, int64_t n_atoms, const double* mass_amu,
                             const double* box, const mhc_tersoff_params* params, int32_t max_neighbors, double skin,
                             mhc_virial** out) {
  g_virial_create_error.clear();
  auto bad = [](const char* msg) {
    g_virial_create_error = msg;
    return MHC_ERR_INVALID_ARG;
  };
  if (!out) return bad("out is NULL");
  *out = nullptr;
  if (n_atoms < 1 || n_atoms > (int64_t(1) << 26)) return bad("n_atoms must be in [1, 2^26]");
  if (!mass_amu || !box || !params) return bad("NULL mass, box or parameters");
  if (max_neighbors < 1 || max_neighbors > 64) return bad("max_neighbors must be in [1, 64]");
  if (!std::isfinite(skin) || skin < 0.0) return bad("skin must be finite and >= 0");
  if (!finite_params(params) || params->reserved != 0) return bad("parameters must be finite, reserved zero");
  if (params->m != 1 && params->m != 3) return bad("m must be 1 or 3");
  if (!(params->D > 0.0) || !(params->R > params->D)) return bad("need R > D > 0");
  if (!(params->n > 0.0) || params->beta < 0.0 || !(params->d != 0.0)) return bad("need n > 0, beta >= 0, d != 0");
  const double rc = params->R + params->D + skin;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(box[a]) || !(box[a] > 2.0 * rc)) return bad("every box edge must exceed twice R + D + skin");
  for (int64_t i = 0; i < n_atoms; ++i)
    if (!std::isfinite(mass_amu[i]) || !(mass_amu[i] > 0.0)) return bad("masses must be finite and positive");
  int nd = 0;
  hipError_t e = hipGetDeviceCount(&nd);
  if (e != hipSuccess || nd == 0) {
    (void)hipGetLastError();
    g_virial_create_error = "no HIP device";
    return MHC_ERR_HIP;
  }
  if (device < 0 || device >= nd) return bad("device index out of range");
  if ((e = hipSetDevice(device)) != hipSuccess) {
    g_virial_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
    return MHC_ERR_HIP;
  }
  mhc_virial* v = new (std::nothrow) mhc_virial();
  if (!v) {
    g_virial_create_error = "host allocation failed";
    return MHC_ERR_OOM;
  }
  v->device = device;
  v->N = n_atoms;
  for (int a = 0; a < 3; ++a) v->box[a] = box[a];
  v->rc = rc;
  v->max_nb = max_neighbors;
  v->cg = make_grid(box, rc, n_atoms);
  const mhc_tersoff_params& p = *params;
  v->tp = TersoffParams{p.A, p.B, p.lambda1, p.lambda2, std::pow(p.lambda3, (double)p.m), p.beta, p.n, p.c * p.c,
                        p.d * p.d, (p.c * p.c) / (p.d * p.d), p.h, p.gamma, p.R, p.D,
                        p.gamma * ((p.c * p.c) / (p.d * p.d)), 2.0 * p.gamma * (p.c * p.c), -0.5 / p.n, p.m};
  auto cleanup = [&](mhc_status st, const char* msg) {
    vfree(v);
    if (v->own_stream) (void)hipStreamDestroy(v->stream);
    delete v;
    g_virial_create_error = msg;
    return st;
  };
  if (hip_stream) {
    v->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&v->stream) != hipSuccess) return cleanup(MHC_ERR_HIP, "hipStreamCreate failed");
    v->own_stream = true;
  }
  const int64_t N = n_atoms, MN = (int64_t)max_neighbors * N;
  const int64_t n_cells = (int64_t)v->cg.nc[0] * v->cg.nc[1] * v->cg.nc[2];
  NeighborBufs& b = v->nb;
  bool ok = valloc(v, N, &v->d_mass) && valloc(v, MN, &b.nbr) && valloc(v, MN, &b.rev) && valloc(v, N, &b.n_nb) &&
            valloc(v, N, &b.cell_of) && valloc(v, N, &b.atoms) && valloc(v, n_cells, &b.count) &&
            valloc(v, n_cells, &b.fill) && valloc(v, n_cells + 1, &b.start) &&
            valloc(v, (n_cells + 1023) / 1024, &b.tile_sums) && valloc(v, 3, &b.flags) &&
            valloc(v, 3 * MN, &v->d_dd) && valloc(v, N, &v->d_U) && valloc(v, 3 * N, &v->d_F) &&
            valloc(v, 4, &v->d_thermo) &&
            valloc(v, std::max(md_nvt_parts(N), gather_blocks(N, 64)), &v->d_kepart) &&
            valloc(v, MN, &v->bb.nbr) && valloc(v, MN, &v->bb.rev) && valloc(v, N, &v->bb.n_nb) &&
            valloc(v, N, &v->bb.mask) && valloc(v, 3 * N, &v->bb.ref) && valloc(v, 12, &v->bb.flags);
  if (!ok) return cleanup(MHC_ERR_OOM, "device allocation failed");
  v->bb.need = v->bb.flags + 8;
  v->bond_skin = std::min(rc - (p.R + p.D), 0.5);
  if (hipMemcpyAsync(v->d_mass, mass_amu, N * sizeof(double), hipMemcpyHostToDevice, v->stream) != hipSuccess ||
      hipStreamSynchronize(v->stream) != hipSuccess)
    return cleanup(MHC_ERR_HIP, "copy of the masses failed");
  *out = v;
  return MHC_OK;
}

mhc_status mhc_virial_destroy(mhc_virial* v) {
  if (!v) return MHC_OK;
  (void)hipSetDevice(v->device);
  (void)hipStreamSynchronize(v->stream);
  vfree(v);
  for (auto e : v->ev) (void)hipEventDestroy(e);
  if (v->own_stream) (void)hipStreamDestroy(v->stream);
  delete v;
  return MHC_OK;
}

const char* mhc_virial_last_error(const mhc_virial* v) {
  if (!v) return g_virial_create_error.c_str();
  return v->err.c_str();
}

mhc_status mhc_virial_neighbors(mhc_virial* v, const double* pos, int32_t* max_found) {
  mhc_status st = venter(v);
  if (st) return st;
  if (!pos) return vfail(v, MHC_ERR_INVALID_ARG, "NULL positions");
  VHIP_TRY(hipSetDevice(v->device), "hipSetDevice");
  v->lists_ok = false;
  VHIP_TRY(launch_neighbors(v->stream, pos, v->N, v->cg, v->rc, v->tp.R + v->tp.D + v->bond_skin, v->max_nb, v->nb),
           "neighbour search");
  int flags[3] = {0, 0, 0};
  VHIP_TRY(hipMemcpyAsync(flags, v->nb.flags, sizeof(flags), hipMemcpyDeviceToHost, v->stream), "read flags");
  VHIP_TRY(hipStreamSynchronize(v->stream), "neighbour search sync");
  if (max_found) *max_found = flags[0];
  if (flags[0] > v->max_nb)
    return vfail(v, MHC_ERR_INVALID_ARG,
                 "an atom has " + std::to_string(flags[0]) + " neighbours within the cutoff, more than max_neighbors = " +
                     std::to_string(v->max_nb));
  if (flags[1]) return vfail(v, MHC_ERR_INVALID_ARG, "neighbour lists are not symmetric (non-finite positions?)");
  v->lpa = tersoff_lanes(flags[0]);
  v->lists_ok = true;
  plan_bonds(v, flags[2]);
  return MHC_OK;
}

mhc_status mhc_virial_read_neighbors(mhc_virial* v, int32_t* counts, int32_t* lists) {
  mhc_status st = venter(v);
  if (st) return st;
  if (!v->lists_ok) return vfail(v, MHC_ERR_STATE, "no valid neighbour lists (call mhc_virial_neighbors)");
  VHIP_TRY(hipSetDevice(v->device), "hipSetDevice");
  const int64_t N = v->N;
  if (counts)
    VHIP_TRY(hipMemcpyAsync(counts, v->nb.n_nb, N * 4, hipMemcpyDeviceToHost, v->stream), "read counts");
  std::vector<int32_t> slot_major;
  if (lists) {
    slot_major.resize((size_t)v->max_nb * N);
    VHIP_TRY(hipMemcpyAsync(slot_major.data(), v->nb.nbr, slot_major.size() * 4, hipMemcpyDeviceToHost, v->stream),
             "read lists");
  }
  std::vector<int32_t> cnt(N);
  VHIP_TRY(hipMemcpyAsync(cnt.data(), v->nb.n_nb, N * 4, hipMemcpyDeviceToHost, v->stream), "read counts");
  VHIP_TRY(hipStreamSynchronize(v->stream), "read sync");
  if (lists) {
    for (int64_t i = 0; i < N; ++i)
      for (int s = 0; s < v->max_nb; ++s)
        lists[i * v->max_nb + s] = s < cnt[i] ? slot_major[(size_t)s * N + i] : -1;
  }
  return MHC_OK;
}

mhc_status mhc_virial_compute(mhc_virial* v, const double* pos, const double* vel, const double* fe, double* U,
                              double* F, double* W, float* W32, double* Fext) {
  mhc_status st = venter(v);
  if (st) return st;
  if (!pos) return vfail(v, MHC_ERR_INVALID_ARG, "NULL positions");
  if (!v->lists_ok) return vfail(v, MHC_ERR_STATE, "no valid neighbour lists (call mhc_virial_neighbors)");
  double f[3] = {0.0, 0.0, 0.0};
  if (fe)
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(fe[a])) return vfail(v, MHC_ERR_INVALID_ARG, "non-finite F_e");
      f[a] = fe[a];
    }
  VHIP_TRY(hipSetDevice(v->device), "hipSetDevice");
  TersoffArgs a{};
  a.pos = pos;
  a.N = v->N;
  for (int q = 0; q < 3; ++q) a.box[q] = v->box[q], a.ibox[q] = 1.0 / v->box[q];
  a.nbr = v->nb.nbr;
  a.n_nb = v->nb.n_nb;
  a.rev = v->nb.rev;
  a.max_nb = v->max_nb;
  a.dd = v->d_dd;
  a.U = U ? U : v->d_U;
  GatherArgs o{};
  o.vel = vel;
  o.mass = v->d_mass;
  for (int q = 0; q < 3; ++q) o.fe[q] = f[q];
  o.ke_unit = KE_UNIT_EV;
  o.rcut2 = rcut2_of(v);
  o.F = F;
  o.W = W;
  o.W32 = W32;
  o.Fext = Fext;
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  if ((st = timing_events(v, e))) return st;
  VHIP_TRY(launch_tersoff(v->stream, a, v->tp, o, v->lpa, e[0], e[1], e[2]), "virial kernels");
  return MHC_OK;
}

}  // extern "C"

namespace {

// NVT with the HNEMD driving force: the drive fe (1/A), the thermostat's
// temperature (K) and mass Q (eV fs^2), g k_B T (eV), and the host state
// (xi, eta) read at entry and written back at the end.
struct NvtArgs {
  double fe[3];
  bool drive;
  double Q, gkt;
  double* state;
};

// The MD loop of mhc_virial_md (nvt null: NVE velocity Verlet) and
// mhc_virial_md_nvt (thermostat half steps around each velocity-Verlet step,
// force + driving force).
mhc_status md_run(mhc_virial* v, double* pos, double* vel, double dt, int32_t n_steps, int32_t rebuild, float* v32,
                  float* W32, double* F, const NvtArgs* nvt) {
  mhc_status st = MHC_OK;
  VHIP_TRY(hipSetDevice(v->device), "hipSetDevice");
  const int64_t N = v->N;
  bool any_compact = false;
  // Evaluation e (0: the entry positions, s + 1: after step s) rebuilds the
  // bond lists if need[e & 1] != 0, which the drift before it sets when an
  // atom has moved more than half the bond lists' skin since their build.
  const double half = 0.5 * v->bond_skin;
  const double thr2 = half * half * (1.0 - 1e-9);
  int64_t e_idx = 0;
  const double c = 0.5 * dt / KE_UNIT_EV;   // half kick: dv = dt/2 F / (m KE)
  int64_t gather_parts = 0;   // work-groups of the last gather launch
  // kick_v32: with nvt, the end of the step on the fly in the gather kernel
  // (second half kick, thermostat scale, float32 velocities, m v^2 partials)
  auto force = [&](float* w32, bool kick_end = false, float* kick_v32 = nullptr) -> mhc_status {
    TersoffArgs a{};
    a.pos = pos;
    a.N = N;
    for (int q = 0; q < 3; ++q) a.box[q] = v->box[q], a.ibox[q] = 1.0 / v->box[q];
    a.nbr = v->nb.nbr;
    a.n_nb = v->nb.n_nb;
    a.rev = v->nb.rev;
    a.max_nb = v->max_nb;
    int lpa = v->lpa;
    if (v->compact) {   // bond lists out of the skin lists, rebuilt when the atoms have moved enough
      any_compact = true;
      const int sl = (int)(e_idx & 1);
      VHIP_TRY(launch_bonds(v->stream, pos, N, v->box, v->nb.nbr, v->nb.n_nb, v->tp.R + v->tp.D + v->bond_skin,
                            v->max_b, v->bb, false, v->bb.need + sl, v->bb.need + (sl ^ 1)),
               "bonds");
      a.nbr = v->bb.nbr;
      a.n_nb = v->bb.n_nb;
      a.rev = v->bb.rev;
      a.max_nb = v->max_b;
      a.bond_need = v->bb.need + sl;   // the site kernel fills their reverse slots after a rebuild
      a.bond_mask = v->bb.mask;
      a.full_nbr = v->nb.nbr;
      a.full_rev = v->nb.rev;
      a.bond_rev = v->bb.rev;
      a.bond_flags = v->bb.flags;
      lpa = v->lpa_b;
    }
    a.dd = v->d_dd;
    a.U = v->d_U;
    GatherArgs o{};
    o.mass = v->d_mass;
    o.ke_unit = KE_UNIT_EV;
    o.rcut2 = rcut2_of(v);
    o.F = v->d_F;
    o.W32 = w32;
    if (nvt && nvt->drive) {   // F + F_ext (Eq. 12), E_i from the velocities now
      o.add_ext = true;
      o.vel = vel;
      for (int q = 0; q < 3; ++q) o.fe[q] = nvt->fe[q];
    }
    if (kick_end) {
      o.kick_vel = vel;
      o.kick_c = c;
      o.kick_scale = v->d_thermo;
      o.kick_v32 = kick_v32;
      o.ke_part = v->d_kepart;
    }
    gather_parts = gather_blocks(N, lpa);
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    mhc_status s2 = timing_events(v, e);
    if (s2) return s2;
    VHIP_TRY(launch_tersoff(v->stream, a, v->tp, o, lpa, e[0], e[1], e[2]), "force kernels");
    return MHC_OK;
  };
  // overflow and reverse-slot flags of the bond passes accumulate over this call's steps
  VHIP_TRY(launch_zero_i32(v->stream, v->bb.flags, 3), "clear bond flags");
  VHIP_TRY(launch_set_i32(v->stream, v->bb.need, 1), "bond rebuild flag");   // the entry evaluation builds
  if ((st = force(nullptr))) return st;     // forces at the entry positions
  if (nvt) {
    // thermostat half steps around each velocity-Verlet step
    VHIP_TRY(launch_thermostat_set(v->stream, v->d_thermo, nvt->state[0], nvt->state[1]), "thermostat state");
    VHIP_TRY(launch_md_ke_partial(v->stream, vel, v->d_mass, N, v->d_kepart), "kinetic energy");
    VHIP_TRY(launch_thermostat(v->stream, v->d_kepart, md_nvt_parts(N), v->d_thermo, dt, nvt->Q, nvt->gkt,
                               KE_UNIT_EV, 2),
             "thermostat");
    for (int32_t s = 0; s < n_steps; ++s) {
      e_idx = s + 1;
      VHIP_TRY(launch_md_nvt_start(v->stream, pos, vel, v->d_F, v->d_mass, c, dt, v->box, N, v->d_thermo,
                                   v->compact ? v->bb.ref : nullptr, thr2, v->bb.need + (e_idx & 1)),
               "kick and drift");
      if (rebuild > 0 && (s + 1) % rebuild == 0) {
        if ((st = mhc_virial_neighbors(v, pos, nullptr))) return st;
        VHIP_TRY(launch_set_i32(v->stream, v->bb.need + (e_idx & 1), 1), "bond rebuild flag");
      }
      // the force, and the end of the step in the same gather kernel
      if ((st = force(W32 ? W32 + (int64_t)s * N * 9 : nullptr, true, v32 ? v32 + (int64_t)s * N * 3 : nullptr)))
        return st;
      VHIP_TRY(launch_thermostat(v->stream, v->d_kepart, gather_parts, v->d_thermo, dt, nvt->Q, nvt->gkt,
                                 KE_UNIT_EV, s + 1 < n_steps ? 3 : 1),
               "thermostat");
    }
  } else {
    // kicks and drifts: before step s's force the first half kick and drift of
    // step s (fused with the second half kick of step s - 1 from s = 1 on);
    // after the last force its second half kick alone
    auto kick_drift = [&](int32_t s) -> mhc_status {
      e_idx = s + 1;   // the evaluation after this drift
      const bool track = v->compact;
      VHIP_TRY(launch_md_step(v->stream, pos, vel, v->d_F, v->d_mass, c, dt, v->box, N, s > 0, true,
                              s > 0 && v32 ? v32 + (int64_t)(s - 1) * N * 3 : nullptr, track ? v->bb.ref : nullptr,
                              thr2, v->bb.need + (e_idx & 1)),
               "kick and drift");
      return MHC_OK;
    };
    for (int32_t s = 0; s < n_steps; ++s) {
      if ((st = kick_drift(s))) return st;
      if (rebuild > 0 && (s + 1) % rebuild == 0) {
        if ((st = mhc_virial_neighbors(v, pos, nullptr))) return st;
        // new lists (and possibly new bond slots): the bond lists follow them
        VHIP_TRY(launch_set_i32(v->stream, v->bb.need + (e_idx & 1), 1), "bond rebuild flag");
      }
      if ((st = force(W32 ? W32 + (int64_t)s * N * 9 : nullptr))) return st;
    }
    VHIP_TRY(launch_md_step(v->stream, pos, vel, v->d_F, v->d_mass, c, dt, v->box, N, true, false,
                            v32 ? v32 + (int64_t)(n_steps - 1) * N * 3 : nullptr, nullptr, 0.0, nullptr),
             "half kick");
  }
  if (F) VHIP_TRY(hipMemcpyAsync(F, v->d_F, (size_t)N * 3 * 8, hipMemcpyDeviceToDevice, v->stream), "copy forces");
  if (any_compact) {
    int f[3] = {0, 0, 0};
    VHIP_TRY(hipMemcpyAsync(f, v->bb.flags, sizeof(f), hipMemcpyDeviceToHost, v->stream), "read bond flags");
    VHIP_TRY(hipStreamSynchronize(v->stream), "md sync");
    if (f[1])
      return vfail(v, MHC_ERR_INVALID_ARG,
                   "an atom's bond count rose to " + std::to_string(f[0]) + ", above the " + std::to_string(v->max_b) +
                       " bond slots set at the last list build (rebuild the lists more often); the steps' results are "
                       "not valid");
    if (f[2]) return vfail(v, MHC_ERR_INVALID_ARG, "bond lists are not symmetric (non-finite positions?)");
  }
  if (nvt) {
    double th[4] = {0.0, 0.0, 0.0, 0.0};
    VHIP_TRY(hipMemcpyAsync(th, v->d_thermo, sizeof(th), hipMemcpyDeviceToHost, v->stream), "read thermostat");
    VHIP_TRY(hipStreamSynchronize(v->stream), "md sync");
    nvt->state[0] = th[0];
    nvt->state[1] = th[1];
  }
  return MHC_OK;
}

mhc_status md_check(mhc_virial* v, double* pos, double* vel, double dt, int32_t n_steps, int32_t rebuild) {
  mhc_status st = venter(v);
  if (st) return st;
  if (!pos || !vel) return vfail(v, MHC_ERR_INVALID_ARG, "NULL positions or velocities");
  if (n_steps < 0 || rebuild < 0) return vfail(v, MHC_ERR_INVALID_ARG, "n_steps and rebuild must be >= 0");
  if (!std::isfinite(dt) || !(dt > 0.0)) return vfail(v, MHC_ERR_INVALID_ARG, "dt must be finite and > 0");
  if (!v->lists_ok) return vfail(v, MHC_ERR_STATE, "no valid neighbour lists (call mhc_virial_neighbors)");
  return MHC_OK;
}

}  // namespace

extern "C" {

mhc_status mhc_virial_md(mhc_virial* v, double* pos, double* vel, double dt, int32_t n_steps, int32_t rebuild,
                         float* v32, float* W32, double* F) {
  mhc_status st = md_check(v, pos, vel, dt, n_steps, rebuild);
  if (st || n_steps == 0) return st;
  return md_run(v, pos, vel, dt, n_steps, rebuild, v32, W32, F, nullptr);
}

mhc_status mhc_virial_md_nvt(mhc_virial* v, double* pos, double* vel, double dt, int32_t n_steps, int32_t rebuild,
                             const double* fe, double temperature, double tau, double* thermostat, float* v32,
                             float* W32, double* F) {
  mhc_status st = md_check(v, pos, vel, dt, n_steps, rebuild);
  if (st) return st;
  if (!std::isfinite(temperature) || !(temperature > 0.0) || !std::isfinite(tau) || !(tau > 0.0))
    return vfail(v, MHC_ERR_INVALID_ARG, "temperature and tau must be finite and > 0");
  if (!thermostat || !std::isfinite(thermostat[0]) || !std::isfinite(thermostat[1]))
    return vfail(v, MHC_ERR_INVALID_ARG, "thermostat must point to two finite numbers (xi, eta)");
  NvtArgs a{};
  a.drive = false;
  for (int q = 0; q < 3; ++q) {
    a.fe[q] = fe ? fe[q] : 0.0;
    if (!std::isfinite(a.fe[q])) return vfail(v, MHC_ERR_INVALID_ARG, "fe must be finite");
    if (a.fe[q] != 0.0) a.drive = true;
  }
  a.gkt = 3.0 * (double)v->N * K_B_EV * temperature;
  a.Q = a.gkt * tau * tau;
  if (!std::isfinite(a.Q) || !(a.Q > 0.0)) return vfail(v, MHC_ERR_INVALID_ARG, "thermostat mass out of range");
  a.state = thermostat;
  if (n_steps == 0) return MHC_OK;
  return md_run(v, pos, vel, dt, n_steps, rebuild, v32, W32, F, &a);
}

mhc_status mhc_virial_synchronize(mhc_virial* v) {
  mhc_status st = venter(v);
  if (st) return st;
  VHIP_TRY(hipSetDevice(v->device), "hipSetDevice");
  VHIP_TRY(hipStreamSynchronize(v->stream), "synchronize");
  return MHC_OK;
}

mhc_status mhc_virial_set_timing(mhc_virial* v, int enable) {
  mhc_status st = venter(v);
  if (st) return st;
  if (enable < 0) return vfail(v, MHC_ERR_INVALID_ARG, "enable is 0 (off) or k >= 1 (every k-th evaluation)");
  v->timing_every = enable;
  v->n_evals = 0;
  return MHC_OK;
}

mhc_status mhc_virial_kernel_timing(mhc_virial* v, int64_t* launches, double* site_ms, double* gather_ms) {
  mhc_status st = venter(v);
  if (st) return st;
  VHIP_TRY(hipSetDevice(v->device), "hipSetDevice");
  VHIP_TRY(hipStreamSynchronize(v->stream), "timing sync");
  double ts = 0.0, tg = 0.0;
  for (size_t q = 0; q + 3 <= v->ev_used; q += 3) {
    float a = 0.0f, b = 0.0f;
    VHIP_TRY(hipEventElapsedTime(&a, v->ev[q], v->ev[q + 1]), "event elapsed");
    VHIP_TRY(hipEventElapsedTime(&b, v->ev[q + 1], v->ev[q + 2]), "event elapsed");
    ts += a;
    tg += b;
  }
  if (launches) *launches = (int64_t)(v->ev_used / 3);
  if (site_ms) *site_ms = ts;
  if (gather_ms) *gather_ms = tg;
  v->ev_used = 0;
  return MHC_OK;
}

}  // extern "C"
