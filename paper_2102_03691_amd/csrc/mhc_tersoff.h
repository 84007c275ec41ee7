// Internal declarations of the per-atom virial kernels (k_tersoff.hip) used
// by the host side in mhc_virial.cpp.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhc {

// Cell grid of the neighbour search: nc cells per axis (1, or at least 3, so
// that the 27 surrounding cells never repeat), each at least the cutoff wide.
struct CellGrid {
  double box[3];
  double ibox[3];   // 1 / box: the minimum-image shift multiplies instead of dividing
  int nc[3];
};

// Device buffers of the neighbour lists: nbr, rev [max_nb][N] (slot-major),
// n_nb [N]; cell_of [N], atoms [N]; count, fill [n_cells], start [n_cells + 1];
// tile_sums [ceil(n_cells / 1024)] (scan workspace); flags[0] = largest
// neighbour count found, flags[1] = 1 if a reverse slot was missing,
// flags[2] = largest count inside the bond lists' cutoff.
struct NeighborBufs {
  int* nbr;
  int* rev;
  int* n_nb;
  int* cell_of;
  int* atoms;
  int* count;
  int* fill;
  int* start;
  int* tile_sums;
  int* flags;
};

// Bond lists (the listed pairs inside R + D + delta, delta the bond lists'
// own skin): nbr, rev [max_b][N] (slot-major), n_nb [N], mask [N] (bit s:
// list slot s is kept), ref [N][3] (positions at their build); flags[0] =
// largest count found, flags[1] = 1 if an atom had more than max_b, flags[2] =
// 1 if a reverse slot was missing; need [2]: the rebuild flags of alternate
// evaluations.
struct BondBufs {
  int* nbr;
  int* rev;
  int* n_nb;
  unsigned long long* mask;
  int* flags;
  double* ref;
  int* need;
};

// Tersoff parameters as the kernels use them: l3m = lambda3^m, c2 = c^2, d2 = d^2,
// c2d2 = c^2 / d^2, gc2d2 = gamma c^2 / d^2, g2c2 = 2 gamma c^2, ninv2 = -1 / (2n).
struct TersoffParams {
  double A, B, l1, l2, l3m, beta, n, c2, d2, c2d2, h, gamma, R, D, gc2d2, g2c2, ninv2;
  int m;
};

// Per-evaluation buffers: positions (device, [N][3]); neighbour lists; the
// partials dd [3][max_nb][N] (dU_i/dr_ij); site energies U [N].
struct TersoffArgs {
  const double* pos;
  int64_t N;
  double box[3];
  double ibox[3];   // 1 / box
  const int* nbr;
  const int* n_nb;
  const int* rev;
  int max_nb;
  double* dd;
  double* U;
  // Bond lists (nbr, n_nb above) just rebuilt from the skin lists: when
  // bond_need is not null and *bond_need != 0 the site kernel also writes
  // their reverse slots to bond_rev (which rev must then point to) from the
  // skin lists' full_nbr / full_rev and the kept-slot masks; bond_flags[2] = 1
  // if one is missing.
  const int* bond_need;
  const unsigned long long* bond_mask;
  const int* full_nbr;
  const int* full_rev;
  int* bond_rev;
  int* bond_flags;
};

// Outputs of the gather kernel (any may be null): F [N][3], W [N][3][3] float64
// and W32 float32 (W[i][mu][nu]), Fext [N][3]; vel [N][3] and mass [N] give the
// kinetic part of E_i (vel null: E_i = U_i).
struct GatherArgs {
  const double* vel;
  const double* mass;
  double fe[3];
  double ke_unit;
  double rcut2;               // (R + D)^2 slightly widened: pairs beyond have zero partials
  double* F;
  double* W;
  float* W32;
  double* Fext;
  bool add_ext;               // F = interatomic force + F_ext (needs fe; vel for E_i)
  // The end of an NVT step on the fly (kick_vel null: none): v += kick_c F / m,
  // v *= kick_scale[2] on kick_vel (after E_i has read vel), its float32 copy to
  // kick_v32 (may be null), and per work-group the sum of m v^2 to ke_part.
  double* kick_vel;
  double kick_c;
  const double* kick_scale;
  float* kick_v32;
  double* ke_part;
};

// Lists of the pairs closer than rc; also counts, per atom, those closer
// than rb (flags[2]: the largest such count).
hipError_t launch_neighbors(hipStream_t s, const double* pos, int64_t N, const CellGrid& cg, double rc, double rb,
                            int max_nb, NeighborBufs b);
// Zero n ints (n > 0).
hipError_t launch_zero_i32(hipStream_t s, int* p, int n);
// Bond lists out of the lists (nbr, n_nb): every pair closer than rb, at
// most max_b per atom (max_nb <= 64), and their kept-slot masks (their
// reverse slots come from the next site kernel: TersoffArgs.bond_need).  The
// flags accumulate over launches unless reset_flags clears them first.  need
// (null: always) makes the build conditional on *need != 0, decided on the
// device; clear (null: none) is zeroed.
hipError_t launch_bonds(hipStream_t s, const double* pos, int64_t N, const double box[3], const int* nbr,
                        const int* n_nb, double rb, int max_b, BondBufs b, bool reset_flags, const int* need,
                        int* clear);
hipError_t launch_set_i32(hipStream_t s, int* p, int value);
// Lanes per atom of the evaluation kernels for a largest neighbour count:
// the next power of two, at least 4 (64 at most: max_nb <= 64).
int tersoff_lanes(int max_count);
// Queues the site and gather kernels with lpa lanes per atom; the optional
// events are recorded before the site kernel (e0), between the two (e1) and
// after the gather kernel (e2).
hipError_t launch_tersoff(hipStream_t s, const TersoffArgs& a, const TersoffParams& p, const GatherArgs& o, int lpa,
                          hipEvent_t e0, hipEvent_t e1, hipEvent_t e2);

// Velocity Verlet between two force evaluations on [N][3] float64 arrays:
// kick2 = the second half kick of a step, vel += c F / mass (v32: the result
// also in float32, NULL to skip); kick1_drift = the first half kick of the
// next step with the same F, then the drift pos += dt vel wrapped into the
// box, and with ref (NULL: none) *need = 1 if an atom is farther than
// sqrt(thr2) from its position in ref.
hipError_t launch_md_step(hipStream_t s, double* pos, double* vel, const double* F, const double* mass, double c,
                          double dt, const double box[3], int64_t N, bool kick2, bool kick1_drift, float* v32,
                          const double* ref, double thr2, int* need);

// Nose-Hoover thermostat steps (state st [4] on the device: xi, eta, the
// velocity scale exp(-xi dt/2), the last kinetic energy).  ke_partial: sums
// of m v^2, one per 64 atoms (md_nvt_parts of them); thermostat: mode 1
// end-of-step, 2 start-of-step, 3 both, from n_part partials; start: the
// scale, the first half kick and the drift (ref, thr2, need as for
// launch_md_step).  The end of a step runs in the gather kernel
// (GatherArgs.kick_vel).
int64_t md_nvt_parts(int64_t N);
hipError_t launch_md_ke_partial(hipStream_t s, const double* vel, const double* mass, int64_t N, double* part);
hipError_t launch_thermostat(hipStream_t s, const double* part, int64_t n_part, double* st, double dt, double Q,
                             double gkt, double ke_unit, int mode);
// Work-groups of the gather kernel for lpa lanes per atom (its ke_part count).
int64_t gather_blocks(int64_t N, int lpa);
hipError_t launch_md_nvt_start(hipStream_t s, double* pos, double* vel, const double* F, const double* mass, double c,
                               double dt, const double box[3], int64_t N, const double* st, const double* ref,
                               double thr2, int* need);
hipError_t launch_thermostat_set(hipStream_t s, double* st, double xi, double eta);

}  // namespace mhc
