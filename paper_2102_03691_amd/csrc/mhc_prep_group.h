// Grouped input preparation (mhc_group_*): the column maxima and the operand
// prep of every system of a group in one launch each, instead of one small
// launch per system.
#pragma once
#include "mhc_common.h"

namespace mhc {

// Per-system arguments (device-resident; the inputs themselves are read
// through tab, the group's block table).  wg0_cs / wg0_prep: first work-group
// of the system in the grouped column-maxima grid (t_pad x n_cc per system)
// and input-prep grid (n_chunks x t_pad/32 per system), ascending in i.
struct PrepDesc {
  const float* sqrt_m; const float* inv_sqrt_m; int64_t N; int t_pad; int n_chunks;
  void* B; int64_t K_pad; double* jt_part; float* col_scale; float* col_part;
  const float* const* tab;
  int dir;            // -1, or DIR_ALL for a system with the one-contraction direction split
  double* jd_part;    // its split Eq. 10 partials (dir = DIR_ALL)
  int wg0_cs, wg0_prep;
};

// Column maxima (e4m3 precisions) and input prep of the n systems of d for a
// full block of t_count steps; n_wg_cs / n_wg_prep are the grid totals.
hipError_t launch_prep_group(hipStream_t s, int prec, const PrepDesc* d, int n, int t_count, int n_wg_cs,
                             int n_wg_prep);

}  // namespace mhc
