// Grouped back end (mhc_group_*): the per-step totals, the bin reduction and
// the GKMA correlation update of every system of a group in one launch each,
// instead of small launches per system.
#pragma once
#include "mhc_common.h"

namespace mhc {

// Per-system arguments of the totals and the correlation update (device-
// resident).  n_rt: row tiles of the correlation grid (0 for a system
// without GKMA); the correlation reads the block's first step index at t0_dev
// and the number of buffered steps to correlate (0: none this block) at
// tbuf_dev.
struct BackDesc {
  const double* jt_part; int n_chunks; double* jtot;
  const double* X; int64_t ldx; int64_t R3; int L; const double* ring; int64_t ring_len;
  double* csum; double* ccomp; const int64_t* t0_dev; const int64_t* tbuf_dev; int n_rt;
};

// Device arrays of one group's back end: descriptors, the reduction
// arguments of every system, and per launch the first work-group of each
// system (ascending) with the grid total.
struct BackGroup {
  const BackDesc* d;
  const ReduceArgs* red;
  const int *wg0_seg, *wg0_red, *wg0_corr;
  int n_wg_seg, n_wg_red, n_wg_corr;
};

// Totals, segment sums, bin sums and correlation updates of the n systems for
// a full block of t_count steps, in that order on stream s.
hipError_t launch_back_group(hipStream_t s, const BackGroup& b, int n, int t_count);

}  // namespace mhc
