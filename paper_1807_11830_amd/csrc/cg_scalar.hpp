// Start-of-iteration scalar logic of device-resident CG, shared by the fused
// 2D normal-operator kernel and the 3D p-update kernel.
//
// At iteration k every block of problem b sums the <r, r> partials left by
// the previous launch, in index order, so all blocks hold the same rho_k and
// take the same decision without any grid-wide synchronisation:
//   rho_k not finite                         -> NONFINITE
//   k > 0, tol > 0, sqrt(rho_k / rho_0) < tol -> CONVERGED
//   rho_k == 0                               -> EXACT
// otherwise beta = rho_k / rho_(k-1) (0 at k = 0).  The designated block
// publishes rho_k (history, the rho[k & 1] slot, rho_cur) and the stop status.
#pragma once

#include "kernels.hpp"
#include "reduce.hpp"

namespace sense {

// Returns false when problem b has stopped (the caller returns); otherwise
// sets beta.  designated: this block publishes the scalars.
__device__ __forceinline__ bool cg_iteration_begin(CgState* st, const double* rr_part, int rr_tiles,
                                                   double* rho_hist, int hist_len, double tol, int b,
                                                   bool designated, double& beta) {
  if (st->status != CG_RUNNING) return false;
  const int k = st->iter;
  const double rho = ordered_sum(rr_part + (long)b * rr_tiles, rr_tiles);
  const double rho0 = (k == 0) ? rho : st->rho0;
  int stop = CG_RUNNING;
  if (!finite64(rho)) stop = CG_NONFINITE;
  else if (k > 0 && tol > 0.0 && sqrt(rho / rho0) < tol) stop = CG_CONVERGED;
  else if (rho == 0.0) stop = CG_EXACT;
  if (designated) {
    if (k == 0) st->rho0 = rho;
    st->rho[k & 1] = rho;
    st->rho_cur = rho;
    if (rho_hist && k < hist_len) rho_hist[(long)b * hist_len + k] = rho;
    if (stop != CG_RUNNING) st->status = stop;
  }
  if (stop != CG_RUNNING) return false;
  beta = (k > 0) ? rho / st->rho[(k - 1) & 1] : 0.0;
  return true;
}

}  // namespace sense
