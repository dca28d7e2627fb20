// Start-of-iteration scalar logic of the fused 2D CG iteration.
#pragma once

#include "kernels.hpp"
#include "reduce.hpp"

namespace sense {

// Fused 2D CG: launch k (k >= 1) finishes iteration k-1 before applying A.
// From the partials of launch k-1 (eta = Re<p,q>, zeta = <q,q>, rho =
// <r,r>, the true residual norm of iterate k-1) it checks, in the order of
// the textbook loop, rho (non-finite; tolerance; exactly 0) and eta
// (non-finite; <= 0), then sets alpha = rho / eta and beta = rho~ / rho with
//     rho~ = <r - alpha q, r - alpha q> = rho - 2 alpha Re<r,q> + alpha^2 zeta
//          = alpha^2 zeta - rho,
// the last form because Re<r, A p> = Re<p, A p> = eta: the direction is
// p = r + beta' p_prev and A-conjugate to p_prev, and alpha eta = rho.
// rho~ serves only for beta; the true <r, r> of the new residual is
// computed by this launch and used from the next launch on, so no error
// accumulates through it.  Launch 0 only checks rho_0 (from the init kernel)
// and leaves alpha = beta = 0.
struct CgFused {
  double alpha, beta;
};

__device__ __forceinline__ bool cg_fused_begin(CgState* st, const double* rr_part, int rr_tiles,
                                               const double* cgpart, int part_batch, int ntiles, int rho_tiles,
                                               int stride,
                                               double* rho_hist, int hist_len, double tol, int k, int b,
                                               bool designated, CgFused& o) {
  o.alpha = 0.0;
  o.beta = 0.0;
  if (st->status != CG_RUNNING) return false;
  if (k == 0) {
    const double rho = ordered_sum(rr_part + (long)b * rr_tiles, rr_tiles);
    int stop = CG_RUNNING;
    if (!finite64(rho)) stop = CG_NONFINITE;
    else if (rho == 0.0) stop = CG_EXACT;
    if (designated) {
      st->rho0 = rho;
      st->rho[0] = rho;
      st->rho_cur = rho;
      if (rho_hist && hist_len > 0) rho_hist[(long)b * hist_len] = rho;
      if (stop != CG_RUNNING) st->status = stop;
    }
    return stop == CG_RUNNING;
  }
  const double* pp = cgpart + ((long)((k - 1) & 1) * part_batch + b) * (long)stride * kCgParts;
  double eta = 0.0, zeta = 0.0, rho = 0.0;
  for (int i = 0; i < ntiles; ++i) {
    eta += pp[kCgParts * i];
    zeta += pp[kCgParts * i + 1];
  }
  for (int i = 0; i < rho_tiles; ++i) rho += pp[kCgParts * i + 2];
  int stop = CG_RUNNING;
  if (!finite64(rho)) stop = CG_NONFINITE;
  else if (k - 1 > 0 && tol > 0.0 && sqrt(rho / st->rho0) < tol) stop = CG_CONVERGED;
  else if (rho == 0.0) stop = CG_EXACT;
  else if (!finite64(eta)) stop = CG_NONFINITE;
  else if (eta <= 0.0) stop = CG_BREAKDOWN;
  if (designated) {
    st->rho[(k - 1) & 1] = rho;
    st->rho_cur = rho;
    if (rho_hist && k - 1 < hist_len) rho_hist[(long)b * hist_len + k - 1] = rho;
    if (stop != CG_RUNNING) st->status = stop;
    else st->iter = k;
  }
  if (stop != CG_RUNNING) return false;
  o.alpha = rho / eta;
  const double rho_next = o.alpha * o.alpha * zeta - rho;
  o.beta = rho_next / rho;
  return true;
}

}  // namespace sense
