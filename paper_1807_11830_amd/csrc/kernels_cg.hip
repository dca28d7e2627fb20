// Conjugate-gradient vector kernels for CG-SENSE (the normal equations
// E^H E x = E^H y), one independent problem per batch element.
//
//   init          x = 0, p = r (= b = E^H y), partial <r, r>;  state reset
//   fused final   2D: the updates of the last fused iteration (x, r) and
//                 the partials of <r, r> for the final test
//   update fused  3D: the tests of iteration k, then x, r and p updates and
//                 the <r, r> partials (one reduction per iteration)
//   finish        final tolerance test and per-problem info
//   combine       2D coil groups: the group partials of q added in order
//
// Inner products, alpha and beta are fp64; vectors are fp32 complex.  Every
// block of a batch element reduces the same partials in the same order, so
// all blocks take the same decisions and the results do not depend on
// scheduling.
#include <algorithm>

#include "bufio.hpp"
#include "cg_scalar.hpp"
#include "kernels.hpp"
#include "reduce.hpp"

namespace sense {

constexpr int CG_NT = 256;      // threads per block
constexpr int CG_VEC = 2;       // complex values per 16-byte access
constexpr int CG_STEPS = 4;     // accesses per thread per block
constexpr int CG_CHUNK = CG_NT * CG_VEC * CG_STEPS;  // complex values per block

int cg_tiles(long nvox) { return (int)((nvox + CG_CHUNK - 1) / CG_CHUNK); }

struct alignas(16) c32x2 {
  c32 a, b;
};

__global__ void __launch_bounds__(CG_NT) cg_init_kernel(const c32* __restrict__ bvec, c32* __restrict__ x,
                                                        c32* __restrict__ r, c32* __restrict__ p,
                                                        c32* __restrict__ q, long nvox, CgArgs cg) {
  __shared__ double red[CG_NT / 64];
  const int b = blockIdx.y;
  const long base = (long)b * nvox + (long)blockIdx.x * CG_CHUNK;
  const long lim = (long)b * nvox + nvox;
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < CG_STEPS; ++s) {
    const long i = base + ((long)s * CG_NT + threadIdx.x) * CG_VEC;
    if (i < lim) {  // nvox is even, so a pair never straddles the end
      c32x2 v = *reinterpret_cast<const c32x2*>(bvec + i);
      if (r != bvec) *reinterpret_cast<c32x2*>(r + i) = v;
      *reinterpret_cast<c32x2*>(p + i) = v;
      *reinterpret_cast<c32x2*>(x + i) = c32x2{{0.f, 0.f}, {0.f, 0.f}};
      if (q) *reinterpret_cast<c32x2*>(q + i) = c32x2{{0.f, 0.f}, {0.f, 0.f}};
      acc += (double)v.a.re * v.a.re + (double)v.a.im * v.a.im + (double)v.b.re * v.b.re +
             (double)v.b.im * v.b.im;
    }
  }
  const double tot = block_sum<CG_NT>(acc, red);
  if (threadIdx.x == 0) {
    cg.rr_part[(long)b * cg.rr_tiles + blockIdx.x] = tot;
    if (blockIdx.x == 0) {
      CgState s{};
      s.iter = 0;
      s.status = CG_RUNNING;
      cg.state[b] = s;
    }
  }
}

// The <r, r> partials of the 3D iterations: launch k reads those of r_k
// (the init kernel's for k = 0, else parity buffer (k - 1) & 1) and writes
// those of r_(k+1) into parity buffer k & 1, so no launch overwrites
// partials that its own blocks still read.
const double* cg3_rr_in(const CgArgs& cg, int batch, int k) {
  return k == 0 ? cg.rr_part : cg.rr_par + (long)((k - 1) & 1) * batch * cg.rr_tiles;
}
double* cg3_rr_out(const CgArgs& cg, int batch, int k) {
  return cg.rr_par + (long)(k & 1) * batch * cg.rr_tiles;
}

// 3D CG iteration k, after q = A p left the partials of eta = Re<p, q> and
// zeta = <q, q>.  Every block sums rho_k (the true <r_k, r_k>), eta and zeta
// from the same partials in the same order and takes the textbook loop's
// decisions on them: rho_k non-finite, the tolerance (k > 0), rho_k == 0,
// then eta non-finite or <= 0.  Then alpha = rho_k / eta, x += alpha p,
// r -= alpha q, p = r + beta p with beta = (alpha^2 zeta - rho_k) / rho_k,
// the exact <r - alpha q, r - alpha q> / rho_k under A-conjugacy (the fused
// 2D iteration uses the same form), and the <r, r> partials of the new
// residual, which re-anchor the next launch.  The iteration index comes
// from the launch, not from the state (which this launch advances).
// A block sums the partials once (thousands of them at 3D sizes, a
// latency-bound preamble) and then strides over the CG_CHUNK tiles
// blockIdx.x, blockIdx.x + gridDim.x, ..., writing each tile's <r, r>
// partial, so the partial layout is that of the init kernel.
constexpr int kUpdateMaxBlocks = 1024;
__global__ void __launch_bounds__(CG_NT) cg_update_fused_kernel(c32* __restrict__ x, c32* __restrict__ r,
                                                                c32* __restrict__ p, const c32* __restrict__ q,
                                                                long nvox, int k, const double* __restrict__ rr_in,
                                                                double* __restrict__ rr_out, CgArgs cg) {
  __shared__ double red[CG_NT / 64];
  const int b = blockIdx.y;
  CgState* st = cg.state + b;
  if (st->status != CG_RUNNING) return;
  const double rho = ordered_sum(rr_in + (long)b * cg.rr_tiles, cg.rr_tiles);
  const double eta = ordered_sum(cg.eta_part + (long)b * cg.eta_tiles, cg.eta_tiles);
  const double zeta = ordered_sum(cg.zeta_part + (long)b * cg.eta_tiles, cg.eta_tiles);
  const double rho0 = k == 0 ? rho : st->rho0;
  int stop = CG_RUNNING;
  if (!finite64(rho)) stop = CG_NONFINITE;
  else if (k > 0 && cg.tol > 0.0 && sqrt(rho / rho0) < cg.tol) stop = CG_CONVERGED;
  else if (rho == 0.0) stop = CG_EXACT;
  else if (!finite64(eta)) stop = CG_NONFINITE;
  else if (eta <= 0.0) stop = CG_BREAKDOWN;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) st->rho0 = rho;
    st->rho[k & 1] = rho;
    st->rho_cur = rho;
    if (cg.rho_hist && k < cg.hist_len) cg.rho_hist[(long)b * cg.hist_len + k] = rho;
    if (stop != CG_RUNNING) st->status = stop;
    else st->iter = k + 1;
  }
  if (stop != CG_RUNNING) return;
  const double alpha = rho / eta;
  const double beta = (alpha * alpha * zeta - rho) / rho;

  for (int tile = blockIdx.x; tile < cg.rr_tiles; tile += gridDim.x) {
    const long base = (long)b * nvox + (long)tile * CG_CHUNK;
    const long lim = (long)b * nvox + nvox;
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < CG_STEPS; ++s) {
      const long i = base + ((long)s * CG_NT + threadIdx.x) * CG_VEC;
      if (i < lim) {
        c32x2 xv = *reinterpret_cast<const c32x2*>(x + i);
        c32x2 rv = *reinterpret_cast<const c32x2*>(r + i);
        c32x2 pv = *reinterpret_cast<const c32x2*>(p + i);
        const c32x2 qv = *reinterpret_cast<const c32x2*>(q + i);
        xv.a.re = (float)((double)xv.a.re + alpha * pv.a.re);
        xv.a.im = (float)((double)xv.a.im + alpha * pv.a.im);
        xv.b.re = (float)((double)xv.b.re + alpha * pv.b.re);
        xv.b.im = (float)((double)xv.b.im + alpha * pv.b.im);
        rv.a.re = (float)((double)rv.a.re - alpha * qv.a.re);
        rv.a.im = (float)((double)rv.a.im - alpha * qv.a.im);
        rv.b.re = (float)((double)rv.b.re - alpha * qv.b.re);
        rv.b.im = (float)((double)rv.b.im - alpha * qv.b.im);
        pv.a.re = (float)((double)rv.a.re + beta * pv.a.re);
        pv.a.im = (float)((double)rv.a.im + beta * pv.a.im);
        pv.b.re = (float)((double)rv.b.re + beta * pv.b.re);
        pv.b.im = (float)((double)rv.b.im + beta * pv.b.im);
        *reinterpret_cast<c32x2*>(x + i) = xv;
        *reinterpret_cast<c32x2*>(r + i) = rv;
        *reinterpret_cast<c32x2*>(p + i) = pv;
        acc += (double)rv.a.re * rv.a.re + (double)rv.a.im * rv.a.im + (double)rv.b.re * rv.b.re +
               (double)rv.b.im * rv.b.im;
      }
    }
    const double tot = block_sum<CG_NT>(acc, red);
    if (threadIdx.x == 0) rr_out[(long)b * cg.rr_tiles + tile] = tot;
    __syncthreads();  // red is reused by the next tile
  }
}

__global__ void __launch_bounds__(64) cg_finish_kernel(CgArgs cg, CgInfo* info, CgInfo* info2) {
  const int b = blockIdx.x;
  CgState* st = cg.state + b;
  const int status0 = st->status;
  // every lane takes part in the ordered sum; lane 0 publishes
  const double rho_all = status0 == CG_RUNNING ? ordered_sum(cg.rr_part + (long)b * cg.rr_tiles, cg.rr_tiles) : 0.0;
  if (threadIdx.x != 0) return;
  const int k = st->iter;
  int status = status0;
  double rho0 = st->rho0;
  double rho_final;
  if (status == CG_RUNNING) {
    const double rho = rho_all;
    if (k == 0) rho0 = rho;
    if (cg.rho_hist && k < cg.hist_len) cg.rho_hist[(long)b * cg.hist_len + k] = rho;
    if (!finite64(rho)) status = CG_NONFINITE;
    else if (k > 0 && cg.tol > 0.0 && sqrt(rho / rho0) < cg.tol) status = CG_CONVERGED;
    else status = CG_MAXITER;
    st->status = status;
    st->rho0 = rho0;
    rho_final = rho;
  } else {
    rho_final = st->rho[k & 1];
  }
  CgInfo o;
  o.iters_run = k;
  o.status = status;
  o.rho0 = rho0;
  o.rho_final = rho_final;
  if (info) info[b] = o;
  if (info2) info2[b] = o;
}

// Last step of the fused 2D iteration: launch K's scalar logic, then
// x += alpha p, r -= alpha q and the partials of <r, r> for the final test.
__global__ void __launch_bounds__(CG_NT) cg_fused_final_kernel(c32* __restrict__ x, c32* __restrict__ r,
                                                               const c32* __restrict__ p,
                                                               const c32* __restrict__ q, long nvox, int K,
                                                               CgArgs cg) {
  __shared__ double red[CG_NT / 64];
  const int b = blockIdx.y;
  CgFused o;
  if (!cg_fused_begin(cg.state + b, cg.rr_part, cg.rr_tiles, cg.cgpart, cg.part_batch, cg.part_tiles,
                      cg.rho_tiles, cg.part_stride,
                      cg.rho_hist, cg.hist_len, cg.tol, K, b, blockIdx.x == 0 && threadIdx.x == 0, o))
    return;
  const double alpha = o.alpha;
  const long base = (long)b * nvox + (long)blockIdx.x * CG_CHUNK;
  const long lim = (long)b * nvox + nvox;
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < CG_STEPS; ++s) {
    const long i = base + ((long)s * CG_NT + threadIdx.x) * CG_VEC;
    if (i < lim) {
      c32x2 xv = *reinterpret_cast<const c32x2*>(x + i);
      c32x2 rv = *reinterpret_cast<const c32x2*>(r + i);
      const c32x2 pv = *reinterpret_cast<const c32x2*>(p + i);
      const c32x2 qv = *reinterpret_cast<const c32x2*>(q + i);
      xv.a.re = (float)((double)xv.a.re + alpha * pv.a.re);
      xv.a.im = (float)((double)xv.a.im + alpha * pv.a.im);
      xv.b.re = (float)((double)xv.b.re + alpha * pv.b.re);
      xv.b.im = (float)((double)xv.b.im + alpha * pv.b.im);
      rv.a.re = (float)((double)rv.a.re - alpha * qv.a.re);
      rv.a.im = (float)((double)rv.a.im - alpha * qv.a.im);
      rv.b.re = (float)((double)rv.b.re - alpha * qv.b.re);
      rv.b.im = (float)((double)rv.b.im - alpha * qv.b.im);
      *reinterpret_cast<c32x2*>(x + i) = xv;
      *reinterpret_cast<c32x2*>(r + i) = rv;
      acc += (double)rv.a.re * rv.a.re + (double)rv.a.im * rv.a.im + (double)rv.b.re * rv.b.re +
             (double)rv.b.im * rv.b.im;
    }
  }
  const double tot = block_sum<CG_NT>(acc, red);
  if (threadIdx.x == 0) cg.rr_part[(long)b * cg.rr_tiles + blockIdx.x] = tot;
}

hipError_t launch_cg_fused_final(const Geom& g, const CgVectors& v, int K, const CgArgs& cg, hipStream_t st) {
  const long nvox = g.nx * g.ny * g.nz;
  dim3 grid((unsigned)cg_tiles(nvox), (unsigned)g.batch);
  // launch K-1 left p_(K-1) and r_(K-1) in buffers K & 1
  hipLaunchKernelGGL(cg_fused_final_kernel, grid, dim3(CG_NT), 0, st, v.x, v.r[K & 1], v.p[K & 1], v.q, nvox,
                     K, cg);
  return hipGetLastError();
}

// Coil-group combine of one problem row: q = sum_g qpart[g] + lambda p, the
// groups added in index order (no lambda p when p is null: the E^H combine).
// CG mode (P.state set) also emits the fp64 partials Re<p,q> and <q,q> of
// launch k into cgpart[k & 1] (one entry per block of this
// kernel; <r,r> comes from the fused kernel's group 0) and skips a problem
// that has stopped.  GB >= G slots: the loads of SU accesses (every group
// partial and p) are all issued before the first add, so a thread waits for memory once per SU accesses rather than once
// per partial; groups past G and accesses past the end use an out-of-range
// buffer offset, which reads nothing.
template <int GB>
__device__ __forceinline__ void combine_body(const EheParams& P, const int b, const int tile, const bool cg) {
  constexpr int SU = GB <= 8 ? 4 : 2;
  static_assert(CG_STEPS % SU == 0, "access batches must divide the steps");
  __shared__ double red[CG_NT / 64];
  if (cg && P.state[b].status != CG_RUNNING) return;
  const long nvox = P.nvox;
  const long base = (long)b * nvox + (long)tile * CG_CHUNK;
  const long lim = (long)b * nvox + nvox;
  if (base >= lim) return;
  const c32* pk = cg ? P.p_out : P.p_in;
  const float lam = P.lambda;
  const int G = P.ngroups;
  const uint32_t vbytes = (uint32_t)(lim * (long)sizeof(c32));
  const Buf bg = make_buf(P.qpart, (uint32_t)((long)G * P.qpart_gstride * (long)sizeof(c32)));
  const Buf bp = make_buf(pk, pk ? vbytes : 0u);
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int s0 = 0; s0 < CG_STEPS; s0 += SU) {
    c32x2 t[SU][GB], pv[SU];
    long idx[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const long i = base + ((long)(s0 + u) * CG_NT + threadIdx.x) * CG_VEC;
      idx[u] = i;
      const bool in = i < lim;
#pragma unroll
      for (int gr = 0; gr < GB; ++gr) {
        const uint32_t off =
            in && gr < G ? (uint32_t)(((long)gr * P.qpart_gstride + i) * (long)sizeof(c32)) : kBufOOB;
        t[u][gr] = __builtin_bit_cast(c32x2, __builtin_amdgcn_raw_buffer_load_b128(bg.r, (int)off, 0, 0));
      }
      const uint32_t vo = in ? (uint32_t)(i * (long)sizeof(c32)) : kBufOOB;
      pv[u] = __builtin_bit_cast(c32x2, __builtin_amdgcn_raw_buffer_load_b128(bp.r, (int)vo, 0, 0));
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      if (idx[u] >= lim) continue;
      c32x2 qs = t[u][0];
#pragma unroll
      for (int gr = 1; gr < GB; ++gr) {
        if (gr < G) {
          qs.a.re += t[u][gr].a.re;
          qs.a.im += t[u][gr].a.im;
          qs.b.re += t[u][gr].b.re;
          qs.b.im += t[u][gr].b.im;
        }
      }
      const c32x2 p = pv[u];
      c32x2 qv;
      qv.a = {qs.a.re + lam * p.a.re, qs.a.im + lam * p.a.im};
      qv.b = {qs.b.re + lam * p.b.re, qs.b.im + lam * p.b.im};
      *reinterpret_cast<c32x2*>(P.q + idx[u]) = qv;
      if (cg) {
        acc[0] += (double)p.a.re * qv.a.re + (double)p.a.im * qv.a.im + (double)p.b.re * qv.b.re +
                  (double)p.b.im * qv.b.im;
        acc[1] += (double)qv.a.re * qv.a.re + (double)qv.a.im * qv.a.im + (double)qv.b.re * qv.b.re +
                  (double)qv.b.im * qv.b.im;
      }
    }
  }
  if (!cg) return;
  double* out = P.cgpart + (((long)(P.k & 1) * P.part_batch + b) * P.part_stride + tile) * kCgParts;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double tot = block_sum<CG_NT>(acc[i], red);
    if (threadIdx.x == 0) out[i] = tot;
    __syncthreads();  // red is reused
  }
}

template <bool CG, int GB>
__global__ void __launch_bounds__(CG_NT) combine_kernel(EheParams P) {
  combine_body<GB>(P, blockIdx.y, blockIdx.x, CG);
}

template <int GB>
__global__ void __launch_bounds__(CG_NT) combine_table_kernel(const EheParams* __restrict__ table) {
  const EheParams& P = table[blockIdx.y];
  if (P.ngroups < 2) return;
  combine_body<GB>(P, 0, blockIdx.x, true);
}

template <int GB>
__global__ void __launch_bounds__(CG_NT) combine_inline_kernel(EheInline table) {
  const EheParams& P = table.p[blockIdx.y];
  if (P.ngroups < 2) return;
  combine_body<GB>(P, 0, blockIdx.x, true);
}

// Calls f(std::integral_constant<int, GB>) with the slot count for G groups.
template <class F>
static void dispatch_slots(int groups, F&& f) {
  if (groups <= 2) f(std::integral_constant<int, 2>{});
  else if (groups <= 4) f(std::integral_constant<int, 4>{});
  else if (groups <= 8) f(std::integral_constant<int, 8>{});
  else f(std::integral_constant<int, kMaxCoilGroups>{});
}

hipError_t launch_combine_inline(const EheInline& table, int nproblems, int max_tiles, int max_groups,
                                 hipStream_t st) {
  if (nproblems > kInlineProblems || max_groups > kMaxCoilGroups) return hipErrorInvalidValue;
  dispatch_slots(max_groups, [&](auto gb) {
    hipLaunchKernelGGL((combine_inline_kernel<decltype(gb)::value>), dim3((unsigned)max_tiles, (unsigned)nproblems),
                       dim3(CG_NT), 0, st, table);
  });
  return hipGetLastError();
}

hipError_t launch_combine(const EheParams& P, int batch, bool cg, hipStream_t st) {
  if (P.ngroups > kMaxCoilGroups) return hipErrorInvalidValue;
  dim3 grid((unsigned)cg_tiles(P.nvox), (unsigned)batch);
  dispatch_slots(P.ngroups, [&](auto gb) {
    constexpr int GB = decltype(gb)::value;
    if (cg) hipLaunchKernelGGL((combine_kernel<true, GB>), grid, dim3(CG_NT), 0, st, P);
    else hipLaunchKernelGGL((combine_kernel<false, GB>), grid, dim3(CG_NT), 0, st, P);
  });
  return hipGetLastError();
}

hipError_t launch_combine_table(const EheParams* d_table, int nproblems, int max_tiles, int max_groups,
                                hipStream_t st) {
  if (max_groups > kMaxCoilGroups) return hipErrorInvalidValue;
  dispatch_slots(max_groups, [&](auto gb) {
    hipLaunchKernelGGL((combine_table_kernel<decltype(gb)::value>), dim3((unsigned)max_tiles, (unsigned)nproblems),
                       dim3(CG_NT), 0, st, d_table);
  });
  return hipGetLastError();
}

hipError_t launch_cg_init(const Geom& g, const c32* bvec, c32* x, c32* r, c32* p, c32* q, const CgArgs& cg,
                          hipStream_t st) {
  const long nvox = g.nx * g.ny * g.nz;
  dim3 grid((unsigned)cg_tiles(nvox), (unsigned)g.batch);
  hipLaunchKernelGGL(cg_init_kernel, grid, dim3(CG_NT), 0, st, bvec, x, r, p, q, nvox, cg);
  return hipGetLastError();
}

hipError_t launch_cg_update_fused(const Geom& g, c32* x, c32* r, c32* p, const c32* q, int k, const CgArgs& cg,
                                  hipStream_t st) {
  const long nvox = g.nx * g.ny * g.nz;
  dim3 grid((unsigned)std::min(cg_tiles(nvox), kUpdateMaxBlocks), (unsigned)g.batch);
  hipLaunchKernelGGL(cg_update_fused_kernel, grid, dim3(CG_NT), 0, st, x, r, p, q, nvox, k,
                     cg3_rr_in(cg, g.batch, k), cg3_rr_out(cg, g.batch, k), cg);
  return hipGetLastError();
}

hipError_t launch_cg_finish(const Geom& g, const CgArgs& cg, CgInfo* info, CgInfo* info2, hipStream_t st) {
  hipLaunchKernelGGL(cg_finish_kernel, dim3((unsigned)g.batch), dim3(64), 0, st, cg, info, info2);
  return hipGetLastError();
}

}  // namespace sense
