// Whole CG-SENSE solves of small 2D slices, one workgroup per batch element.
//
// For a slice of at most 64 columns and 64 rows every vector of the solve
// (x, r, p, q: E values per thread) stays in registers and one workgroup
// runs all K iterations of the textbook loop (the same order of tests and
// updates as the host CG of the normal equations): q = A p by the
// readout-decoupled normal operator (per column: coil product, masked
// forward/inverse transform pair along y, conjugate coil sum), then
// Re<p, q>, the updates of x and r, <r, r> and the new direction.  Both
// inner products are block reductions in fp64 with a fixed order, so the
// result is deterministic; no wait ever spans two workgroups.  One launch
// replaces the per-iteration launches whose latency dominates a small
// solve.  The launch after E^H y (which has written b into r) is the whole
// solve, including the per-problem info.
#include "bufio.hpp"
#include "kernels.hpp"
#include "lengths.hpp"
#include "reduce.hpp"

namespace sense {

constexpr int kSmallCols = 64;  // columns per workgroup: the whole slice

struct SmallParams {
  const void* maps;
  const c32* b;      // E^H y [B][ny][nx]
  c32* x;            // [B][ny][nx]
  const c32* tw;     // [ny]
  const float* mu;   // [ny] uncentred mask / ny
  long nx;
  long maps_bstride;
  int ncoils;
  int K;
  float lambda;
  double tol;
  CgState* state;    // [B]
  CgInfo* info;      // [B] plan copy
  CgInfo* info2;     // [B] caller copy or null
  double* rho_hist;  // [B][hist_len] or null
  int hist_len;
};

template <int N>
constexpr bool small_len() {
  return N == 8 || N == 16 || N == 32 || N == 48 || N == 64;
}

// Sum of v over the block, returned to every thread (fixed order).
template <int NT>
__device__ __forceinline__ double block_sum_all(double v, double* red, double* bcast) {
  const double t = block_sum<NT>(v, red);
  if (threadIdx.x == 0) *bcast = t;
  __syncthreads();
  const double r = *bcast;
  __syncthreads();  // red and bcast are reused
  return r;
}

template <int N, int ST>
__global__ void __launch_bounds__(Len<N>::T * kSmallCols) cg_small_kernel(SmallParams P) {
  constexpr int T = Len<N>::T;
  constexpr int E = Len<N>::E;
  constexpr int TX = kSmallCols;
  constexpr int NT = T * TX;
  using Rad = typename Len<N>::R;
  using SType = typename StorageT<ST>::T;

  __shared__ c32 xbuf[N * TX];
  __shared__ c32 tw[N];
  __shared__ float mu[N];
  __shared__ double red[NT / 64];
  __shared__ double bcast;

  const int tid = threadIdx.x;
  const int cx = tid % TX;
  const int t = tid / TX;
  const int b = blockIdx.x;
  const long nx = P.nx;
  const bool valid = cx < nx;
  const uint32_t xl = (uint32_t)(valid ? cx : nx - 1);
  const long nvox = (long)N * nx;
  const uint32_t voff = (uint32_t)t * (uint32_t)nx + xl;
  const uint32_t rstep = (uint32_t)T * (uint32_t)nx;
  const uint32_t img_bytes = (uint32_t)(nvox * (long)sizeof(c32));

  for (int i = tid; i < N; i += NT) {
    tw[i] = P.tw[i];
    mu[i] = P.mu[i];
  }

  c32 x[E], r[E], p[E], q[E];
  double rr = 0.0;
  {
    const Buf bb = make_buf(P.b + (long)b * nvox, img_bytes);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      r[j] = buf_load_c64(bb, voff * 8u, (uint32_t)j * rstep * 8u);
      p[j] = r[j];
      x[j] = {0.f, 0.f};
      if (valid) rr += (double)r[j].re * (double)r[j].re + (double)r[j].im * (double)r[j].im;
    }
  }
  __syncthreads();

  using TwC = TwChoice<N, T, Rad>;
  typename TwC::type twsrc;
  if constexpr (TwC::regs) twsrc.load(tw, t);
  else twsrc.tw = tw;
  LineView<TX> lv{&xbuf[cx]};

  const SType* S = static_cast<const SType*>(P.maps) + (long)b * P.maps_bstride;
  const uint32_t coil_bytes = (uint32_t)(nvox * (long)sizeof(SType));
  double* hist = P.rho_hist ? P.rho_hist + (long)b * P.hist_len : nullptr;

  double rho = block_sum_all<NT>(rr, red, &bcast);
  const double rho0 = rho;
  if (tid == 0 && hist && P.hist_len > 0) hist[0] = rho;
  int status = finite64(rho) ? CG_RUNNING : CG_NONFINITE;
  int k = 0;
  while (status == CG_RUNNING && k < P.K) {
    if (rho == 0.0) {
      status = CG_EXACT;
      break;
    }
    // q = A p
#pragma unroll
    for (int j = 0; j < E; ++j) q[j] = {0.f, 0.f};
    for (int c = 0; c < P.ncoils; ++c) {
      const Buf bs = make_buf(S + (long)c * nvox, coil_bytes);
      c32 s[E], u[E];
#pragma unroll
      for (int j = 0; j < E; ++j) s[j] = buf_load_st<ST>(bs, voff, (uint32_t)j * rstep);
#pragma unroll
      for (int j = 0; j < E; ++j) u[j] = cmul(s[j], p[j]);
      fft_line<N, T, -1>(u, t, twsrc, lv, Rad{});
#pragma unroll
      for (int j = 0; j < E; ++j) u[j] = cscale(u[j], mu[t + T * j]);
      fft_line<N, T, +1>(u, t, twsrc, lv, Rad{});
#pragma unroll
      for (int j = 0; j < E; ++j) q[j] = cfma_conj(q[j], s[j], u[j]);
    }
    double pq = 0.0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      q[j] = {q[j].re + P.lambda * p[j].re, q[j].im + P.lambda * p[j].im};
      if (valid) pq += (double)p[j].re * (double)q[j].re + (double)p[j].im * (double)q[j].im;
    }
    const double eta = block_sum_all<NT>(pq, red, &bcast);
    if (!finite64(eta)) {
      status = CG_NONFINITE;
      break;
    }
    if (eta <= 0.0) {
      status = CG_BREAKDOWN;
      break;
    }
    const double alpha = rho / eta;
    rr = 0.0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      x[j] = {(float)((double)x[j].re + alpha * p[j].re), (float)((double)x[j].im + alpha * p[j].im)};
      r[j] = {(float)((double)r[j].re - alpha * q[j].re), (float)((double)r[j].im - alpha * q[j].im)};
      if (valid) rr += (double)r[j].re * (double)r[j].re + (double)r[j].im * (double)r[j].im;
    }
    const double rho_new = block_sum_all<NT>(rr, red, &bcast);
    ++k;
    if (tid == 0 && hist && k < P.hist_len) hist[k] = rho_new;
    if (!finite64(rho_new)) {
      status = CG_NONFINITE;
      rho = rho_new;
      break;
    }
    if (P.tol > 0.0 && sqrt(rho_new / rho0) < P.tol) {
      status = CG_CONVERGED;
      rho = rho_new;
      break;
    }
    const double beta = rho_new / rho;
#pragma unroll
    for (int j = 0; j < E; ++j)
      p[j] = {(float)((double)r[j].re + beta * p[j].re), (float)((double)r[j].im + beta * p[j].im)};
    rho = rho_new;
  }
  if (status == CG_RUNNING) status = CG_MAXITER;

  if (valid) {
    const Buf bx = make_buf(P.x + (long)b * nvox, img_bytes);
#pragma unroll
    for (int j = 0; j < E; ++j) buf_store_c64(bx, x[j], voff * 8u, (uint32_t)j * rstep * 8u);
  }
  if (tid == 0) {
    CgState st{};
    st.iter = k;
    st.status = status;
    st.rho0 = rho0;
    st.rho[k & 1] = rho;
    st.rho_cur = rho;
    P.state[b] = st;
    CgInfo o;
    o.iters_run = k;
    o.status = status;
    o.rho0 = rho0;
    o.rho_final = rho;
    P.info[b] = o;
    if (P.info2) P.info2[b] = o;
  }
}

bool small_solve_supported(const Geom& g) {
  if (g.nz != 1 || g.nx > kSmallCols || g.nx < 1) return false;
  bool ok = false;
  dispatch_length(g.ny, [&](auto nc) { ok = small_len<decltype(nc)::value>(); });
  return ok;
}

hipError_t launch_cg_small(const Geom& g, const Tables& tb, const void* maps, const c32* bvec, c32* x, int K,
                           float lambda, const CgArgs& cg, CgInfo* info, CgInfo* info2, hipStream_t st) {
  if (!small_solve_supported(g)) return hipErrorInvalidValue;
  SmallParams P{};
  P.maps = maps;
  P.b = bvec;
  P.x = x;
  P.tw = tb.tw_y;
  P.mu = tb.mu_y;
  P.nx = g.nx;
  P.maps_bstride = g.maps_bstride;
  P.ncoils = g.ncoils;
  P.K = K;
  P.lambda = lambda;
  P.tol = cg.tol;
  P.state = cg.state;
  P.info = info;
  P.info2 = info2;
  P.rho_hist = cg.rho_hist;
  P.hist_len = cg.hist_len;
  hipError_t err = hipErrorInvalidValue;
  dispatch_length(g.ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if constexpr (small_len<N>()) {
      const dim3 grid((unsigned)g.batch), block(Len<N>::T * kSmallCols);
      switch (g.maps_storage) {
        case ST_C64: hipLaunchKernelGGL((cg_small_kernel<N, ST_C64>), grid, block, 0, st, P); break;
        case ST_BF16: hipLaunchKernelGGL((cg_small_kernel<N, ST_BF16>), grid, block, 0, st, P); break;
        case ST_FP16: hipLaunchKernelGGL((cg_small_kernel<N, ST_FP16>), grid, block, 0, st, P); break;
        default: return;
      }
      err = hipGetLastError();
    }
  });
  return err;
}

}  // namespace sense
