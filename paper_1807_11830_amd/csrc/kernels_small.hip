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
// solve.  The launch after the x rows of E^H y is the whole solve: it first
// finishes b = E^H y (per coil: masked column loads of the rows' output,
// inverse transform along y, conjugate-sensitivity sum; the arithmetic of
// the E^H column pass, so b is bitwise the one E^H gives), then iterates,
// and writes the per-problem info.
//
// Two thread layouts.  With wave-local lines (WL) the T threads of a column
// are consecutive lanes of one wavefront and every column has its own LDS
// line, so the transform's exchanges need no block barrier and the only
// block barriers of an iteration are those of the two inner products.
// Otherwise a wavefront spans 64 columns at one row offset (whole-line map
// reads) and the exchanges take block barriers.  When the slice has at most
// SmallLen<N>::CR coils the sensitivity maps are read once, before the
// first iteration, and held in registers (MREG: 32 complex values per
// thread, 8 coils at 32 rows, where one wave per SIMD leaves room for 64);
// otherwise each iteration reads them again (from L2).  Measured on
// MI355X, 20 iterations of one slice: 64^2 with 4 coils 172.8 us with the
// maps re-read and the block layout, 129.6 us with the maps in registers and
// wave-local lines, 145.1 us with the maps in registers and the block
// layout.  Without MREG wave-local lines are faster except for complex64
// maps at 64 rows (wave-local against block layout: 48^2 x 8 coils, BF16
// maps, 272 against 319 us; 64^2 x 8 coils, complex64 maps, 333 against
// 298 us).  Maps in registers against re-read, wave-local lines: 16^2 x 8
// coils 123.8 -> 99.6 us, 32^2 x 8 coils 210.2 -> 185.7 us, 48^2 x 2 coils
// 120.5 -> 99.6 us.  Four threads per 64-point line (three radix-4 stages,
// four waves per SIMD) do not leave room for the maps; eight threads per
// 32-point line (three stages) were slower (109 -> 134 us at 4 coils).
#include "bufio.hpp"
#include "kernels.hpp"
#include "lengths.hpp"
#include "reduce.hpp"

namespace sense {

constexpr int kSmallCols = 64;  // columns per workgroup: the whole slice

struct SmallParams {
  const void* maps;
  const c32* w;      // x rows of E^H y [B][C][ny][nx] (unsampled lines unwritten)
  const uint8_t* mask_c;  // [ny] centred mask
  float scale;       // unitary scale and centring sign of E^H
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

// The transform configuration of the whole-solve kernel, and CR: the most
// coils whose maps it holds in registers.
template <int N>
struct SmallLen : Len<N> {
  static constexpr int CR = 32 / Len<N>::E;
};
template <>
struct SmallLen<32> : Len<32> {
  static constexpr int CR = 8;
};

template <int N>
constexpr bool small_len() {
  return N == 8 || N == 16 || N == 32 || N == 48 || N == 64;
}

// Sum of v over the block, returned to every thread.  Lane 0 of each wave
// stores the wave's sum in slots[par][wave]; after one barrier every thread
// adds the W slots in index order (the same order in every thread, so all
// hold the same value).  Successive calls alternate between the two slot
// arrays: the stores of a call can only meet the reads of the call before
// the previous one, and those completed before the previous call's barrier.
template <int NT>
__device__ __forceinline__ double block_allsum(double v, double (*slots)[NT / 64], int& par) {
  constexpr int W = NT / 64;
  v = wave_sum(v);
  if constexpr (W == 1) {
    return v;
  } else {
    if ((threadIdx.x & 63) == 0) slots[par][threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < W; ++i) s += slots[par][i];
    par ^= 1;
    return s;
  }
}

// q += S^H F^H (M/ny) F (S p) over one coil's maps s (column transforms).
template <int N, int T, int SY, class View, class Tw, class Rad>
__device__ __forceinline__ void coil_term(const c32* s, const c32* p, c32* q, const float* mu, int t, const Tw& tw,
                                          View lv, Rad) {
  constexpr int E = N / T;
  c32 u[E];
#pragma unroll
  for (int j = 0; j < E; ++j) u[j] = cmul(s[j], p[j]);
  fft_line<N, T, -1, SY>(u, t, tw, lv, Rad{});
#pragma unroll
  for (int j = 0; j < E; ++j) u[j] = cscale(u[j], mu[j]);
  fft_line<N, T, +1, SY>(u, t, tw, lv, Rad{});
#pragma unroll
  for (int j = 0; j < E; ++j) q[j] = cfma_conj(q[j], s[j], u[j]);
}

template <bool WL>
struct SmallView;
template <>
struct SmallView<true> {
  using type = PadLineView;
  template <int LP>
  __device__ static type make(c32* xbuf, int cx) { return {xbuf + cx * LP}; }
};
template <>
struct SmallView<false> {
  using type = LineView<kSmallCols>;
  template <int LP>
  __device__ static type make(c32* xbuf, int cx) { return {xbuf + cx}; }
};

template <int N, int ST, bool MREG, bool WL>
__global__ void __launch_bounds__(SmallLen<N>::T * kSmallCols) cg_small_kernel(SmallParams P) {
  constexpr int T = SmallLen<N>::T;
  constexpr int E = SmallLen<N>::E;
  constexpr int NT = T * kSmallCols;
  constexpr int LP = padded_line<N>();
  constexpr int CR = MREG ? SmallLen<N>::CR : 1;
  static_assert(64 % T == 0, "a column's threads must share one wavefront");
  using Rad = typename SmallLen<N>::R;
  using SType = typename StorageT<ST>::T;

  __shared__ c32 xbuf[kSmallCols * LP];
  __shared__ c32 tw[N];
  __shared__ double slots[2][NT / 64];

  const int tid = threadIdx.x;
  const int t = WL ? tid % T : tid / kSmallCols;   // position in the column's line
  const int cx = WL ? tid / T : tid % kSmallCols;  // column
  constexpr int SY = WL ? kSyncWave : kSyncBlock;
  const int b = blockIdx.x;
  const long nx = P.nx;
  const bool valid = cx < nx;
  const uint32_t xl = (uint32_t)(valid ? cx : nx - 1);
  const long nvox = (long)N * nx;
  const uint32_t voff = (uint32_t)t * (uint32_t)nx + xl;
  const uint32_t rstep = (uint32_t)T * (uint32_t)nx;
  const uint32_t img_bytes = (uint32_t)(nvox * (long)sizeof(c32));

  for (int i = tid; i < N; i += NT) tw[i] = P.tw[i];
  float mu[E];
  bool sampled[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    mu[j] = P.mu[t + T * j];
    sampled[j] = P.mask_c[t + T * j] != 0;
  }

  const SType* S = static_cast<const SType*>(P.maps) + (long)b * P.maps_bstride;
  const uint32_t coil_bytes = (uint32_t)(nvox * (long)sizeof(SType));
  c32 sm[CR][E];
  if constexpr (MREG) {
#pragma unroll
    for (int c = 0; c < CR; ++c) {
      if (c < P.ncoils) {
        const Buf bs = make_buf(S + (long)c * nvox, coil_bytes);
#pragma unroll
        for (int j = 0; j < E; ++j) sm[c][j] = buf_load_st<ST>(bs, voff, (uint32_t)j * rstep);
      }
    }
  }
  __syncthreads();

  using TwC = TwChoice<N, T, Rad>;
  typename TwC::type twsrc;
  if constexpr (TwC::regs) twsrc.load(tw, t);
  else twsrc.tw = tw;
  const auto lv = SmallView<WL>::template make<LP>(xbuf, cx);

  // b = E^H y from the x rows: per coil the checkerboard-signed masked
  // column (unsampled lines read nothing), inverse transform along y,
  // conj(S) times the signed result summed over the coils, then the scale
  c32 x[E], r[E], p[E], q[E];
  {
    const float sgn = (t & 1) ? -1.f : 1.f;
    c32 acc[E];
#pragma unroll
    for (int j = 0; j < E; ++j) acc[j] = {0.f, 0.f};
    auto adj_coil = [&](int c, const c32* s) {
      const Buf bw = make_buf(P.w + ((long)b * P.ncoils + c) * nvox, img_bytes);
      c32 u[E];
#pragma unroll
      for (int j = 0; j < E; ++j)
        u[j] = cscale(buf_load_c64(bw, sampled[j] ? (voff + (uint32_t)j * rstep) * 8u : kBufOOB, 0), sgn);
      fft_line<N, T, +1, SY>(u, t, twsrc, lv, Rad{});
#pragma unroll
      for (int j = 0; j < E; ++j) acc[j] = cfma_conj(acc[j], s[j], cscale(u[j], sgn));
    };
    if constexpr (MREG) {
#pragma unroll
      for (int c = 0; c < CR; ++c)
        if (c < P.ncoils) adj_coil(c, sm[c]);
    } else {
      for (int c = 0; c < P.ncoils; ++c) {
        const Buf bs = make_buf(S + (long)c * nvox, coil_bytes);
        c32 s[E];
#pragma unroll
        for (int j = 0; j < E; ++j) s[j] = buf_load_st<ST>(bs, voff, (uint32_t)j * rstep);
        adj_coil(c, s);
      }
    }
#pragma unroll
    for (int j = 0; j < E; ++j) r[j] = cscale(acc[j], P.scale);
  }
  double rr = 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    p[j] = r[j];
    x[j] = {0.f, 0.f};
    if (valid) rr += (double)r[j].re * (double)r[j].re + (double)r[j].im * (double)r[j].im;
  }

  double* hist = P.rho_hist ? P.rho_hist + (long)b * P.hist_len : nullptr;
  int par = 0;
  double rho = block_allsum<NT>(rr, slots, par);
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
    if constexpr (MREG) {
#pragma unroll
      for (int c = 0; c < CR; ++c)
        if (c < P.ncoils) coil_term<N, T, SY>(sm[c], p, q, mu, t, twsrc, lv, Rad{});
    } else {
      for (int c = 0; c < P.ncoils; ++c) {
        const Buf bs = make_buf(S + (long)c * nvox, coil_bytes);
        c32 s[E];
#pragma unroll
        for (int j = 0; j < E; ++j) s[j] = buf_load_st<ST>(bs, voff, (uint32_t)j * rstep);
        coil_term<N, T, SY>(s, p, q, mu, t, twsrc, lv, Rad{});
      }
    }
    double pq = 0.0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      q[j] = {q[j].re + P.lambda * p[j].re, q[j].im + P.lambda * p[j].im};
      if (valid) pq += (double)p[j].re * (double)q[j].re + (double)p[j].im * (double)q[j].im;
    }
    const double eta = block_allsum<NT>(pq, slots, par);
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
    const double rho_new = block_allsum<NT>(rr, slots, par);
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

template <int N, int ST>
static void launch_small_st(const SmallParams& P, int batch, hipStream_t st) {
  const dim3 grid((unsigned)batch), block(SmallLen<N>::T * kSmallCols);
  constexpr bool kWaveLines = !(ST == ST_C64 && N == 64);
  if (P.ncoils <= SmallLen<N>::CR)
    hipLaunchKernelGGL((cg_small_kernel<N, ST, true, true>), grid, block, 0, st, P);
  else
    hipLaunchKernelGGL((cg_small_kernel<N, ST, false, kWaveLines>), grid, block, 0, st, P);
}

hipError_t launch_cg_small(const Geom& g, const Tables& tb, const void* maps, const c32* work, c32* x, int K,
                           float lambda, const CgArgs& cg, CgInfo* info, CgInfo* info2, hipStream_t st) {
  if (!small_solve_supported(g)) return hipErrorInvalidValue;
  SmallParams P{};
  P.maps = maps;
  P.w = work;
  P.mask_c = tb.mask_c;
  P.scale = adjoint_scale(g);
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
      switch (g.maps_storage) {
        case ST_C64: launch_small_st<N, ST_C64>(P, g.batch, st); break;
        case ST_BF16: launch_small_st<N, ST_BF16>(P, g.batch, st); break;
        case ST_FP16: launch_small_st<N, ST_FP16>(P, g.batch, st); break;
        default: return;
      }
      err = hipGetLastError();
    }
  });
  return err;
}

}  // namespace sense
