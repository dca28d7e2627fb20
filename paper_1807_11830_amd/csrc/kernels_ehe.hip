// Fused normal operator q = E^H E p + lambda p for 2D Cartesian SENSE.
//
// With a mask that depends on ky only, the centred 2D transforms factor as
// F = F_x (x) F_y and F^H diag(M) F = I_x (x) (F_y^H diag(M_y) F_y).  For even
// Ny the centring shifts are circular shifts by Ny/2, which commute with the
// circulant F_y^H diag(M_y) F_y, so
//     F_y^H diag(M_y) F_y = DFT^-1 diag(M_u / Ny) DFT,  M_u[k] = M_y[(k+Ny/2) mod Ny]
// (DFT unnormalised, DFT^-1 its conjugate transpose).  Hence
//     q[:, x] = sum_c conj(S_c[:, x]) * DFT^-1( (M_u/Ny) * DFT( S_c[:, x] * p[:, x] ) )
// for every readout column x independently: only length-Ny transforms along
// y, no readout transform and no centring signs.  This is the coil product
// and conjugate-sensitivity coil sum of the paper's reconstruction equation
// (Eq. (1)) around a masked forward/inverse transform pair.
//
// One block owns TX adjacent columns of one batch element (coalesced rows of
// TX complex values) and loops over the coils; p, the coil's S column
// segment and the accumulator q stay in registers, and the forward/inverse
// transforms exchange through LDS only between Stockham stages.  The block
// also emits its fp64 partial of Re<p, q> for CG.
#include "bufio.hpp"
#include "cg_scalar.hpp"
#include "kernels.hpp"
#include "lengths.hpp"
#include "reduce.hpp"

namespace sense {


template <int N, int ST, bool CG>
__device__ __forceinline__ void ehe2d_body(const EheParams& P, const int tile, const int b) {
  constexpr int T = EheLen<N>::T;
  constexpr int E = EheLen<N>::E;
  constexpr int TX = EheLen<N>::TX;
  constexpr int NT = T * TX;
  using Rad = typename EheLen<N>::R;
  constexpr int NEX = exchanges(Rad{});

#ifndef SENSE_EHE_SINGLEBUF
#define SENSE_EHE_SINGLEBUF 1
#endif
  constexpr int NBUF = SENSE_EHE_SINGLEBUF ? 1 : 2;
  __shared__ c32 xbuf[NBUF][N * TX];
  __shared__ c32 tw[N];
  __shared__ float mu[N];
  __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];

  const int tid = threadIdx.x;
  const int cx = tid % TX;
  const int t = tid / TX;
  const long x = (long)tile * TX + cx;
  const bool valid = x < P.nx;
  const long nx = P.nx;

  double beta = 0.0;
  if constexpr (CG) {
    if (!cg_iteration_begin(P.state + b, P.rr_part, P.rr_tiles, P.rho_hist, P.hist_len, P.tol, b,
                            tile == 0 && tid == 0, beta))
      return;
  }

  for (int i = tid; i < N; i += NT) {
    tw[i] = P.tw[i];
    mu[i] = P.mu[i];
  }

  // Element (row, column) of a batch element's image sits at row * nx + col.
  // Columns past nx (ragged last tile) read column nx-1 instead of
  // branching; their results are never stored or reduced.
  const long nvox = (long)N * nx;
  const uint32_t xl = (uint32_t)(valid ? x : nx - 1);
  const uint32_t voff = (uint32_t)t * (uint32_t)nx + xl;  // element offset of row t
  const uint32_t rstep = (uint32_t)T * (uint32_t)nx;      // rows t -> t + T
  const uint32_t img_bytes = (uint32_t)(nvox * (long)sizeof(c32));
  const Buf bq = make_buf(P.q + (long)b * nvox, img_bytes);
  c32 p[E], q[E];
  {
    const Buf bp = make_buf(P.p_in + (long)b * nvox, img_bytes);
    [[maybe_unused]] Buf br, bpo;
    if constexpr (CG) {
      br = make_buf(P.r + (long)b * nvox, img_bytes);
      bpo = make_buf(P.p_out + (long)b * nvox, img_bytes);
    }
#pragma unroll
    for (int j = 0; j < E; ++j) {
      c32 v = buf_load_c64(bp, voff * 8u, (uint32_t)j * rstep * 8u);
      if constexpr (CG) {
        const c32 rv = buf_load_c64(br, voff * 8u, (uint32_t)j * rstep * 8u);
        v = {(float)((double)rv.re + beta * (double)v.re),
             (float)((double)rv.im + beta * (double)v.im)};
        if (valid) buf_store_c64(bpo, v, voff * 8u, (uint32_t)j * rstep * 8u);
      }
      p[j] = v;
      q[j] = {0.f, 0.f};
    }
  }
  __syncthreads();

  using TwC = TwChoice<N, T, Rad>;
  typename TwC::type twsrc;
  if constexpr (TwC::regs) twsrc.load(tw, t);
  else twsrc.tw = tw;

  using SType = typename StorageT<ST>::T;
  const SType* S = static_cast<const SType*>(P.maps) + (long)b * P.maps_bstride;
  const uint32_t coil_bytes = (uint32_t)(nvox * (long)sizeof(SType));
  LineView<TX> v0{&xbuf[0][cx]}, v1{&xbuf[NBUF - 1][cx]};

  auto load_s = [&](c32* s, int c) {
    const Buf bs = make_buf(S + (long)c * nvox, coil_bytes);
#pragma unroll
    for (int j = 0; j < E; ++j) s[j] = buf_load_st<ST>(bs, voff, (uint32_t)j * rstep);
  };
  // One coil: u = S p, forward transform, mask, inverse transform,
  // q += conj(S) u.  The transform pair uses an even number of exchanges,
  // so every coil starts on LDS buffer 0.
  auto coil = [&](const c32* s) {
    c32 u[E];
#pragma unroll
    for (int j = 0; j < E; ++j) u[j] = cmul(s[j], p[j]);
    if constexpr (NBUF == 1) fft_line_sb<N, T, -1>(u, t, twsrc, v0, Rad{});
    else fft_line<N, T, -1, 0>(u, t, twsrc, v0, v1, Rad{});
#pragma unroll
    for (int j = 0; j < E; ++j) u[j] = cscale(u[j], mu[t + T * j]);
    if constexpr (NBUF == 1) fft_line_sb<N, T, +1>(u, t, twsrc, v0, Rad{});
    else fft_line<N, T, +1, NEX & 1>(u, t, twsrc, v0, v1, Rad{});
#pragma unroll
    for (int j = 0; j < E; ++j) q[j] = cfma_conj(q[j], s[j], u[j]);
  };

#ifndef SENSE_EHE_PREFETCH
#define SENSE_EHE_PREFETCH 0
#endif
  const int C = P.ncoils;
#if SENSE_EHE_PREFETCH
  // Maps of coil c+1 are loaded while coil c is transformed.
  c32 sc[E], sn[E];
  load_s(sc, 0);
  for (int c = 0; c < C; ++c) {
    if (c + 1 < C) load_s(sn, c + 1);
    coil(sc);
#pragma unroll
    for (int j = 0; j < E; ++j) sc[j] = sn[j];
  }
#else
  for (int c = 0; c < C; ++c) {
    c32 sc[E];
    load_s(sc, c);
    coil(sc);
  }
#endif

  double eta = 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    c32 qq = {q[j].re + P.lambda * p[j].re, q[j].im + P.lambda * p[j].im};
    if (valid) {
      buf_store_c64(bq, qq, voff * 8u, (uint32_t)j * rstep * 8u);
      eta += (double)p[j].re * (double)qq.re + (double)p[j].im * (double)qq.im;
    }
  }
  if (P.eta_part) {
    const double tot = block_sum<NT>(eta, red);
    if (tid == 0) P.eta_part[(long)b * P.ntiles + tile] = tot;
  }
}

template <int N, int ST, bool CG>
__global__ void __launch_bounds__(EheLen<N>::T * EheLen<N>::TX) ehe2d_kernel(EheParams P) {
  ehe2d_body<N, ST, CG>(P, blockIdx.x, blockIdx.y);
}

// Batched CG launch over many independent single-slice problems of the same
// ny: block row blockIdx.y runs the problem described by table[blockIdx.y]
// (its own maps, vectors, partials and CG state), so every problem computes
// exactly what its own launch would.
template <int N, int ST>
__global__ void __launch_bounds__(EheLen<N>::T * EheLen<N>::TX)
    ehe2d_table_kernel(const EheParams* __restrict__ table) {
  const EheParams P = table[blockIdx.y];
  if ((long)blockIdx.x >= (long)P.ntiles) return;
  ehe2d_body<N, ST, true>(P, blockIdx.x, 0);
}

int ehe_tile_width(long ny) {
  int tx = 0;
  dispatch_length(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    tx = EheLen<N>::TX;
  });
  return tx;
}

template <bool CG>
static hipError_t launch_ehe_impl(const Geom& g, const Tables& tb, EheParams P, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  P.tw = tb.tw_y;
  P.mu = tb.mu_y;
  P.nx = g.nx;
  P.ntiles = (int)((g.nx + ehe_tile_width(g.ny) - 1) / ehe_tile_width(g.ny));
  P.maps_bstride = g.maps_bstride;
  P.ncoils = g.ncoils;
  dispatch_length(g.ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    constexpr int T = EheLen<N>::T;
    constexpr int TX = EheLen<N>::TX;
    dim3 grid((unsigned)((g.nx + TX - 1) / TX), (unsigned)g.batch);
    dim3 block(T * TX);
    switch (g.maps_storage) {
      case ST_C64: hipLaunchKernelGGL((ehe2d_kernel<N, ST_C64, CG>), grid, block, 0, st, P); break;
      case ST_BF16: hipLaunchKernelGGL((ehe2d_kernel<N, ST_BF16, CG>), grid, block, 0, st, P); break;
      case ST_FP16: hipLaunchKernelGGL((ehe2d_kernel<N, ST_FP16, CG>), grid, block, 0, st, P); break;
      default: return;
    }
    err = hipGetLastError();
  });
  return err;
}

void fill_ehe_cg_params(const Geom& g, const Tables& tb, const void* maps, const c32* r, c32* p, c32* q,
                        float lambda, const CgArgs& cg, EheParams* out) {
  EheParams P{};
  P.maps = maps;
  P.r = r;
  P.p_in = p;
  P.p_out = p;
  P.q = q;
  P.lambda = lambda;
  P.eta_part = cg.eta_part;
  P.state = cg.state;
  P.rr_part = cg.rr_part;
  P.rr_tiles = cg.rr_tiles;
  P.rho_hist = cg.rho_hist;
  P.hist_len = cg.hist_len;
  P.tol = cg.tol;
  P.tw = tb.tw_y;
  P.mu = tb.mu_y;
  P.nx = g.nx;
  P.ntiles = (int)((g.nx + ehe_tile_width(g.ny) - 1) / ehe_tile_width(g.ny));
  P.maps_bstride = g.maps_bstride;
  P.ncoils = g.ncoils;
  *out = P;
}

hipError_t launch_ehe_table(long ny, int maps_storage, const EheParams* d_table, int nproblems, int max_tiles,
                            hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  dispatch_length(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    dim3 grid((unsigned)max_tiles, (unsigned)nproblems);
    dim3 block(EheLen<N>::T * EheLen<N>::TX);
    switch (maps_storage) {
      case ST_C64: hipLaunchKernelGGL((ehe2d_table_kernel<N, ST_C64>), grid, block, 0, st, d_table); break;
      case ST_BF16: hipLaunchKernelGGL((ehe2d_table_kernel<N, ST_BF16>), grid, block, 0, st, d_table); break;
      case ST_FP16: hipLaunchKernelGGL((ehe2d_table_kernel<N, ST_FP16>), grid, block, 0, st, d_table); break;
      default: return;
    }
    err = hipGetLastError();
  });
  return err;
}

hipError_t launch_ehe(const Geom& g, const Tables& tb, const void* maps, const c32* p, c32* q,
                      float lambda, double* eta_part, hipStream_t st) {
  EheParams P{};
  P.maps = maps;
  P.p_in = p;
  P.q = q;
  P.lambda = lambda;
  P.eta_part = eta_part;
  return launch_ehe_impl<false>(g, tb, P, st);
}

hipError_t launch_ehe_cg(const Geom& g, const Tables& tb, const void* maps, const c32* r, c32* p,
                         c32* q, float lambda, const CgArgs& cg, hipStream_t st) {
  EheParams P{};
  P.maps = maps;
  P.r = r;
  P.p_in = p;
  P.p_out = p;
  P.q = q;
  P.lambda = lambda;
  P.eta_part = cg.eta_part;
  P.state = cg.state;
  P.rr_part = cg.rr_part;
  P.rr_tiles = cg.rr_tiles;
  P.rho_hist = cg.rho_hist;
  P.hist_len = cg.hist_len;
  P.tol = cg.tol;
  return launch_ehe_impl<true>(g, tb, P, st);
}

}  // namespace sense
