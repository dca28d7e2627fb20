// Full-grid forward operator E and adjoint E^H for 2D Cartesian SENSE.
//
//   E:   y_c = M .* F(S_c .* x)            F = centred unitary 2D DFT
//   E^H: x   = sum_c conj(S_c) .* F^H(M .* y_c)
//
// E^H with a full mask is the paper's reconstruction equation (Eq. (1)):
// inverse transform of every coil's k-space, product with the conjugate
// sensitivity, and a sum over the coils of the same frame.  Here the coil
// product and the coil sum are fused into the column pass of the inverse
// transform so x is written once.
//
// For even N the centred transform is F_c v = (-1)^(N/2) (-1)^k DFT((-1)^n v) / sqrt(N)
// (fftshift/ifftshift are circular shifts by N/2).  Each thread holds the
// positions t + T*j of a line with T even, so both checkerboards reduce to
// the factor (-1)^t per thread; the global (-1)^(N/2)/sqrt(N) of both axes
// is one scalar applied at the last store.
//
// Passes (W = plan workspace, c64, [B][C][Ny][Nx]):
//   E:   column pass  W = mask_y( F_y( S_c .* x ) )      (sampled rows only stored)
//        row pass     y = scale * F_x( W )               (sampled rows; others zero)
//   E^H: row pass     W = F_x^H( y )                     (sampled rows only)
//        column pass  x = scale * sum_c conj(S_c) .* F_y^H( mask_y(W_c) )
#include "kernels.hpp"
#include "lengths.hpp"

#include <cmath>

namespace sense {

constexpr int ROW_NT = 256;

struct RowParams {
  const void* in;
  void* out;
  const int32_t* rows;  // sampled row ids (z * ny + y), count nrows
  int nrows;
  long lines;           // nbc * nrows
  long rows_total;      // ny * nz
  long nx;
  const c32* tw;
  float scale;
};

template <int N, int DIR, int ST_IN, int ST_OUT>
__global__ void __launch_bounds__(ROW_NT) row_fft_kernel(RowParams P) {
  constexpr int T = Len<N>::T;
  constexpr int E = Len<N>::E;
  constexpr int TR = ROW_NT / T;
  constexpr int LDL = N + 1;
  using Rad = typename Len<N>::R;
  __shared__ c32 buf[2][TR * LDL];
  __shared__ c32 tw[N];

  const int tid = threadIdx.x;
  const int t = tid % T;
  const int l = tid / T;
  const long L = (long)blockIdx.x * TR + l;
  const bool valid = L < P.lines;
  for (int i = tid; i < N; i += ROW_NT) tw[i] = P.tw[i];

  long off = 0;
  if (valid) {
    const long bc = L / P.nrows;
    const long row = P.rows[L % P.nrows];
    off = (bc * P.rows_total + row) * P.nx;
  }
  using TI = typename StorageT<ST_IN>::T;
  using TO = typename StorageT<ST_OUT>::T;
  const TI* in = static_cast<const TI*>(P.in) + off;
  const float sgn = (t & 1) ? -1.f : 1.f;
  c32 v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = valid ? cscale(load_c<ST_IN>(in, t + T * j), sgn) : c32{0.f, 0.f};
  __syncthreads();
  LineView<1> b0{&buf[0][l * LDL]}, b1{&buf[1][l * LDL]};
  fft_line<N, T, DIR, 0>(v, t, TwTable{tw}, b0, b1, Rad{});
  if (valid) {
    TO* out = static_cast<TO*>(P.out) + off;
    const float s = sgn * P.scale;
#pragma unroll
    for (int j = 0; j < E; ++j) store_c<ST_OUT>(out, t + T * j, cscale(v[j], s));
  }
}

// Zero the listed rows of every (b, c) image (E writes zeros off the mask).
// One block per line.
template <int ST>
__global__ void zero_rows_kernel(void* out, const int32_t* rows, int nrows, long rows_total, long nx) {
  using TO = typename StorageT<ST>::T;
  const long L = blockIdx.x;
  const long bc = L / nrows;
  const long row = rows[L % nrows];
  TO* o = static_cast<TO*>(out) + (bc * rows_total + row) * nx;
  for (long i = threadIdx.x; i < nx; i += blockDim.x) store_c<ST>(o, i, c32{0.f, 0.f});
}

struct ColParams {
  const void* maps;
  const c32* x;       // E: image
  c32* w;             // workspace
  c32* xout;          // E^H: image
  const uint8_t* mask;
  const c32* tw;
  long nx;
  long maps_bstride;
  int ncoils;
  float scale;
};

// E column pass: one block per (x tile, coil, batch element).
template <int N, int ST>
__global__ void __launch_bounds__(Len<N>::T * col_tile<Len<N>::T>()) col_fwd_kernel(ColParams P) {
  constexpr int T = Len<N>::T;
  constexpr int E = Len<N>::E;
  constexpr int TX = col_tile<T>();
  constexpr int NT = T * TX;
  using Rad = typename Len<N>::R;
  __shared__ c32 buf[2][N * TX];
  __shared__ c32 tw[N];
  const int tid = threadIdx.x, cx = tid % TX, t = tid / TX;
  const long x = (long)blockIdx.x * TX + cx;
  const int c = blockIdx.y, b = blockIdx.z;
  const bool valid = x < P.nx;
  const long nx = P.nx;
  for (int i = tid; i < N; i += NT) tw[i] = P.tw[i];

  using SType = typename StorageT<ST>::T;
  const SType* S = static_cast<const SType*>(P.maps) + (long)b * P.maps_bstride + (long)c * N * nx + x;
  const c32* X = P.x + (long)b * N * nx + x;
  const float sgn = (t & 1) ? -1.f : 1.f;
  c32 u[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const long o = (long)(t + T * j) * nx;
    u[j] = valid ? cscale(cmul(load_c<ST>(S, o), X[o]), sgn) : c32{0.f, 0.f};
  }
  __syncthreads();
  LineView<TX> b0{&buf[0][cx]}, b1{&buf[1][cx]};
  fft_line<N, T, -1, 0>(u, t, TwTable{tw}, b0, b1, Rad{});
  if (valid) {
    c32* W = P.w + ((long)b * P.ncoils + c) * N * nx + x;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = t + T * j;
      if (P.mask[k]) W[(long)k * nx] = cscale(u[j], sgn);
    }
  }
}

// E^H column pass: one block per (x tile, batch element), coils summed in
// increasing order in registers.
template <int N, int ST>
__global__ void __launch_bounds__(Len<N>::T * col_tile<Len<N>::T>()) col_adj_kernel(ColParams P) {
  constexpr int T = Len<N>::T;
  constexpr int E = Len<N>::E;
  constexpr int TX = col_tile<T>();
  constexpr int NT = T * TX;
  constexpr int NEX = exchanges(typename Len<N>::R{});
  using Rad = typename Len<N>::R;
  __shared__ c32 buf[2][N * TX];
  __shared__ c32 tw[N];
  const int tid = threadIdx.x, cx = tid % TX, t = tid / TX;
  const long x = (long)blockIdx.x * TX + cx;
  const int b = blockIdx.y;
  const bool valid = x < P.nx;
  const long nx = P.nx;
  for (int i = tid; i < N; i += NT) tw[i] = P.tw[i];
  __syncthreads();

  using SType = typename StorageT<ST>::T;
  const SType* S = static_cast<const SType*>(P.maps) + (long)b * P.maps_bstride + x;
  const c32* W = P.w + (long)b * P.ncoils * N * nx + x;
  const float sgn = (t & 1) ? -1.f : 1.f;
  LineView<TX> b0{&buf[0][cx]}, b1{&buf[1][cx]};
  c32 acc[E];
#pragma unroll
  for (int j = 0; j < E; ++j) acc[j] = {0.f, 0.f};
  for (int c = 0; c < P.ncoils; ++c) {
    const c32* Wc = W + (long)c * N * nx;
    c32 u[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = t + T * j;
      u[j] = (valid && P.mask[k]) ? cscale(Wc[(long)k * nx], sgn) : c32{0.f, 0.f};
    }
    // the two exchange buffers alternate across coils: an even number of
    // exchanges per coil keeps the start buffer fixed
    if constexpr ((NEX & 1) == 0) {
      fft_line<N, T, +1, 0>(u, t, TwTable{tw}, b0, b1, Rad{});
    } else {
      if (c & 1) fft_line<N, T, +1, 1>(u, t, TwTable{tw}, b0, b1, Rad{});
      else fft_line<N, T, +1, 0>(u, t, TwTable{tw}, b0, b1, Rad{});
    }
    const SType* Sc = S + (long)c * N * nx;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const c32 s = valid ? load_c<ST>(Sc, (long)(t + T * j) * nx) : c32{0.f, 0.f};
      acc[j] = cfma_conj(acc[j], s, cscale(u[j], sgn));
    }
  }
  if (valid) {
    c32* X = P.xout + (long)b * N * nx + x;
#pragma unroll
    for (int j = 0; j < E; ++j) X[(long)(t + T * j) * nx] = cscale(acc[j], P.scale);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int DIR, int ST_IN, int ST_OUT>
static hipError_t launch_rows(const Geom& g, const c32* tw, const void* in, void* out,
                              const int32_t* rows, int nrows, float scale, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  RowParams P{};
  P.in = in;
  P.out = out;
  P.rows = rows;
  P.nrows = nrows;
  P.lines = (long)g.batch * g.ncoils * nrows;
  P.rows_total = g.ny * g.nz;
  P.nx = g.nx;
  P.tw = tw;
  P.scale = scale;
  hipError_t err = hipErrorInvalidValue;
  dispatch_length(g.nx, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    constexpr int TR = ROW_NT / Len<N>::T;
    dim3 grid((unsigned)((P.lines + TR - 1) / TR));
    hipLaunchKernelGGL((row_fft_kernel<N, DIR, ST_IN, ST_OUT>), grid, dim3(ROW_NT), 0, st, P);
    err = hipGetLastError();
  });
  return err;
}

template <int ST>
static hipError_t launch_zero_rows(const Geom& g, void* out, const int32_t* rows, int nrows,
                                   hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  const long lines = (long)g.batch * g.ncoils * nrows;
  hipLaunchKernelGGL((zero_rows_kernel<ST>), dim3((unsigned)lines), dim3(256), 0, st, out, rows,
                     nrows, g.ny * g.nz, g.nx);
  return hipGetLastError();
}

// (-1)^(nx/2 + ny/2) / sqrt(nx ny): the global factor of the centred unitary
// 2D transform in checkerboard form (both directions).
static float centred_scale(long nx, long ny) {
  const long h = (nx / 2 + ny / 2) & 1;
  return (float)((h ? -1.0 : 1.0) / std::sqrt((double)nx * (double)ny));
}

template <int STM>
static hipError_t launch_col_fwd(const Geom& g, ColParams P, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  dispatch_length(g.ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    constexpr int TX = col_tile<Len<N>::T>();
    dim3 grid((unsigned)((g.nx + TX - 1) / TX), (unsigned)g.ncoils, (unsigned)g.batch);
    hipLaunchKernelGGL((col_fwd_kernel<N, STM>), grid, dim3(Len<N>::T * TX), 0, st, P);
    err = hipGetLastError();
  });
  return err;
}

template <int STM>
static hipError_t launch_col_adj(const Geom& g, ColParams P, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  dispatch_length(g.ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    constexpr int TX = col_tile<Len<N>::T>();
    dim3 grid((unsigned)((g.nx + TX - 1) / TX), (unsigned)g.batch);
    hipLaunchKernelGGL((col_adj_kernel<N, STM>), grid, dim3(Len<N>::T * TX), 0, st, P);
    err = hipGetLastError();
  });
  return err;
}

hipError_t launch_E(const Geom& g, const Tables& tb, const void* maps, const c32* x, c32* work,
                    void* y, hipStream_t st) {
  if (g.nz != 1) return hipErrorInvalidValue;
  ColParams P{};
  P.maps = maps;
  P.x = x;
  P.w = work;
  P.mask = tb.mask_c;
  P.tw = tb.tw_y;
  P.nx = g.nx;
  P.maps_bstride = g.maps_bstride;
  P.ncoils = g.ncoils;
  P.scale = 1.f;
  hipError_t err = hipErrorInvalidValue;
  switch (g.maps_storage) {
    case ST_C64: err = launch_col_fwd<ST_C64>(g, P, st); break;
    case ST_BF16: err = launch_col_fwd<ST_BF16>(g, P, st); break;
    case ST_FP16: err = launch_col_fwd<ST_FP16>(g, P, st); break;
  }
  if (err != hipSuccess) return err;
  const float sc = centred_scale(g.nx, g.ny);
  switch (g.kspace_storage) {
    case ST_C64:
      err = launch_rows<-1, ST_C64, ST_C64>(g, tb.tw_x, work, y, tb.rows_s, tb.n_rows_s, sc, st);
      if (err == hipSuccess) err = launch_zero_rows<ST_C64>(g, y, tb.rows_u, tb.n_rows_u, st);
      break;
    case ST_BF16:
      err = launch_rows<-1, ST_C64, ST_BF16>(g, tb.tw_x, work, y, tb.rows_s, tb.n_rows_s, sc, st);
      if (err == hipSuccess) err = launch_zero_rows<ST_BF16>(g, y, tb.rows_u, tb.n_rows_u, st);
      break;
    case ST_FP16:
      err = launch_rows<-1, ST_C64, ST_FP16>(g, tb.tw_x, work, y, tb.rows_s, tb.n_rows_s, sc, st);
      if (err == hipSuccess) err = launch_zero_rows<ST_FP16>(g, y, tb.rows_u, tb.n_rows_u, st);
      break;
    default: err = hipErrorInvalidValue;
  }
  return err;
}

hipError_t launch_EH(const Geom& g, const Tables& tb, const void* maps, const void* y, c32* work,
                     c32* x, hipStream_t st) {
  if (g.nz != 1) return hipErrorInvalidValue;
  hipError_t err = hipErrorInvalidValue;
  switch (g.kspace_storage) {
    case ST_C64: err = launch_rows<+1, ST_C64, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st); break;
    case ST_BF16: err = launch_rows<+1, ST_BF16, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st); break;
    case ST_FP16: err = launch_rows<+1, ST_FP16, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st); break;
  }
  if (err != hipSuccess) return err;
  ColParams P{};
  P.maps = maps;
  P.w = work;
  P.xout = x;
  P.mask = tb.mask_c;
  P.tw = tb.tw_y;
  P.nx = g.nx;
  P.maps_bstride = g.maps_bstride;
  P.ncoils = g.ncoils;
  P.scale = centred_scale(g.nx, g.ny);
  switch (g.maps_storage) {
    case ST_C64: return launch_col_adj<ST_C64>(g, P, st);
    case ST_BF16: return launch_col_adj<ST_BF16>(g, P, st);
    case ST_FP16: return launch_col_adj<ST_FP16>(g, P, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace sense
