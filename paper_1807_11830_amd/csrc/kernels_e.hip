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
#include "bufio.hpp"
#include "kernels.hpp"
#include "lengths.hpp"
#include "reduce.hpp"
#include "xcd.hpp"

#include <algorithm>
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
  int compact_in, compact_out;  // that side holds only the listed rows, in list order
};

template <int N, int DIR, int ST_IN, int ST_OUT>
__global__ void __launch_bounds__(ROW_NT) row_fft_kernel(RowParams P) {
  constexpr int T = Len<N>::T;
  constexpr int E = Len<N>::E;
  constexpr int TR = ROW_NT / T;
  constexpr int LDL = padded_line<N>();
  using Rad = typename Len<N>::R;
  __shared__ c32 buf[TR * LDL];
  __shared__ c32 tw[N];

  const int tid = threadIdx.x;
  const int t = tid % T;
  const int l = tid / T;
  const long L = (long)xcd_order(blockIdx.x, gridDim.x) * TR + l;
  const bool valid = L < P.lines;
  for (int i = tid; i < N; i += ROW_NT) tw[i] = P.tw[i];

  long off_in = 0, off_out = 0;
  if (valid) {
    const long bc = L / P.nrows;
    const long li = L % P.nrows;
    const long full = (bc * P.rows_total + P.rows[li]) * P.nx;
    const long compact = (bc * P.nrows + li) * P.nx;
    off_in = P.compact_in ? compact : full;
    off_out = P.compact_out ? compact : full;
  }
  using TI = typename StorageT<ST_IN>::T;
  using TO = typename StorageT<ST_OUT>::T;
  const TI* in = static_cast<const TI*>(P.in) + off_in;
  const float sgn = (t & 1) ? -1.f : 1.f;
  c32 v[E];
#pragma unroll
  // unconditional loads (a line past the end reads the buffer's first line,
  // never stored): a per-element branch would serialise the loads
  for (int j = 0; j < E; ++j) v[j] = cscale(load_c<ST_IN>(in, t + T * j), sgn);
  __syncthreads();
  PadLineView lv{&buf[l * LDL]};
  // a line's T threads are consecutive lanes of one wave (T divides 64):
  // its stage exchanges need no block barrier
  static_assert(64 % T == 0, "a row line must sit inside one wavefront");
  fft_line<N, T, DIR, kSyncWave>(v, t, TwTable{tw}, lv, Rad{});
  if (valid) {
    TO* out = static_cast<TO*>(P.out) + off_out;
    const float s = sgn * P.scale;
#pragma unroll
    for (int j = 0; j < E; ++j) store_c<ST_OUT>(out, t + T * j, cscale(v[j], s));
  }
}

// Zero the listed rows of every (b, c) image (E writes zeros off the mask).
// 16-byte streaming stores over (line, chunk) pairs, grid-stride: every
// supported nx makes a line a whole number of 16-byte chunks, and the
// launcher takes this path only for a 16-byte aligned k-space base.  The
// zeros are written once and not read back by this operator, so they are
// streamed past the caches.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) zero_rows16_kernel(char* out, const int32_t* rows, int nrows,
                                                          long rows_total, long line_bytes, long lines) {
  const long cpl = line_bytes / 16;
  const long total = lines * cpl;
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
    const long L = i / cpl, ch = i % cpl;
    const long bc = L / nrows;
    const long row = rows[L % nrows];
    __builtin_nontemporal_store(z, reinterpret_cast<u32x4*>(out + (bc * rows_total + row) * line_bytes + ch * 16));
  }
}

// The same with one element per store, for a k-space base that is not
// 16-byte aligned.  One block per line.
template <int ST>
__global__ void zero_rows_kernel(void* out, const int32_t* rows, int nrows, long rows_total, long nx) {
  using TO = typename StorageT<ST>::T;
  const long L = blockIdx.x;
  const long bc = L / nrows;
  const long row = rows[L % nrows];
  TO* o = static_cast<TO*>(out) + (bc * rows_total + row) * nx;
  for (long i = threadIdx.x; i < nx; i += blockDim.x) store_c<ST>(o, i, c32{0.f, 0.f});
}

// Column passes: transforms along y (element stride nx) or z (stride nx*ny)
// for TX adjacent x columns per block.  Modes:
//   FWD_COIL  u = S_c .* X, forward transform, optional mask, store W[b][c]
//   FWD       forward transform of W in place, optional mask
//   ADJ       optional masked load, inverse transform of W in place
//   ADJ_COIL  for every coil: optional masked load of W[b][c], inverse
//             transform, accumulate conj(S_c) .* u; store X[b] (+ lambda p,
//             fp64 partial Re<p, X> for CG)
//   PROJ      F^H diag(M) F of W in place along z (the (ky, kz) mask of the
//             current ky plane): the middle of the 3D normal operator
enum ColMode : int { CM_FWD_COIL = 0, CM_FWD = 1, CM_ADJ = 2, CM_ADJ_COIL = 3, CM_PROJ = 4 };

struct ColPass {
  const void* maps;
  const c32* src;
  c32* dst;
  const c32* addp;     // ADJ_COIL: p for lambda p and eta (may be null)
  double* eta_part;    // ADJ_COIL: [b][gridDim.x * gridDim.y] (may be null)
  double* zeta_part;   // ADJ_COIL: <q, q> partials, same layout (may be null)
  const uint8_t* mask; // centred [nz][ny]
  const c32* tw;
  long nx, ny, nz;
  long maps_bstride;
  int ncoils;
  int mask_store;
  int mask_load;
  float scale;
  float lambda;
  // ADJ_COIL / RSS coil groups: with ngroups > 1 grid z is batch x groups,
  // and each block writes its group's partial sum to part[g][b] (complex
  // for ADJ_COIL, real for RSS) for a combine pass
  void* part;
  long part_gstride;  // elements between groups (batch * nvox)
  int ngroups;
};

// Columns per block of a pass along AXIS.  Along z consecutive rows of a
// column are a whole x-y plane apart, so each row segment is its own DRAM
// page: wider segments (32 columns, 256 bytes) where the block stays within
// 256 threads.
template <int T, int AXIS>
constexpr int pass_tile() {
  return (AXIS == 2 && T * 32 <= 256) ? 32 : col_tile<T>();
}

// STREAM: the launch's data is read or written once and far exceeds the
// caches, so whole-line accesses take the streaming policy (bufio.hpp); the
// image X of the forward coil pass is read once per coil and keeps the
// default policy.
template <int N, int AXIS, int MODE, int ST, bool STREAM>
__global__ void __launch_bounds__((Len<N>::T * pass_tile<Len<N>::T, AXIS>())) colpass_kernel(ColPass P) {
  constexpr int T = Len<N>::T;
  constexpr int E = Len<N>::E;
  constexpr int TX = pass_tile<T, AXIS>();
  constexpr int NT = T * TX;
  using Rad = typename Len<N>::R;
  using SType0 = typename StorageT<ST>::T;
  constexpr int CPW = stream_policy<STREAM, TX * 8>();                      // complex64 data
  constexpr int CPS = stream_policy<STREAM, TX * (int)sizeof(SType0)>();  // maps
  __shared__ c32 buf[N * TX];
  __shared__ c32 tw[N];
  __shared__ uint8_t msk[N];  // the mask along this pass's line
  __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];

  const int tid = threadIdx.x, cx = tid % TX, t = tid / TX;
  const long nx = P.nx, ny = P.ny;
  const BlockId id = xcd_block();
  const long x = (long)id.x * TX + cx;
  const bool valid = x < nx;
  const uint32_t xl = (uint32_t)(valid ? x : nx - 1);
  const long pl = id.y;  // z for AXIS 1, y for AXIS 2
  const long nvox = nx * ny * P.nz;
  const uint32_t es = (uint32_t)(AXIS == 1 ? nx : nx * ny);
  const uint32_t lbase = (uint32_t)(AXIS == 1 ? pl * ny * nx : pl * nx) + xl;
  const uint32_t voff = lbase + (uint32_t)t * es;
  const uint32_t rstep = (uint32_t)T * es;
  const uint32_t vbytes = (uint32_t)(nvox * 8);
  // The mask along the line is staged in LDS once, so masked loads and
  // stores never wait on a global byte load (which would also wait for
  // every data load issued before it).
  for (int i = tid; i < N; i += NT) {
    tw[i] = P.tw[i];
    msk[i] = P.mask ? (AXIS == 1 ? P.mask[pl * ny + i] : P.mask[(long)i * ny + pl]) : 1;
  }
  auto mask_at = [&](int k) -> bool { return msk[k] != 0; };
  __syncthreads();

  using SType = typename StorageT<ST>::T;
  const float sgn = (t & 1) ? -1.f : 1.f;
  LineView<TX> lv{&buf[cx]};
  const TwTable twt{tw};

  if constexpr (MODE != CM_ADJ_COIL) {
    const long bc = id.z;
    const long b = bc / P.ncoils, c = bc % P.ncoils;
    c32 u[E];
    if constexpr (MODE == CM_FWD_COIL) {
      const Buf bs = make_buf(static_cast<const SType*>(P.maps) + b * P.maps_bstride + c * nvox,
                              (uint32_t)(nvox * sizeof(SType)));
      const Buf bx = make_buf(P.src + b * nvox, vbytes);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const uint32_t o = voff + (uint32_t)j * rstep;
        u[j] = cscale(cmul(buf_load_st<ST, CPS>(bs, o, 0), buf_load_c64(bx, o * 8u, 0)), sgn);
      }
    } else {
      const Buf bw = make_buf(P.src + bc * nvox, vbytes);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        // masked-out lines are not read at all: an out-of-range offset
        // returns zero without a memory request, and without a branch that
        // would serialise the loads
        const bool on = MODE == CM_ADJ && P.mask_load ? mask_at(t + T * j) : true;
        const uint32_t o = on ? (voff + (uint32_t)j * rstep) * 8u : kBufOOB;
        u[j] = cscale(buf_load_c64<CPW>(bw, o, 0), sgn);
      }
    }
    if constexpr (MODE == CM_ADJ) {
      fft_line<N, T, +1>(u, t, twt, lv, Rad{});
    } else if constexpr (MODE == CM_PROJ) {
      static_assert(AXIS == 2, "the projector runs along z");
      fft_line<N, T, -1>(u, t, twt, lv, Rad{});
      // checkerboards of the forward output and inverse input cancel
#pragma unroll
      for (int j = 0; j < E; ++j)
        if (!mask_at(t + T * j)) u[j] = {0.f, 0.f};
      fft_line<N, T, +1>(u, t, twt, lv, Rad{});
    } else {
      fft_line<N, T, -1>(u, t, twt, lv, Rad{});
    }
    if (valid) {
      const Buf bd = make_buf(P.dst + bc * nvox, vbytes);
      const float sc = sgn * P.scale;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const bool on = (MODE == CM_FWD_COIL || MODE == CM_FWD) && P.mask_store ? mask_at(t + T * j) : true;
        if (on) buf_store_c64<CPW>(bd, cscale(u[j], sc), (voff + (uint32_t)j * rstep) * 8u, 0);
      }
    }
  } else {
    const int G = P.ngroups;
    const long b = id.z / G;
    const int grp = (int)(id.z % G);
    const int c0 = (int)((long)grp * P.ncoils / G), c1 = (int)((long)(grp + 1) * P.ncoils / G);
    c32 acc[E];
#pragma unroll
    for (int j = 0; j < E; ++j) acc[j] = {0.f, 0.f};
    for (int c = c0; c < c1; ++c) {
      const Buf bw = make_buf(P.src + (b * P.ncoils + c) * nvox, vbytes);
      const Buf bs = make_buf(static_cast<const SType*>(P.maps) + b * P.maps_bstride + (long)c * nvox,
                              (uint32_t)(nvox * sizeof(SType)));
      c32 u[E];
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const bool on = P.mask_load ? mask_at(t + T * j) : true;
        const uint32_t o = on ? (voff + (uint32_t)j * rstep) * 8u : kBufOOB;
        u[j] = cscale(buf_load_c64<CPW>(bw, o, 0), sgn);
      }
      // the coil's maps are loaded before the transform so their latency
      // hides behind it (measured 16% faster for 256^2 x 12 coils x 160
      // slices than loading them after it, at one wave less per SIMD)
      c32 sv[E];
#pragma unroll
      for (int j = 0; j < E; ++j) sv[j] = buf_load_st<ST, CPS>(bs, voff + (uint32_t)j * rstep, 0);
      fft_line<N, T, +1>(u, t, twt, lv, Rad{});
#pragma unroll
      for (int j = 0; j < E; ++j) acc[j] = cfma_conj(acc[j], sv[j], cscale(u[j], sgn));
    }
    if (G > 1) {
      // this group's partial coil sum (scaled); the combine pass adds them
      if (valid) {
        const Buf bg = make_buf(static_cast<c32*>(P.part) + grp * P.part_gstride + b * nvox, vbytes);
#pragma unroll
        for (int j = 0; j < E; ++j) buf_store_c64<CPW>(bg, cscale(acc[j], P.scale), (voff + (uint32_t)j * rstep) * 8u, 0);
      }
      return;
    }
    const Buf bd = make_buf(P.dst + b * nvox, vbytes);
    double eta = 0.0, zeta = 0.0;
    // p for lambda p and Re<p, q>: all loads first (an out-of-range offset
    // when there is no p), so no wait falls between two of them
    const Buf bp = make_buf(P.addp ? P.addp + b * nvox : P.dst, vbytes);
    c32 pv[E];
#pragma unroll
    for (int j = 0; j < E; ++j) pv[j] = buf_load_c64<CPW>(bp, P.addp ? (voff + (uint32_t)j * rstep) * 8u : kBufOOB, 0);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const uint32_t o = (voff + (uint32_t)j * rstep) * 8u;
      c32 qq = cscale(acc[j], P.scale);
      qq = {qq.re + P.lambda * pv[j].re, qq.im + P.lambda * pv[j].im};
      eta += (double)pv[j].re * (double)qq.re + (double)pv[j].im * (double)qq.im;
      zeta += (double)qq.re * (double)qq.re + (double)qq.im * (double)qq.im;
      if (valid) buf_store_c64<CPW>(bd, qq, o, 0);
    }
    const long pidx = b * (long)gridDim.x * gridDim.y + (long)id.y * gridDim.x + id.x;
    if (P.eta_part) {
      if (!valid) eta = 0.0;
      const double tot = block_sum<NT>(eta, red);
      if (tid == 0) P.eta_part[pidx] = tot;
    }
    if (P.zeta_part) {
      if (!valid) zeta = 0.0;
      if (P.eta_part) __syncthreads();  // red is reused
      const double tot = block_sum<NT>(zeta, red);
      if (tid == 0) P.zeta_part[pidx] = tot;
    }
  }
}

// Root-sum-of-squares coil combine along y (the paper's RSS reconstruction):
// for every coil, optional masked load of W[b][c], inverse transform, then
// |u|^2 summed over the coils; out[b] = sqrt(sum) / sqrt(nx ny nz), real.
template <int N>
__global__ void __launch_bounds__(Len<N>::T * col_tile<Len<N>::T>()) rss_colpass_kernel(ColPass P, float* out) {
  constexpr int T = Len<N>::T;
  constexpr int E = Len<N>::E;
  constexpr int TX = col_tile<T>();
  constexpr int NT = T * TX;
  using Rad = typename Len<N>::R;
  __shared__ c32 buf[N * TX];
  __shared__ c32 tw[N];
  __shared__ uint8_t msk[N];

  const int tid = threadIdx.x, cx = tid % TX, t = tid / TX;
  const long nx = P.nx, ny = P.ny;
  const BlockId id = xcd_block();
  const long x = (long)id.x * TX + cx;
  const bool valid = x < nx;
  const uint32_t xl = (uint32_t)(valid ? x : nx - 1);
  const long pl = id.y;  // z plane
  const int G = P.ngroups;
  const long b = id.z / G;
  const int grp = (int)(id.z % G);
  const int c0 = (int)((long)grp * P.ncoils / G), c1 = (int)((long)(grp + 1) * P.ncoils / G);
  const long nvox = nx * ny * P.nz;
  const uint32_t voff = (uint32_t)(pl * ny * nx) + xl + (uint32_t)t * (uint32_t)nx;
  const uint32_t rstep = (uint32_t)T * (uint32_t)nx;
  const uint32_t vbytes = (uint32_t)(nvox * 8);
  for (int i = tid; i < N; i += NT) {
    tw[i] = P.tw[i];
    msk[i] = P.mask_load ? P.mask[pl * ny + i] : 1;
  }
  __syncthreads();
  const float sgn = (t & 1) ? -1.f : 1.f;  // output sign is irrelevant to |u|^2
  LineView<TX> lv{&buf[cx]};
  const TwTable twt{tw};
  float acc[E];
#pragma unroll
  for (int j = 0; j < E; ++j) acc[j] = 0.f;
  for (int c = c0; c < c1; ++c) {
    const Buf bw = make_buf(P.src + (b * P.ncoils + c) * nvox, vbytes);
    c32 u[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const uint32_t o = msk[t + T * j] ? (voff + (uint32_t)j * rstep) * 8u : kBufOOB;
      u[j] = cscale(buf_load_c64(bw, o, 0), sgn);
    }
    fft_line<N, T, +1>(u, t, twt, lv, Rad{});
#pragma unroll
    for (int j = 0; j < E; ++j) acc[j] += u[j].re * u[j].re + u[j].im * u[j].im;
  }
  if (!valid) return;
  if (G > 1) {
    // this group's partial sum of squares; the combine pass finishes
    float* o = static_cast<float*>(P.part) + grp * P.part_gstride + b * nvox + voff;
#pragma unroll
    for (int j = 0; j < E; ++j) o[(long)j * rstep] = acc[j];
    return;
  }
  float* o = out + b * nvox + voff;
#pragma unroll
  for (int j = 0; j < E; ++j) o[(long)j * rstep] = sqrtf(acc[j]) * P.scale;
}

// RSS combine of G partial sums of squares, added in group order.
__global__ void __launch_bounds__(256) rss_combine_kernel(const float* __restrict__ part, long gstride, int G,
                                                          long n, float scale, float* __restrict__ out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float a = part[i];
  for (int g = 1; g < G; ++g) a += part[(long)g * gstride + i];
  out[i] = sqrtf(a) * scale;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int DIR, int ST_IN, int ST_OUT>
static hipError_t launch_rows(const Geom& g, const c32* tw, const void* in, void* out,
                              const int32_t* rows, int nrows, float scale, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  RowParams P{};
  // the k-space side: the output of the forward rows, the input of the inverse
  P.compact_in = DIR > 0 ? g.kspace_compact : 0;
  P.compact_out = DIR < 0 ? g.kspace_compact : 0;
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
  const long line_bytes = g.nx * (long)sizeof(typename StorageT<ST>::T);
  if (reinterpret_cast<uintptr_t>(out) % 16 == 0 && line_bytes % 16 == 0) {
    const long chunks = lines * (line_bytes / 16);
    const long blocks = std::min<long>((chunks + 255) / 256, 8192);
    hipLaunchKernelGGL(zero_rows16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<char*>(out),
                       rows, nrows, g.ny * g.nz, line_bytes, lines);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((zero_rows_kernel<ST>), dim3((unsigned)lines), dim3(256), 0, st, out, rows,
                     nrows, g.ny * g.nz, g.nx);
  return hipGetLastError();
}


// (-1)^(n/2) / sqrt(n): the global factor of one centred unitary axis
// transform in checkerboard form (both directions); 1 for an absent axis.
static double axis_scale(long n) {
  if (n <= 1) return 1.0;
  return (((n / 2) & 1) ? -1.0 : 1.0) / std::sqrt((double)n);
}

template <int AXIS, int MODE>
static hipError_t launch_colpass(const Geom& g, ColPass P, long n, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  if (P.ngroups < 1) P.ngroups = 1;
  P.nx = g.nx;
  P.ny = g.ny;
  P.nz = g.nz;
  P.maps_bstride = g.maps_bstride;
  P.ncoils = g.ncoils;
  dispatch_length(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    constexpr int TX = pass_tile<Len<N>::T, AXIS>();
    const long planes = AXIS == 1 ? g.nz : g.ny;
    const long zdim = MODE == CM_ADJ_COIL ? (long)g.batch * (P.ngroups > 0 ? P.ngroups : 1)
                                          : (long)g.batch * g.ncoils;
    dim3 grid((unsigned)((g.nx + TX - 1) / TX), (unsigned)planes, (unsigned)zdim);
    dim3 block(Len<N>::T * TX);
    // every mode reads or writes about two complex64 values per coil voxel;
    // streaming instantiations exist from 128 points on
    const bool stream = N >= 128 && (double)g.batch * g.ncoils * (double)(g.nx * g.ny * g.nz) * 16.0 >= kStreamBytes;
    auto go = [&](auto stc) {
      constexpr bool S = decltype(stc)::value;
      if constexpr (S && N < 128) {
        return;
      } else {
        switch (g.maps_storage) {
          case ST_C64: hipLaunchKernelGGL((colpass_kernel<N, AXIS, MODE, ST_C64, S>), grid, block, 0, st, P); break;
          case ST_BF16: hipLaunchKernelGGL((colpass_kernel<N, AXIS, MODE, ST_BF16, S>), grid, block, 0, st, P); break;
          case ST_FP16: hipLaunchKernelGGL((colpass_kernel<N, AXIS, MODE, ST_FP16, S>), grid, block, 0, st, P); break;
          default: return;
        }
        err = hipGetLastError();
      }
    };
    if (stream) go(std::true_type{});
    else go(std::false_type{});
  });
  return err;
}

int adj_tiles(long nx, long ny, long nz) {
  int tx = 0;
  dispatch_length(ny, [&](auto nc) { tx = col_tile<Len<decltype(nc)::value>::T>(); });
  return tx ? (int)(((nx + tx - 1) / tx) * nz) : 0;
}

// E x -> y, through the workspace W:  y-pass (coil product), z-pass (3D),
// x rows of the sampled (kz, ky) lines, zeros elsewhere.
hipError_t launch_E(const Geom& g, const Tables& tb, const void* maps, const c32* x, c32* work,
                    void* y, hipStream_t st) {
  const bool is3d = g.nz > 1;
  ColPass P{};
  P.maps = maps;
  P.src = x;
  P.dst = work;
  P.mask = tb.mask_c;
  P.tw = tb.tw_y;
  P.mask_store = is3d ? 0 : 1;
  P.scale = 1.f;
  hipError_t err = launch_colpass<1, CM_FWD_COIL>(g, P, g.ny, st);
  if (err == hipSuccess && is3d) {
    ColPass Z{};
    Z.src = work;
    Z.dst = work;
    Z.mask = tb.mask_c;
    Z.tw = tb.tw_z;
    Z.mask_store = 1;
    Z.scale = 1.f;
    err = launch_colpass<2, CM_FWD>(g, Z, g.nz, st);
  }
  if (err != hipSuccess) return err;
  const float sc = (float)(axis_scale(g.nx) * axis_scale(g.ny) * axis_scale(g.nz));
  switch (g.kspace_storage) {
    case ST_C64:
      err = launch_rows<-1, ST_C64, ST_C64>(g, tb.tw_x, work, y, tb.rows_s, tb.n_rows_s, sc, st);
      if (err == hipSuccess && !g.kspace_compact) err = launch_zero_rows<ST_C64>(g, y, tb.rows_u, tb.n_rows_u, st);
      break;
    case ST_BF16:
      err = launch_rows<-1, ST_C64, ST_BF16>(g, tb.tw_x, work, y, tb.rows_s, tb.n_rows_s, sc, st);
      if (err == hipSuccess && !g.kspace_compact) err = launch_zero_rows<ST_BF16>(g, y, tb.rows_u, tb.n_rows_u, st);
      break;
    case ST_FP16:
      err = launch_rows<-1, ST_C64, ST_FP16>(g, tb.tw_x, work, y, tb.rows_s, tb.n_rows_s, sc, st);
      if (err == hipSuccess && !g.kspace_compact) err = launch_zero_rows<ST_FP16>(g, y, tb.rows_u, tb.n_rows_u, st);
      break;
    default: err = hipErrorInvalidValue;
  }
  return err;
}

// The adjoint passes after the x rows: z-pass (3D, masked loads) and the
// y-pass with the conjugate-sensitivity coil sum into x.
static hipError_t launch_EH_tail(const Geom& g, const Tables& tb, const void* maps, c32* work, c32* x,
                                 const c32* addp, float lambda, double* eta_part, c32* part, int ngroups,
                                 hipStream_t st) {
  const bool is3d = g.nz > 1;
  hipError_t err = hipSuccess;
  if (is3d) {
    ColPass Z{};
    Z.src = work;
    Z.dst = work;
    Z.mask = tb.mask_c;
    Z.tw = tb.tw_z;
    Z.mask_load = 1;
    Z.scale = 1.f;
    err = launch_colpass<2, CM_ADJ>(g, Z, g.nz, st);
    if (err != hipSuccess) return err;
  }
  ColPass P{};
  P.maps = maps;
  P.src = work;
  P.dst = x;
  P.addp = addp;
  P.lambda = lambda;
  P.eta_part = eta_part;
  P.mask = tb.mask_c;
  P.tw = tb.tw_y;
  P.mask_load = is3d ? 0 : 1;
  P.scale = (float)(axis_scale(g.nx) * axis_scale(g.ny) * axis_scale(g.nz));
  const bool split = ngroups > 1 && part && !addp && !eta_part;
  P.ngroups = split ? ngroups : 1;
  P.part = part;
  P.part_gstride = (long)g.batch * g.nx * g.ny * g.nz;
  err = launch_colpass<1, CM_ADJ_COIL>(g, P, g.ny, st);
  if (err != hipSuccess || !split) return err;
  // x = sum of the group partials, in group order
  EheParams C{};
  C.qpart = part;
  C.qpart_gstride = P.part_gstride;
  C.ngroups = ngroups;
  C.q = x;
  C.nvox = g.nx * g.ny * g.nz;
  return launch_combine(C, g.batch, false, st);
}

hipError_t launch_EH_rows(const Geom& g, const Tables& tb, const void* y, c32* work, hipStream_t st) {
  switch (g.kspace_storage) {
    case ST_C64: return launch_rows<+1, ST_C64, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st);
    case ST_BF16: return launch_rows<+1, ST_BF16, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st);
    case ST_FP16: return launch_rows<+1, ST_FP16, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st);
  }
  return hipErrorInvalidValue;
}

float adjoint_scale(const Geom& g) { return (float)(axis_scale(g.nx) * axis_scale(g.ny) * axis_scale(g.nz)); }

hipError_t launch_EH(const Geom& g, const Tables& tb, const void* maps, const void* y, c32* work,
                     c32* x, c32* part, int ngroups, hipStream_t st) {
  const hipError_t err = launch_EH_rows(g, tb, y, work, st);
  if (err != hipSuccess) return err;
  return launch_EH_tail(g, tb, maps, work, x, nullptr, 0.f, nullptr, part, ngroups, st);
}

// Normal operator from column passes (3D).  With a (ky, kz) mask the
// readout transforms cancel (F_x^H F_x = I), so
//   q = sum_c conj(S_c) .* F_y^H [ F_z^H diag(M) F_z ] F_y (S_c .* p) + lambda p
// as three passes: y forward with the coil product, the z projector per
// (ky, x) line, y inverse with the conjugate-sensitivity coil sum.  Each
// centred axis pair contributes 1/n, applied once: scale 1/(ny nz).
hipError_t launch_EHE_composed(const Geom& g, const Tables& tb, const void* maps, const c32* p, c32* q,
                               c32* work, float lambda, double* eta_part, double* zeta_part, hipStream_t st) {
  ColPass P{};
  P.maps = maps;
  P.src = p;
  P.dst = work;
  P.mask = tb.mask_c;
  P.tw = tb.tw_y;
  P.mask_store = g.nz > 1 ? 0 : 1;
  P.scale = 1.f;
  hipError_t err = launch_colpass<1, CM_FWD_COIL>(g, P, g.ny, st);
  if (err == hipSuccess && g.nz > 1) {
    ColPass Z{};
    Z.src = work;
    Z.dst = work;
    Z.mask = tb.mask_c;
    Z.tw = tb.tw_z;
    Z.scale = 1.f;
    err = launch_colpass<2, CM_PROJ>(g, Z, g.nz, st);
  }
  if (err != hipSuccess) return err;
  ColPass A{};
  A.maps = maps;
  A.src = work;
  A.dst = q;
  A.addp = p;
  A.lambda = lambda;
  A.eta_part = eta_part;
  A.zeta_part = zeta_part;
  A.mask = tb.mask_c;
  A.tw = tb.tw_y;
  A.mask_load = g.nz > 1 ? 0 : 1;
  A.scale = (float)(1.0 / ((double)g.ny * (double)g.nz));
  return launch_colpass<1, CM_ADJ_COIL>(g, A, g.ny, st);
}

// RSS image from k-space: the x rows of the sampled lines, the z pass (3D),
// then the coil combine along y.  out is real [B][nz][ny][nx].
hipError_t launch_rss(const Geom& g, const Tables& tb, const void* y, c32* work, float* out, void* part,
                      int ngroups, hipStream_t st) {
  const bool is3d = g.nz > 1;
  hipError_t err = hipErrorInvalidValue;
  switch (g.kspace_storage) {
    case ST_C64: err = launch_rows<+1, ST_C64, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st); break;
    case ST_BF16: err = launch_rows<+1, ST_BF16, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st); break;
    case ST_FP16: err = launch_rows<+1, ST_FP16, ST_C64>(g, tb.tw_x, y, work, tb.rows_s, tb.n_rows_s, 1.f, st); break;
  }
  if (err == hipSuccess && is3d) {
    ColPass Z{};
    Z.src = work;
    Z.dst = work;
    Z.mask = tb.mask_c;
    Z.tw = tb.tw_z;
    Z.mask_load = 1;
    Z.scale = 1.f;
    err = launch_colpass<2, CM_ADJ>(g, Z, g.nz, st);
  }
  if (err != hipSuccess) return err;
  ColPass P{};
  P.src = work;
  P.mask = tb.mask_c;
  P.tw = tb.tw_y;
  P.mask_load = is3d ? 0 : 1;
  P.nx = g.nx;
  P.ny = g.ny;
  P.nz = g.nz;
  P.ncoils = g.ncoils;
  P.scale = (float)(1.0 / std::sqrt((double)g.nx * (double)g.ny * (double)g.nz));
  const bool split = ngroups > 1 && part;
  P.ngroups = split ? ngroups : 1;
  P.part = part;
  const long nvox = g.nx * g.ny * g.nz;
  P.part_gstride = (long)g.batch * nvox;
  err = hipErrorInvalidValue;
  dispatch_length(g.ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    constexpr int TX = col_tile<Len<N>::T>();
    dim3 grid((unsigned)((g.nx + TX - 1) / TX), (unsigned)g.nz, (unsigned)(g.batch * P.ngroups));
    hipLaunchKernelGGL((rss_colpass_kernel<N>), grid, dim3(Len<N>::T * TX), 0, st, P, out);
    err = hipGetLastError();
  });
  if (err != hipSuccess || !split) return err;
  const long n = (long)g.batch * nvox;
  hipLaunchKernelGGL(rss_combine_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     static_cast<const float*>(part), P.part_gstride, P.ngroups, n, P.scale, out);
  return hipGetLastError();
}

}  // namespace sense
