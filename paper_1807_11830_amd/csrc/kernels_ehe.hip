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
// TX complex values) and loops over the coils of its coil group; p, the
// coil's S column segment and the accumulator q stay in registers, and the
// forward/inverse transforms exchange through LDS only between Stockham
// stages.  With one group the block also emits the fp64 partials of the CG
// scalars; with several, each group writes its partial coil sum and a
// combine pass adds them in group order.
#include "bufio.hpp"
#include "cg_scalar.hpp"
#include "kernels.hpp"
#include "lengths.hpp"
#include "reduce.hpp"
#include "xcd.hpp"

namespace sense {

// Maps staged through LDS.  With staging, the next coil's maps tile is
// copied from HBM straight into LDS (buf_load_lds16: 16 bytes per lane, no
// register held while the copy is in flight) during the current coil's
// transforms.  Every wave fills and reads only its own part of the tile, so
// the copy needs a wait on the wave's own counter and no block barrier, and
// the transform exchanges use LDS-only barriers that leave it in flight.
// The tile costs N * TX * (bytes per maps value) of LDS per block.
// Measured on MI355X (fused CG launch, 12 or 32 coils): with 16-bit maps at
// 256 points staging halves the launch time for BF16 (597 -> 291 us at 160
// slices; the register path's 4-byte loads run at half speed there) and
// matches the register path for FP16; with complex64 maps, and at 160, 192,
// 320 and 384 points, it is slower or no faster (384 points, 32 coils,
// complex64: 164 -> 197 us), so only 16-bit maps at 256 points use it.
constexpr int kLdsBytesPerCU = 160 * 1024;
template <int N>
constexpr int ehe_base_lds() {
  constexpr int NT = EheLen<N>::T * EheLen<N>::TX;
  return N * EheLen<N>::TX * 8 + N * 8 + N * 4 + 8 * (NT / 64 > 0 ? NT / 64 : 1);
}
template <int N, int ST>
constexpr int ehe_stage_bytes() {
  return N * EheLen<N>::TX * (ST == ST_C64 ? 8 : 4);
}
template <int N, int ST>
constexpr bool ehe_stage_maps() {
  if constexpr (ST == ST_C64 || N != 256) {
    return false;
  } else {
    // whole 16-byte chunks per wave and row, and 3 blocks per CU
    return (EheLen<N>::E * 4) % 16 == 0 && 64 % EheLen<N>::TX == 0 &&
           3 * (ehe_base_lds<N>() + ehe_stage_bytes<N, ST>() + 512) <= kLdsBytesPerCU;
  }
}

// Cache policy of the fused kernel's accesses (STREAM = streaming launch):
// streamed where one block's row segment (TX values) covers whole 128-byte
// lines, default otherwise.  Streaming pays only when a launch's data is
// far larger than the caches and read once (160 slices of 256^2 with 12
// coils: 1.66 GB per launch, 357.7 -> 340.5 us); problems that stay in L2
// and the memory-side cache between launches lose their hits (one 256^2
// slice with 16 coils: 26.2 -> 28.0 us; 16 slices of 320^2 with 32 coils,
// 0.52 GB: 238 -> 240 us).  Plan launches stream from kStreamBytes of
// algorithmic traffic on; batched serving launches never do.  Streaming
// instantiations exist from 128 points on (smaller slices reach 1 GiB per
// launch only at batches of thousands, which take the default policy).
template <int N, int SB>
constexpr int ehe_cache_policy() {
  return EheLen<N>::TX * SB >= 128 ? kCacheStream : kCacheDefault;
}
template <int N>
constexpr bool ehe_has_stream() {
  return N >= 128;
}

template <int N, int ST, bool CG, bool SM, bool STREAM>
__device__ __forceinline__ void ehe2d_body(const EheParams& P, const int tile, const int b, const int grp) {
  constexpr int T = EheLen<N>::T;
  constexpr int E = EheLen<N>::E;
  constexpr int TX = EheLen<N>::TX;
  constexpr int NT = T * TX;
  using Rad = typename EheLen<N>::R;
  using SType = typename StorageT<ST>::T;
  constexpr int SB = (int)sizeof(SType);
  constexpr int CPS = STREAM ? ehe_cache_policy<N, SB>() : kCacheDefault;                 // maps
  constexpr int CPV = STREAM ? ehe_cache_policy<N, (int)sizeof(c32)>() : kCacheDefault;  // image vectors

  // one LDS exchange buffer (each stage boundary waits for its readers)
  __shared__ c32 xbuf[N * TX];
  __shared__ c32 tw[N];
  __shared__ float mu[N];
  __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];
  // the staged maps tile: wave w's part holds its rows j = 0..E-1, one
  // 64-lane row of values after another
  __shared__ __attribute__((aligned(16))) unsigned char stage[SM ? ehe_stage_bytes<N, ST>() : 16];

  const int tid = threadIdx.x;
  const int cx = tid % TX;
  const int t = tid / TX;
  const long x = (long)tile * TX + cx;
  const bool valid = x < P.nx;
  const long nx = P.nx;

  // CG: the start-of-iteration scalars (every block derives the same ones)
  [[maybe_unused]] CgFused cgs{};
  if constexpr (CG) {
    if (!cg_fused_begin(P.state + b, P.rr_part, P.rr_tiles, P.cgpart, P.part_batch, P.part_tiles, P.rho_tiles,
                        P.part_stride, P.rho_hist, P.hist_len, P.tol, P.k, b, tile == 0 && grp == 0 && tid == 0,
                        cgs))
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

  // this block's coil group and its maps
  const int c0 = (int)((long)grp * P.ncoils / P.ngroups);
  const int c1 = (int)((long)(grp + 1) * P.ncoils / P.ngroups);
  const SType* S = static_cast<const SType*>(P.maps) + (long)b * P.maps_bstride;
  const uint32_t coil_bytes = (uint32_t)(nvox * (long)sizeof(SType));

  // Staged maps: wave wv copies its E rows of coil c into its part of the
  // tile, 1024 bytes (JI = 1024 / ROWB rows j) per instruction.  A lane's
  // 16-byte chunk holds 16 / SB values of row j = i JI + lane / (64 / JI),
  // lanes l0 .. l0 + 16/SB - 1 of that row (never across a row of TX
  // columns); its offset is the lane's offset for i = 0 plus a uniform
  // i JI T nx SB.  Rows are whole chunks (nx SB is a multiple of 16 on this
  // path), so a chunk is either inside the image or wholly past nx, where it
  // reads nothing (out-of-range offset).
  [[maybe_unused]] const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  [[maybe_unused]] constexpr int ROWB = 64 * SB;  // bytes of one row j of a wave's part
  [[maybe_unused]] constexpr int JI = 1024 / ROWB;
  [[maybe_unused]] unsigned char* const wstage = stage + wv * (E * ROWB);
  [[maybe_unused]] const uint32_t wstage_lds = lds_address(stage) + (uint32_t)(wv * (E * ROWB));
  [[maybe_unused]] uint32_t go0 = 0;
  if constexpr (SM) {
    const int j = (lane * 16) / ROWB;
    const int l0 = ((lane * 16) % ROWB) / SB;
    const uint32_t tt = (uint32_t)(wv * (64 / TX) + l0 / TX);
    const long col = (long)tile * TX + l0 % TX;
    go0 = col < nx ? (((tt + (uint32_t)(T * j)) * (uint32_t)nx + (uint32_t)col) * (uint32_t)SB) : kBufOOB;
  }
  [[maybe_unused]] auto stage_coil = [&](int c) {
    const v4i32 rs = make_rsrc(S + (long)c * nvox, coil_bytes);
    const uint32_t step = (uint32_t)(JI * T) * (uint32_t)nx * (uint32_t)SB;
    sfor<E / JI>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      buf_load_lds16(rs, wstage_lds + i * 1024, go0, (uint32_t)i * step);
    });
  };
  if constexpr (SM) {
    if (c0 < c1) stage_coil(c0);  // every copy issued is waited for in the coil loop
  }

  c32 p[E], q[E];
  [[maybe_unused]] double rho_acc = 0.0;
  if constexpr (!CG) {
    const Buf bp = make_buf(P.p_in + (long)b * nvox, img_bytes);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      p[j] = buf_load_c64<CPV>(bp, voff * 8u, (uint32_t)j * rstep * 8u);
      q[j] = {0.f, 0.f};
    }
  } else {
    // iteration k > 0 first finishes iteration k-1:
    //   x += alpha p,  r -= alpha q,  p = r + beta p
    // Every coil group computes the new p for its own transforms; group 0
    // stores x, r, p (the other groups do not read x: its loads take an
    // out-of-range offset, which reads nothing).
    const Buf bp = make_buf(P.p_in + (long)b * nvox, img_bytes);
    const Buf br = make_buf(P.r + (long)b * nvox, img_bytes);
    const Buf bx = make_buf(P.x + (long)b * nvox, img_bytes);
    const Buf bpo = make_buf(P.p_out + (long)b * nvox, img_bytes);
    const Buf bro = make_buf(P.r_out + (long)b * nvox, img_bytes);
    const bool owner = grp == 0;
    // Groups of G rows in a two-slot software pipeline: the loads of group
    // g+1 are issued before group g is updated and stored, so a wait for
    // group g never includes the stores of the group before it, and at most
    // two groups of loads hold registers (the transform's are still free).
    // Launch 0 runs the same code: alpha = beta = 0 and q is zero there
    // (the init kernel clears it), so the update leaves x, r, p as they are.
    constexpr int G = E % 4 == 0 ? 4 : 1;
    constexpr int NG = E / G;
    const uint32_t lo = voff * 8u;
    const uint32_t lox = owner ? lo : kBufOOB;
    const double a = cgs.alpha, bt = cgs.beta;
    c32 lp[2][G], lr[2][G], lq[2][G], lx[2][G];
    auto load_group = [&](auto gc, int slot) {
      constexpr int g0 = decltype(gc)::value * G;
      sfor<G>([&](auto jc) {
        constexpr int i = decltype(jc)::value;
        const uint32_t so = (uint32_t)(g0 + i) * rstep * 8u;
        lp[slot][i] = buf_load_c64<CPV>(bp, lo, so);
        lr[slot][i] = buf_load_c64<CPV>(br, lo, so);
        lq[slot][i] = buf_load_c64<CPV>(bq, lo, so);
        lx[slot][i] = buf_load_c64<CPV>(bx, lox, so);  // unconditional: keeps the waits exact
      });
    };
    auto update_group = [&](auto gc, int slot) {
      constexpr int g0 = decltype(gc)::value * G;
      sfor<G>([&](auto jc) {
        constexpr int i = decltype(jc)::value;
        constexpr int j = g0 + i;
        const uint32_t so = (uint32_t)j * rstep * 8u;
        const c32 pv0 = lp[slot][i], qv = lq[slot][i], xv0 = lx[slot][i];
        const c32 xv = {(float)((double)xv0.re + a * pv0.re), (float)((double)xv0.im + a * pv0.im)};
        const c32 rv = {(float)((double)lr[slot][i].re - a * qv.re), (float)((double)lr[slot][i].im - a * qv.im)};
        const c32 pv = {(float)((double)rv.re + bt * pv0.re), (float)((double)rv.im + bt * pv0.im)};
        if (valid && owner) {
          buf_store_c64<CPV>(bx, xv, lo, so);
          buf_store_c64<CPV>(bro, rv, lo, so);
          buf_store_c64<CPV>(bpo, pv, lo, so);
        }
        p[j] = pv;
        if (valid) rho_acc += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
        q[j] = {0.f, 0.f};
      });
    };
    load_group(std::integral_constant<int, 0>{}, 0);
    sfor<NG>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      if constexpr (g + 1 < NG) load_group(std::integral_constant<int, g + 1>{}, (g + 1) & 1);
      asm volatile("" ::: "memory");
      update_group(gc, g & 1);
    });
  }
  __syncthreads();

  using TwC = TwChoice<N, T, Rad>;
  typename TwC::type twsrc;
  if constexpr (TwC::regs) twsrc.load(tw, t);
  else twsrc.tw = tw;

  LineView<TX> lv{&xbuf[cx]};

  auto load_s = [&](c32* s, int c) {
    const Buf bs = make_buf(S + (long)c * nvox, coil_bytes);
#pragma unroll
    for (int j = 0; j < E; ++j) s[j] = buf_load_st<ST, CPS>(bs, voff, (uint32_t)j * rstep);
  };
  // One coil: u = S p, forward transform, mask, inverse transform,
  // q += conj(S) u.
  auto coil = [&](const c32* s) {
    c32 u[E];
#pragma unroll
    for (int j = 0; j < E; ++j) u[j] = cmul(s[j], p[j]);
    fft_line<N, T, -1, SM>(u, t, twsrc, lv, Rad{});
#pragma unroll
    for (int j = 0; j < E; ++j) u[j] = cscale(u[j], mu[t + T * j]);
    fft_line<N, T, +1, SM>(u, t, twsrc, lv, Rad{});
#pragma unroll
    for (int j = 0; j < E; ++j) q[j] = cfma_conj(q[j], s[j], u[j]);
  };

  if constexpr (SM) {
    for (int c = c0; c < c1; ++c) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's copy of coil c
      c32 sc[E];
      const SType* ws = reinterpret_cast<const SType*>(wstage) + lane;
#pragma unroll
      for (int j = 0; j < E; ++j) sc[j] = load_c<ST>(ws, (long)j * 64);
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // read before the part is refilled
      if (c + 1 < c1) stage_coil(c + 1);
      coil(sc);
    }
  } else {
    for (int c = c0; c < c1; ++c) {
      c32 sc[E];
      load_s(sc, c);
      coil(sc);
    }
  }

  if (P.ngroups > 1) {
    // partial coil sum of this group; the combine pass does the rest
    const Buf bg = make_buf(P.qpart + (long)grp * P.qpart_gstride + (long)b * nvox, img_bytes);
    if (valid) {
#pragma unroll
      for (int j = 0; j < E; ++j) buf_store_c64<CPV>(bg, q[j], voff * 8u, (uint32_t)j * rstep * 8u);
    }
    if constexpr (CG) {
      // group 0 leaves <r,r> of the residual it stored in the prologue
      if (grp == 0) {
        const double tot = block_sum<NT>(rho_acc, red);
        if (tid == 0)
          P.cgpart[(((long)(P.k & 1) * P.part_batch + b) * P.part_stride + tile) * kCgParts + 2] = tot;
      }
    }
    return;
  }
  if constexpr (!CG) {
    double eta = 0.0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      c32 qq = {q[j].re + P.lambda * p[j].re, q[j].im + P.lambda * p[j].im};
      if (valid) {
        buf_store_c64<CPV>(bq, qq, voff * 8u, (uint32_t)j * rstep * 8u);
        eta += (double)p[j].re * (double)qq.re + (double)p[j].im * (double)qq.im;
      }
    }
    if (P.eta_part) {
      const double tot = block_sum<NT>(eta, red);
      if (tid == 0) P.eta_part[(long)b * P.ntiles + tile] = tot;
    }
  } else {
    // q = A p; fp64 partials of Re<p,q>, <q,q> and <r,r> (the new
    // residual, summed in the prologue) for the next launch
    double acc[kCgParts] = {0.0, 0.0, rho_acc};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      c32 qq = {q[j].re + P.lambda * p[j].re, q[j].im + P.lambda * p[j].im};
      if (valid) {
        buf_store_c64<CPV>(bq, qq, voff * 8u, (uint32_t)j * rstep * 8u);
        acc[0] += (double)p[j].re * (double)qq.re + (double)p[j].im * (double)qq.im;
        acc[1] += (double)qq.re * (double)qq.re + (double)qq.im * (double)qq.im;
      }
    }
    double* out = P.cgpart + (((long)(P.k & 1) * P.part_batch + b) * P.part_stride + tile) * kCgParts;
#pragma unroll
    for (int i = 0; i < kCgParts; ++i) {
      const double tot = block_sum<NT>(acc[i], red);
      if (tid == 0) out[i] = tot;
      if constexpr (NT / 64 > 1) __syncthreads();  // red is reused
    }
  }
}

template <int N, int ST, bool CG, bool SM, bool STREAM>
__global__ void __launch_bounds__(EheLen<N>::T * EheLen<N>::TX) ehe2d_kernel(EheParams P) {
  const BlockId id = xcd_block();
  ehe2d_body<N, ST, CG, SM, STREAM>(P, (int)id.x, (int)id.y, (int)id.z);
}

// Batched CG launch over many independent single-slice problems of the same
// ny: block row blockIdx.y runs the problem described by table[blockIdx.y]
// (its own maps, vectors, partials and CG state), so every problem computes
// exactly what its own launch would.
template <int N, int ST, bool SM>
__global__ void __launch_bounds__(EheLen<N>::T * EheLen<N>::TX)
    ehe2d_table_kernel(const EheParams* __restrict__ table) {
  const EheParams P = table[blockIdx.y];
  if ((long)blockIdx.x >= (long)P.ntiles || (int)blockIdx.z >= P.ngroups) return;
  ehe2d_body<N, ST, true, SM, false>(P, blockIdx.x, 0, blockIdx.z);
}

// The same with the table passed by value in the kernel arguments.
template <int N, int ST, bool SM>
__global__ void __launch_bounds__(EheLen<N>::T * EheLen<N>::TX) ehe2d_inline_kernel(EheInline table) {
  const EheParams& P = table.p[blockIdx.y];
  if ((long)blockIdx.x >= (long)P.ntiles || (int)blockIdx.z >= P.ngroups) return;
  ehe2d_body<N, ST, true, SM, false>(P, blockIdx.x, 0, blockIdx.z);
}

int ehe_tile_width(long ny) {
  int tx = 0;
  dispatch_length(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    tx = EheLen<N>::TX;
  });
  return tx;
}

int auto_coil_groups(long nx, long ny, int ncoils, int batch) {
  const int tx = ehe_tile_width(ny);
  if (tx == 0) return 1;
  const long blocks = (nx + tx - 1) / tx * (long)batch;
  if (blocks >= kFillBlocks) return 1;
  long gr = (kFillBlocks + blocks - 1) / blocks;
  if (gr > ncoils / 2) gr = ncoils / 2;
  if (gr > kMaxCoilGroups) gr = kMaxCoilGroups;
  return (int)(gr < 1 ? 1 : gr);
}

static void fill_common(const Geom& g, const Tables& tb, EheParams& P) {
  P.tw = tb.tw_y;
  P.mu = tb.mu_y;
  P.nx = g.nx;
  P.nvox = g.nx * g.ny;
  P.ntiles = (int)((g.nx + ehe_tile_width(g.ny) - 1) / ehe_tile_width(g.ny));
  P.maps_bstride = g.maps_bstride;
  P.ncoils = g.ncoils;
  P.qpart_gstride = (long)g.batch * P.nvox;
}

// Staged maps need 16-byte aligned rows (nx values of the maps storage) and
// maps base; other problems take the register path.  The choice depends on
// the problem alone, so a batched launch computes what a single one does.
bool ehe_staged(long ny, int maps_storage, long nx, const void* maps) {
  bool can = false;
  dispatch_length(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    switch (maps_storage) {
      case ST_C64: can = ehe_stage_maps<N, ST_C64>(); break;
      case ST_BF16: can = ehe_stage_maps<N, ST_BF16>(); break;
      case ST_FP16: can = ehe_stage_maps<N, ST_FP16>(); break;
      default: break;
    }
  });
  const long sb = maps_storage == ST_C64 ? 8 : 4;
  return can && (nx * sb) % 16 == 0 && reinterpret_cast<uintptr_t>(maps) % 16 == 0;
}

template <int N, int ST, bool CG, bool STREAM>
static void launch_ehe_kernel_nt(const Geom& g, const EheParams& P, dim3 grid, dim3 block, hipStream_t st) {
  if constexpr (ehe_stage_maps<N, ST>()) {
    if (ehe_staged(N, ST, g.nx, P.maps)) {
      hipLaunchKernelGGL((ehe2d_kernel<N, ST, CG, true, STREAM>), grid, block, 0, st, P);
      return;
    }
  }
  hipLaunchKernelGGL((ehe2d_kernel<N, ST, CG, false, STREAM>), grid, block, 0, st, P);
}

// Whether a plan launch of this shape streams its accesses (see
// ehe_cache_policy): algorithmic bytes of one fused launch, maps in their
// storage plus eight image vectors per slice.
static bool ehe_stream(const Geom& g) {
  const double sb = g.maps_storage == ST_C64 ? 8.0 : 4.0;
  const double bytes = (double)g.batch * (double)(g.nx * g.ny) * (g.ncoils * sb + 64.0);
  return bytes >= kStreamBytes;
}

template <int N, int ST, bool CG>
static void launch_ehe_kernel(const Geom& g, const EheParams& P, dim3 grid, dim3 block, hipStream_t st) {
  if constexpr (ehe_has_stream<N>()) {
    if (ehe_stream(g)) {
      launch_ehe_kernel_nt<N, ST, CG, true>(g, P, grid, block, st);
      return;
    }
  }
  launch_ehe_kernel_nt<N, ST, CG, false>(g, P, grid, block, st);
}

template <int N, int ST>
static void launch_table_kernel(bool staged, const EheParams* d_table, dim3 grid, dim3 block, hipStream_t st) {
  if constexpr (ehe_stage_maps<N, ST>()) {
    if (staged) {
      hipLaunchKernelGGL((ehe2d_table_kernel<N, ST, true>), grid, block, 0, st, d_table);
      return;
    }
  }
  hipLaunchKernelGGL((ehe2d_table_kernel<N, ST, false>), grid, block, 0, st, d_table);
}

template <int N, int ST>
static void launch_inline_kernel(bool staged, const EheInline& table, dim3 grid, dim3 block, hipStream_t st) {
  if constexpr (ehe_stage_maps<N, ST>()) {
    if (staged) {
      hipLaunchKernelGGL((ehe2d_inline_kernel<N, ST, true>), grid, block, 0, st, table);
      return;
    }
  }
  hipLaunchKernelGGL((ehe2d_inline_kernel<N, ST, false>), grid, block, 0, st, table);
}

template <bool CG>
static hipError_t launch_ehe_impl(const Geom& g, const EheParams& P, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  dispatch_length(g.ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    constexpr int T = EheLen<N>::T;
    constexpr int TX = EheLen<N>::TX;
    dim3 grid((unsigned)((g.nx + TX - 1) / TX), (unsigned)g.batch, (unsigned)P.ngroups);
    dim3 block(T * TX);
    switch (g.maps_storage) {
      case ST_C64: launch_ehe_kernel<N, ST_C64, CG>(g, P, grid, block, st); break;
      case ST_BF16: launch_ehe_kernel<N, ST_BF16, CG>(g, P, grid, block, st); break;
      case ST_FP16: launch_ehe_kernel<N, ST_FP16, CG>(g, P, grid, block, st); break;
      default: return;
    }
    err = hipGetLastError();
  });
  return err;
}

void fill_ehe_cg_params(const Geom& g, const Tables& tb, const void* maps, const CgVectors& v, float lambda,
                        int k, const CgArgs& cg, EheParams* out) {
  EheParams P{};
  fill_common(g, tb, P);
  P.maps = maps;
  P.x = v.x;
  P.r = v.r[k & 1];
  P.r_out = v.r[(k + 1) & 1];
  P.p_in = v.p[k & 1];
  P.p_out = v.p[(k + 1) & 1];
  P.q = v.q;
  P.qpart = v.qpart;
  P.ngroups = v.ngroups;
  P.k = k;
  P.lambda = lambda;
  P.eta_part = cg.eta_part;
  P.state = cg.state;
  P.rr_part = cg.rr_part;
  P.rr_tiles = cg.rr_tiles;
  P.cgpart = cg.cgpart;
  P.part_batch = cg.part_batch;
  P.part_tiles = cg.part_tiles;
  P.rho_tiles = cg.rho_tiles;
  P.part_stride = cg.part_stride;
  P.rho_hist = cg.rho_hist;
  P.hist_len = cg.hist_len;
  P.tol = cg.tol;
  *out = P;
}

hipError_t launch_ehe_table(long ny, int maps_storage, bool staged, const EheParams* d_table, int nproblems,
                            int max_tiles, int max_groups, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  dispatch_length(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    dim3 grid((unsigned)max_tiles, (unsigned)nproblems, (unsigned)max_groups);
    dim3 block(EheLen<N>::T * EheLen<N>::TX);
    switch (maps_storage) {
      case ST_C64: launch_table_kernel<N, ST_C64>(staged, d_table, grid, block, st); break;
      case ST_BF16: launch_table_kernel<N, ST_BF16>(staged, d_table, grid, block, st); break;
      case ST_FP16: launch_table_kernel<N, ST_FP16>(staged, d_table, grid, block, st); break;
      default: return;
    }
    err = hipGetLastError();
  });
  return err;
}

hipError_t launch_ehe_inline(long ny, int maps_storage, bool staged, const EheInline& table, int nproblems,
                             int max_tiles, int max_groups, hipStream_t st) {
  if (nproblems > kInlineProblems) return hipErrorInvalidValue;
  hipError_t err = hipErrorInvalidValue;
  dispatch_length(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    dim3 grid((unsigned)max_tiles, (unsigned)nproblems, (unsigned)max_groups);
    dim3 block(EheLen<N>::T * EheLen<N>::TX);
    switch (maps_storage) {
      case ST_C64: launch_inline_kernel<N, ST_C64>(staged, table, grid, block, st); break;
      case ST_BF16: launch_inline_kernel<N, ST_BF16>(staged, table, grid, block, st); break;
      case ST_FP16: launch_inline_kernel<N, ST_FP16>(staged, table, grid, block, st); break;
      default: return;
    }
    err = hipGetLastError();
  });
  return err;
}

hipError_t launch_ehe(const Geom& g, const Tables& tb, const void* maps, const c32* p, c32* q,
                      float lambda, double* eta_part, c32* qpart, int ngroups, hipStream_t st) {
  EheParams P{};
  fill_common(g, tb, P);
  P.maps = maps;
  P.p_in = p;
  P.q = q;
  P.qpart = qpart;
  P.ngroups = ngroups;
  P.lambda = lambda;
  P.eta_part = eta_part;
  hipError_t e = launch_ehe_impl<false>(g, P, st);
  if (e == hipSuccess && ngroups > 1) e = launch_combine(P, g.batch, false, st);
  return e;
}

hipError_t launch_ehe_cg(const Geom& g, const Tables& tb, const void* maps, const CgVectors& v,
                         float lambda, int k, const CgArgs& cg, hipStream_t st) {
  EheParams P{};
  fill_ehe_cg_params(g, tb, maps, v, lambda, k, cg, &P);
  hipError_t e = launch_ehe_impl<true>(g, P, st);
  if (e == hipSuccess && v.ngroups > 1) e = launch_combine(P, g.batch, true, st);
  return e;
}

}  // namespace sense
