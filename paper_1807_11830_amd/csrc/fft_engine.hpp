// Stockham FFT of one line of length N held by T cooperating threads.
//
// Register layout: thread t (0 <= t < T) holds the E = N/T elements at line
// positions t + T*j, j = 0..E-1, in v[j].  A radix-R Stockham stage with
// span NS (product of the radices already done) treats butterfly jb as the
// elements jb + r*(N/R), r < R; thread t owns butterflies jb = t + T*m,
// m < E/R, whose inputs are exactly its own registers v[m + r*E/R] whenever
// R divides E.  The stage multiplies input r by W_(NS*R)^(r * (jb mod NS)),
// takes the radix-R DFT and writes output r to position
//     (jb / NS) * NS * R + (jb mod NS) + r * NS.
// After the last stage (NS * R = N) that position is t + T*(m + r*E/R): the
// thread's own register again, so transforms start and end in the same
// layout and no reordering pass is ever needed.  Between two stages the
// block exchanges through one LDS buffer (a barrier before each exchange
// write, so it never races the previous read, and one after it).
//
// The inverse transform (DIR = +1) runs the same stages with conjugated
// twiddles, so a forward/inverse pair returns every value to the thread and
// register that held it.
#pragma once

#include "dft_small.hpp"

#include <type_traits>

namespace sense {

// Block barrier for the exchanges of a transform that must not wait for the
// wave's global loads in flight: __syncthreads() also waits for every
// outstanding global load and store of the wave (its workgroup fence),
// which would end an asynchronous prefetch at the first exchange.  This one
// waits for the wave's LDS operations only; the memory clobber keeps the
// compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Exchanges whose partners all sit in one wavefront (the line's threads are
// consecutive lanes of one wave): the wave's LDS operations are performed
// in order, so waiting for its own writes (and keeping the compiler from
// moving LDS accesses across the wait) is all an exchange needs; no block
// barrier.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Synchronisation of the stage exchanges: a block barrier, an LDS-only
// block barrier, or a wave-local wait.
enum : int { kSyncBlock = 0, kSyncLds = 1, kSyncWave = 2 };

template <int SY>
__device__ __forceinline__ void exchange_barrier() {
  if constexpr (SY == kSyncLds) lds_barrier();
  else if constexpr (SY == kSyncWave) wave_lds_sync();
  else __syncthreads();
}

template <int... Rs>
struct Radices {
  static constexpr int count = sizeof...(Rs);
};

template <int... Rs>
constexpr int radix_product(Radices<Rs...>) {
  return (1 * ... * Rs);
}

// LDS view for one line: element at position p sits at base[p * PS].
template <int PS>
struct LineView {
  c32* base;
  __device__ __forceinline__ c32& at(int p) const { return base[p * PS]; }
};

// A line stored contiguously with one pad element after every 16: Stockham
// writes at stride 16 (the radix-16 and radix-16-span patterns) would
// otherwise land all 16 threads of a line on the same LDS bank pair.
struct PadLineView {
  c32* base;
  __device__ __forceinline__ c32& at(int p) const { return base[p + (p >> 4)]; }
};
// Elements of one padded line of length N (plus one, so consecutive lines
// start on different banks).
template <int N>
constexpr int padded_line() {
  return N + N / 16 + 1;
}

// Twiddle sources.  A stage of span NS and radix R multiplies input r of
// butterfly jb (m-th of the thread) by exp(DIR 2 pi i r (jb mod NS) / (NS R)),
// read from tw[e] = exp(-2 pi i e / N) at e = (jb mod NS) * r * N / (NS R).
struct TwTable {
  const c32* tw;  // N entries (LDS or global)
  template <int N, int NS, int R, int m, int r>
  __device__ __forceinline__ c32 get(int jm) const {
    return tw[jm * (r * (N / (NS * R)))];
  }
};

// Register copy of the second-stage twiddles of a two-stage transform, loaded
// once per block and reused by every forward and inverse transform.
template <int N, int T, int R1, int R2>
struct TwRegs2 {
  static constexpr int E = N / T;
  static constexpr int M = E / R2;
  c32 w[M * (R2 - 1)];
  __device__ __forceinline__ void load(const c32* tw, int t) {
    sfor<M>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      const int jm = (t + T * m) % R1;
      sfor<R2 - 1>([&](auto rc) {
        constexpr int r = decltype(rc)::value + 1;
        w[m * (R2 - 1) + r - 1] = tw[jm * (r * (N / (R1 * R2)))];
      });
    });
  }
  template <int N_, int NS, int R, int m, int r>
  __device__ __forceinline__ c32 get(int) const {
    static_assert(NS == R1 && R == R2, "register twiddles cover the second stage only");
    return w[m * (R2 - 1) + r - 1];
  }
};

// One Stockham stage.
template <int N, int T, int R, int NS, int DIR, bool LAST, class View, class Tw>
__device__ __forceinline__ void stockham_stage(c32* v, int t, const Tw& tw, View out) {
  constexpr int E = N / T;
  constexpr int M = E / R;
  static_assert(E % R == 0, "each radix must divide the elements per thread");
  sfor<M>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    c32 a[R];
    sfor<R>([&](auto rc) { a[decltype(rc)::value] = v[m + decltype(rc)::value * M]; });
    const int jb = t + T * m;
    const int jm = jb % NS;
    if constexpr (NS > 1) {
      sfor<R - 1>([&](auto rc) {
        constexpr int r = decltype(rc)::value + 1;
        const c32 w = tw.template get<N, NS, R, m, r>(jm);
        a[r] = (DIR < 0) ? cmul(a[r], w) : cmulc(a[r], w);
      });
    }
    DFT<R, DIR>::run(a);
    if constexpr (LAST) {
      sfor<R>([&](auto rc) { v[m + decltype(rc)::value * M] = a[decltype(rc)::value]; });
    } else {
      const int base = (jb / NS) * (NS * R) + jm;
      sfor<R>([&](auto rc) { out.at(base + decltype(rc)::value * NS) = a[decltype(rc)::value]; });
    }
  });
}

// Recursive driver over the radix list.  One LDS buffer serves every
// exchange: the barrier in front of each exchange write keeps it behind the
// previous exchange's reads (or the previous transform's), and the one after
// it makes the write visible.
template <int N, int T, int DIR, int NS, int LB, class View, class Tw, int R, int... Rest>
__device__ __forceinline__ void fft_stages(c32* v, int t, const Tw& tw, View b) {
  constexpr bool last = sizeof...(Rest) == 0;
  if constexpr (!last) exchange_barrier<LB>();
  stockham_stage<N, T, R, NS, DIR, last>(v, t, tw, b);
  if constexpr (!last) {
    exchange_barrier<LB>();
    constexpr int E = N / T;
    sfor<E>([&](auto jc) { v[decltype(jc)::value] = b.at(t + T * decltype(jc)::value); });
    fft_stages<N, T, DIR, NS * R, LB, View, Tw, Rest...>(v, t, tw, b);
  }
}

// Transform of one line held as v[j] = line[t + T j] by its T threads
// (unnormalised; DIR = -1 forward, +1 inverse); the result returns to the
// same positions.  b is the line's view of the LDS exchange buffer.  LB
// selects the exchange synchronisation (exchange_barrier; a bool true is
// kSyncLds).
template <int N, int T, int DIR, int LB = kSyncBlock, class View, class Tw, int... Rs>
__device__ __forceinline__ void fft_line(c32* v, int t, const Tw& tw, View b, Radices<Rs...>) {
  static_assert(radix_product(Radices<Rs...>{}) == N, "radices must multiply to N");
  fft_stages<N, T, DIR, 1, LB, View, Tw, Rs...>(v, t, tw, b);
}

// Twiddle source of the fused kernels: registers for two-stage transforms
// with at most 8 elements per thread, the LDS table otherwise.
constexpr int kTwRegMaxE = 8;
template <int N, int T, class Rad>
struct TwChoice {
  using type = TwTable;
  static constexpr bool regs = false;
};
template <int N, int T, int R1, int R2>
struct TwChoice<N, T, Radices<R1, R2>> {
  static constexpr bool regs = (N / T) <= kTwRegMaxE;
  using type = std::conditional_t<regs, TwRegs2<N, T, R1, R2>, TwTable>;
};

}  // namespace sense
