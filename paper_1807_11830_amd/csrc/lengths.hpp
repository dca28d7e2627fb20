// Compile-time transform configurations: threads per line T and the
// Stockham radix list for every supported length N.  Each radix divides the
// per-thread element count E = N / T (see fft_engine.hpp).
#pragma once

#include "fft_engine.hpp"

namespace sense {

template <int N>
struct Len;

// Columns per block for column-mode kernels: at least one full wavefront.
template <int T>
constexpr int col_tile() {
  return T >= 4 ? 16 : 32;
}

#define SENSE_LEN(N_, T_, ...)                 \
  template <>                                  \
  struct Len<N_> {                             \
    static constexpr int T = T_;               \
    static constexpr int E = N_ / T_;          \
    using R = Radices<__VA_ARGS__>;            \
  };

SENSE_LEN(8, 2, 4, 2)
SENSE_LEN(16, 4, 4, 4)
SENSE_LEN(32, 4, 8, 4)
SENSE_LEN(48, 4, 12, 4)
SENSE_LEN(64, 8, 8, 8)
SENSE_LEN(80, 4, 20, 4)
SENSE_LEN(96, 8, 12, 4, 2)
SENSE_LEN(128, 8, 16, 8)
SENSE_LEN(160, 8, 20, 4, 2)
SENSE_LEN(192, 8, 24, 8)
SENSE_LEN(256, 16, 16, 16)
SENSE_LEN(320, 16, 20, 4, 4)
SENSE_LEN(384, 16, 24, 4, 4)
#undef SENSE_LEN

// Configuration of the fused E^H E kernel along y: threads per column T,
// radix list, columns per block TX.  Fewer elements per thread than the
// generic configuration where that buys occupancy (the kernel keeps p, q,
// two sets of maps and the working column in registers).
template <int N>
struct EheLen : Len<N> {
  static constexpr int TX = col_tile<Len<N>::T>();
};

// 256 = 16 * 16: two radix-16 stages over 16 threads per column (measured
// faster than 32 threads x 8 elements with radices 8, 8, 4, and than 8 or
// 32 columns per block).
template <>
struct EheLen<256> {
  static constexpr int T = 16;
  static constexpr int E = 16;
  using R = Radices<16, 16>;
  static constexpr int TX = 16;
};
template <>
struct EheLen<128> {
  static constexpr int T = 16;
  static constexpr int E = 8;
  using R = Radices<8, 4, 4>;
  static constexpr int TX = 16;
};
// 384 = 12 * 4 * 4 * 2 over 32 threads per column: 12 elements per thread
// instead of 24 keeps the kernel within 3 waves per SIMD, and twice the
// threads per column fill the chip at small batches.  (320 stays at 16
// threads x 20 elements: 32 threads would need six stages, 10 x 2^5, and
// measured slower.)
template <>
struct EheLen<384> {
  static constexpr int T = 32;
  static constexpr int E = 12;
  using R = Radices<12, 4, 4, 2>;
  static constexpr int TX = 8;
};
template <>
struct EheLen<192> {
  static constexpr int T = 16;
  static constexpr int E = 12;
  using R = Radices<12, 4, 4>;
  static constexpr int TX = 16;
};

// Calls f(std::integral_constant<int, N>) for the runtime length n; returns
// false when n is not instantiated.
template <class F>
inline bool dispatch_length(long n, F&& f) {
  switch (n) {
#define SENSE_CASE(N_) \
  case N_:             \
    f(std::integral_constant<int, N_>{}); \
    return true;
    SENSE_CASE(8)
    SENSE_CASE(16)
    SENSE_CASE(32)
    SENSE_CASE(48)
    SENSE_CASE(64)
    SENSE_CASE(80)
    SENSE_CASE(96)
    SENSE_CASE(128)
    SENSE_CASE(160)
    SENSE_CASE(192)
    SENSE_CASE(256)
    SENSE_CASE(320)
    SENSE_CASE(384)
#undef SENSE_CASE
    default:
      return false;
  }
}


}  // namespace sense
