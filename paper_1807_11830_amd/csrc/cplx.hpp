// Complex float helpers, compile-time roots of unity and static loops for
// the gfx950 kernels.  Device code only uses plain fp32 arithmetic here; the
// constants are exact double-precision evaluations rounded once to float.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace sense {

struct alignas(8) c32 {
  float re, im;
};

__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ c32 cscale(c32 a, float s) { return {a.re * s, a.im * s}; }
// a * b
__device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
__device__ __forceinline__ c32 cmulc(c32 a, c32 b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// acc + conj(s) * v
__device__ __forceinline__ c32 cfma_conj(c32 acc, c32 s, c32 v) {
  return {acc.re + s.re * v.re + s.im * v.im, acc.im + s.re * v.im - s.im * v.re};
}
// a * (dir * i):  dir = -1 -> multiply by -i, dir = +1 -> by +i
template <int DIR>
__device__ __forceinline__ c32 mul_dir_i(c32 a) {
  if constexpr (DIR < 0) return {a.im, -a.re};
  else return {-a.im, a.re};
}

// ---------------------------------------------------------------------------
// Compile-time cos/sin of 2*pi*m/R: octant reduction to |phi| <= pi/4 and
// Taylor series in double (error below 1e-17 there).
// ---------------------------------------------------------------------------
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}

struct cs {
  double c, s;
};

// cos and sin of 2*pi*m/R, exact at multiples of pi/2.
constexpr cs root_cs(long m, long R) {
  m %= R;
  if (m < 0) m += R;
  long q = (4 * m) / R;      // quadrant
  long r = 4 * m - q * R;    // angle within quadrant = (pi/2) * r / R
  double c = 1.0, s = 0.0;
  if (r != 0) {
    if (2 * r <= R) {
      double phi = (kPi / 2.0) * (double)r / (double)R;
      c = taylor_cos(phi);
      s = taylor_sin(phi);
    } else {
      double phi = (kPi / 2.0) * (double)(R - r) / (double)R;
      c = taylor_sin(phi);
      s = taylor_cos(phi);
    }
  }
  switch (q) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
  }
}

// a * exp(DIR * 2*pi*i * K / R), specialised for the exact roots.
template <long K, long R, int DIR>
__device__ __forceinline__ c32 twc(c32 a) {
  constexpr long m = ((K % R) + R) % R;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (4 * m == R) {
    return mul_dir_i<DIR>(a);
  } else if constexpr (2 * m == R) {
    return {-a.re, -a.im};
  } else if constexpr (4 * m == 3 * R) {
    return mul_dir_i<-DIR>(a);
  } else if constexpr (8 * m == R || 8 * m == 3 * R || 8 * m == 5 * R || 8 * m == 7 * R) {
    constexpr cs w = root_cs(m, R);
    constexpr float h = (float)(w.c > 0 ? w.c : -w.c);  // sqrt(2)/2
    constexpr float sc = w.c > 0 ? 1.f : -1.f;
    constexpr float ss = (DIR * w.s) > 0 ? 1.f : -1.f;
    // (re + i im)(sc + i ss) h
    float re = sc * a.re - ss * a.im;
    float im = sc * a.im + ss * a.re;
    return {re * h, im * h};
  } else {
    constexpr cs w = root_cs(m, R);
    constexpr float c = (float)w.c;
    constexpr float s = (float)(DIR * w.s);
    return {a.re * c - a.im * s, a.re * s + a.im * c};
  }
}

// ---------------------------------------------------------------------------
// Static loops: f(std::integral_constant<int, i>) for i in [0, N).
// ---------------------------------------------------------------------------
template <class F, int... Is>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// Reduced-precision interleaved complex storage (re first, then im).
// ---------------------------------------------------------------------------
enum Storage : int { ST_C64 = 0, ST_BF16 = 1, ST_FP16 = 2 };

template <int ST>
struct StorageT;
template <>
struct StorageT<ST_C64> {
  using T = c32;
};
template <>
struct StorageT<ST_BF16> {
  using T = uint32_t;
};
template <>
struct StorageT<ST_FP16> {
  using T = uint32_t;
};

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

template <int ST>
__device__ __forceinline__ c32 load_c(const typename StorageT<ST>::T* p, long i) {
  if constexpr (ST == ST_C64) {
    return p[i];
  } else if constexpr (ST == ST_BF16) {
    uint32_t w = p[i];
    return {bf16_to_f32(w & 0xffffu), bf16_to_f32(w >> 16)};
  } else {
    uint32_t w = p[i];
    _Float16 lo = __builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
    _Float16 hi = __builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
    return {(float)lo, (float)hi};
  }
}

template <int ST>
__device__ __forceinline__ void store_c(typename StorageT<ST>::T* p, long i, c32 v) {
  if constexpr (ST == ST_C64) {
    p[i] = v;
  } else if constexpr (ST == ST_BF16) {
    p[i] = f32_to_bf16_rne(v.re) | (f32_to_bf16_rne(v.im) << 16);
  } else {
    _Float16 lo = (_Float16)v.re;  // round to nearest even
    _Float16 hi = (_Float16)v.im;
    p[i] = (uint32_t)__builtin_bit_cast(unsigned short, lo) |
           ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
  }
}

}  // namespace sense
