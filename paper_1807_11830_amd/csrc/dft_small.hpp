// In-register DFTs of small radix R: a[0..R) -> X[k] = sum_n a[n] W^(nk),
// W = exp(DIR * 2*pi*i / R), natural order in and out.  Radix 2, 3, 4 and 5
// are written out; composite radices are Cooley-Tukey splits R = R1 * R2
// with compile-time twiddles (all indices static, so the arrays stay in
// VGPRs).
#pragma once

#include "cplx.hpp"

namespace sense {

template <int R, int DIR>
struct DFT;

template <int DIR>
struct DFT<1, DIR> {
  static __device__ __forceinline__ void run(c32*) {}
};

template <int DIR>
struct DFT<2, DIR> {
  static __device__ __forceinline__ void run(c32* a) {
    c32 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <int DIR>
struct DFT<3, DIR> {
  // X1,2 = a0 - (a1 + a2)/2 +- DIR i (sqrt(3)/2)(a1 - a2)
  static __device__ __forceinline__ void run(c32* a) {
    constexpr float s3 = 0.8660254037844386f;
    c32 t1 = cadd(a[1], a[2]);
    c32 t2 = csub(a[1], a[2]);
    c32 m = {a[0].re - 0.5f * t1.re, a[0].im - 0.5f * t1.im};
    c32 d = mul_dir_i<DIR>(cscale(t2, s3));
    a[0] = cadd(a[0], t1);
    a[1] = cadd(m, d);
    a[2] = csub(m, d);
  }
};

template <int DIR>
struct DFT<4, DIR> {
  static __device__ __forceinline__ void run(c32* a) {
    c32 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    c32 s13 = cadd(a[1], a[3]), d13 = mul_dir_i<DIR>(csub(a[1], a[3]));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, d13);
    a[3] = csub(d02, d13);
  }
};

template <int DIR>
struct DFT<5, DIR> {
  // t1 = a1 + a4, t2 = a2 + a3, t3 = a1 - a4, t4 = a2 - a3
  // X1,4 = a0 + c1 t1 + c2 t2 +- DIR i (s1 t3 + s2 t4)
  // X2,3 = a0 + c2 t1 + c1 t2 +- DIR i (s2 t3 - s1 t4)
  static __device__ __forceinline__ void run(c32* a) {
    constexpr cs w1 = root_cs(1, 5), w2 = root_cs(2, 5);
    constexpr float c1 = (float)w1.c, s1 = (float)w1.s, c2 = (float)w2.c, s2 = (float)w2.s;
    c32 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    c32 t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
    c32 b1 = {a[0].re + c1 * t1.re + c2 * t2.re, a[0].im + c1 * t1.im + c2 * t2.im};
    c32 b2 = {a[0].re + c2 * t1.re + c1 * t2.re, a[0].im + c2 * t1.im + c1 * t2.im};
    c32 d1 = mul_dir_i<DIR>(c32{s1 * t3.re + s2 * t4.re, s1 * t3.im + s2 * t4.im});
    c32 d2 = mul_dir_i<DIR>(c32{s2 * t3.re - s1 * t4.re, s2 * t3.im - s1 * t4.im});
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(b1, d1);
    a[4] = csub(b1, d1);
    a[2] = cadd(b2, d2);
    a[3] = csub(b2, d2);
  }
};

// First factor of a composite radix: 4 where possible, else 2, 3, 5.
constexpr int split_factor(int R) {
  if (R % 4 == 0 && R != 4) return 4;
  if (R % 2 == 0 && R != 2) return 2;
  if (R % 3 == 0 && R != 3) return 3;
  if (R % 5 == 0 && R != 5) return 5;
  return 0;
}

// Cooley-Tukey R = R1 * R2:  n = R2 n1 + n2,  k = k1 + R1 k2.
//   Y[k1][n2] = W_R^(n2 k1) * DFT_R1 over n1 of a[R2 n1 + n2]
//   X[k1 + R1 k2] = DFT_R2 over n2 of Y[k1][n2]
template <int R1, int R2, int DIR>
__device__ __forceinline__ void dft_ct(c32* a) {
  constexpr int R = R1 * R2;
  c32 y[R];
  sfor<R2>([&](auto n2c) {
    constexpr int n2 = decltype(n2c)::value;
    c32 t[R1];
    sfor<R1>([&](auto n1c) { t[decltype(n1c)::value] = a[R2 * decltype(n1c)::value + n2]; });
    DFT<R1, DIR>::run(t);
    sfor<R1>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      y[k1 * R2 + n2] = twc<(long)n2 * k1, R, DIR>(t[k1]);
    });
  });
  sfor<R1>([&](auto k1c) {
    constexpr int k1 = decltype(k1c)::value;
    c32 t[R2];
    sfor<R2>([&](auto n2c) { t[decltype(n2c)::value] = y[k1 * R2 + decltype(n2c)::value]; });
    DFT<R2, DIR>::run(t);
    sfor<R2>([&](auto k2c) { a[k1 + R1 * decltype(k2c)::value] = t[decltype(k2c)::value]; });
  });
}

template <int R, int DIR>
struct DFT {
  static_assert(split_factor(R) != 0, "radix must be a product of 2, 3 and 5");
  static __device__ __forceinline__ void run(c32* a) {
    dft_ct<split_factor(R), R / split_factor(R), DIR>(a);
  }
};

}  // namespace sense
