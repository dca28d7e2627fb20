// Raw buffer loads and stores for the column kernels.  A buffer resource
// (base, size) lives in scalar registers; each access takes a per-thread
// byte offset (one VGPR) plus a wavefront-uniform byte offset (SGPR), so the
// strided row accesses of a column need no 64-bit per-access address math.
// Every offset used here stays inside the resource's range, except
// kBufOOB: the buffer unit range-checks raw accesses against the resource
// size and returns zero for an out-of-range load without a memory request,
// so a load at kBufOOB is a branch-free masked load.
#pragma once

#include "cplx.hpp"

namespace sense {

// Word 3 of a raw gfx9 buffer descriptor (32-bit data format, no swizzle).
constexpr int kBufWord3 = 0x00020000;

// Per-thread byte offset beyond every resource made here (one image or coil
// image is below 2^31 bytes, which plan validation enforces).
constexpr uint32_t kBufOOB = 0x80000000u;

struct Buf {
  __amdgpu_buffer_rsrc_t r;
};

// Cache policy of an access (the immediate cache-policy operand of the
// buffer instruction): kCacheDefault, or kCacheStream (nt: the line is
// streamed through L2 without being kept for reuse).  Measured on MI355X in
// the 256-point fused kernel, where every access covers whole 128-byte
// lines read or written once per launch: 357.8 -> 340.9 us per fused CG
// launch at 160 slices of 256^2 with 12 coils.  Where a block covers only
// part of a line (8-column tiles, 16-bit maps), the neighbouring block's
// half of the line must stay in L2, and streaming it costs a second HBM
// read (384 points, 8 columns: 714 -> 867 us).
constexpr int kCacheDefault = 0;
constexpr int kCacheStream = 2;
// Algorithmic traffic from which a plan launch streams (the kernels choose
// per access whether a streamed line is whole).
constexpr double kStreamBytes = 1024.0 * 1024.0 * 1024.0;
// Policy of an access whose block row segment is seg_bytes long.
template <bool STREAM, int SEG_BYTES>
constexpr int stream_policy() {
  return STREAM && SEG_BYTES >= 128 ? kCacheStream : kCacheDefault;
}

__device__ __forceinline__ Buf make_buf(const void* base, uint32_t bytes) {
  return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3)};
}

template <int CP = kCacheDefault>
__device__ __forceinline__ c32 buf_load_c64(Buf b, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)voff, (int)soff, CP));
}

template <int CP = kCacheDefault>
__device__ __forceinline__ uint32_t buf_load_b32(Buf b, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)voff, (int)soff, CP);
}

template <int CP = kCacheDefault>
__device__ __forceinline__ void buf_store_c64(Buf b, c32 v, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, v),
                                        b.r, (int)voff, (int)soff, CP);
}

// 16-byte chunks copied from global memory straight into LDS
// (buffer_load_dwordx4 ... lds).  Lane l of the wave writes bytes
// [16 l, 16 l + 16) of the LDS window at lds_addr (an LDS byte address, the
// same for every lane), reading resource offset voff + soff; the access is
// range-checked like any buffer access.  It is issued from inline assembly:
// the compiler cannot tell the copy's LDS window from other LDS arrays and
// would otherwise wait for the copy before every later LDS read.  The caller
// therefore waits itself (s_waitcnt vmcnt(0)) before reading the window, and
// must not refill a window before its own reads of it have completed
// (s_waitcnt lgkmcnt(0)).  M0 carries the LDS address and is restored
// after the copy is issued.
typedef int v4i32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4i32 make_rsrc(const void* base, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  return {(int)(uint32_t)a, (int)((uint32_t)(a >> 32) & 0xffffu), (int)bytes, kBufWord3};
}

__device__ __forceinline__ void buf_load_lds16(v4i32 rsrc, uint32_t lds_addr, uint32_t voff, uint32_t soff) {
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "buffer_load_dwordx4 %2, %3, %4 offen lds\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "s"(lds_addr), "v"(voff), "s"(rsrc), "s"(soff)
      : "memory");
}

// LDS byte address of a pointer into a __shared__ array.
template <class T>
__device__ __forceinline__ uint32_t lds_address(T* p) {
  return (uint32_t)reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) T*)p);
}

// Complex value in storage ST at (voff + soff) element offsets, converted to fp32.
template <int ST, int CP = kCacheDefault>
__device__ __forceinline__ c32 buf_load_st(Buf b, uint32_t vi, uint32_t si) {
  if constexpr (ST == ST_C64) {
    return buf_load_c64<CP>(b, vi * 8u, si * 8u);
  } else {
    const uint32_t w = buf_load_b32<CP>(b, vi * 4u, si * 4u);
    if constexpr (ST == ST_BF16) {
      return {bf16_to_f32(w & 0xffffu), bf16_to_f32(w >> 16)};
    } else {
      _Float16 lo = __builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
      _Float16 hi = __builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
      return {(float)lo, (float)hi};
    }
  }
}

}  // namespace sense
