// Packed 16-bit cell arithmetic shared by the inter-task kernels.  A 32-bit
// register holds two independent cells (bits 0..15 and 16..31).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swdb {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// signed saturating add per half (v_pk_add_i16 clamp)
__device__ __forceinline__ uint32_t add_sat(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(
                                          __builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b)));
}
// per half: max(a - b, 0) with a, b read as unsigned (v_pk_sub_u16 clamp)
__device__ __forceinline__ uint32_t sub_floor(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(
                                          __builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}
// signed max per half (v_pk_max_i16)
__device__ __forceinline__ uint32_t vmax(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(
                                          __builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b)));
}

// One cell of Gotoh's recurrence on both halves, with E and F kept as
// max(E, 0) and max(F, 0):
//   h = max(hd + p, E, F); best = max(best, h); t = max(h - o, 0);
//   E = max(E - e, t);  F = max(F - e, t)
// hd enters as H(i-1, j-1) and leaves as H(i, j-1) (the next row's
// diagonal); H enters as H(i, j-1) and leaves as H(i, j).
__device__ __forceinline__ void cell(uint32_t& hd, uint32_t& H, uint32_t& E, uint32_t& F,
                                     uint32_t& best, uint32_t p, uint32_t go, uint32_t ge) {
  const uint32_t h = vmax(vmax(add_sat(hd, p), E), F);
  hd = H;
  H = h;
  best = vmax(best, h);
  const uint32_t t = sub_floor(h, go);
  E = vmax(sub_floor(E, ge), t);
  F = vmax(sub_floor(F, ge), t);
}

}  // namespace swdb
