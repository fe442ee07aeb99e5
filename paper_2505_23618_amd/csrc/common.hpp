// Shared definitions of the libtadj device code (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables_gen.h"

#define TA_DEV __device__ __forceinline__

namespace ta {

typedef short s2v __attribute__((ext_vector_type(2)));
typedef unsigned short u2v __attribute__((ext_vector_type(2)));

// Transform kinds of one 1-D pass (forward orientation).  The DST-2/DST-3
// are the section 2.1 relations around the DCT-2/DCT-3 butterflies:
//   DST-2 = R DCT-2 S,  DST-3 = S DCT-3 R;  DCT-8 = S DST-7 R (eq. 3).
enum Core : int { C_DCT2 = 0, C_DCT3 = 1, C_DST2 = 2, C_DST3 = 3, C_DST7 = 4, C_DCT8 = 5 };
enum Adj : int { ADJ_NONE = 0, ADJ_BAND = 1, ADJ_POST = 2 };

// Transpose of a core (used by the inverse): DCT-2^T = DCT-3, DST-2^T = DST-3.
constexpr int core_transpose(int c) {
  return c == C_DCT2 ? C_DCT3 : c == C_DCT3 ? C_DCT2 : c == C_DST2 ? C_DST3 : c == C_DST3 ? C_DST2 : c;
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

// Integer DCT-2 coefficient of the N-point table (nested in the 64-point one).
template <int N>
TA_DEV constexpr int c2i(int k, int n) { return ta_c2_64[k * (64 / N)][n]; }

template <int N>
TA_DEV constexpr int s7i(int k, int n) {
  if constexpr (N == 4) return ta_s7_4[k][n];
  else if constexpr (N == 8) return ta_s7_8[k][n];
  else if constexpr (N == 16) return ta_s7_16[k][n];
  else if constexpr (N == 32) return ta_s7_32[k][n];
  else return ta_s7_64[k][n];
}

template <int N>
TA_DEV constexpr double s7f(int k, int n) {
  if constexpr (N == 4) return ta_s7f_4[k][n];
  else if constexpr (N == 8) return ta_s7f_8[k][n];
  else if constexpr (N == 16) return ta_s7f_16[k][n];
  else if constexpr (N == 32) return ta_s7f_32[k][n];
  else return ta_s7f_64[k][n];
}

// Transform parameters (band taps, sub-block matrices) are read through the
// constant address space: they are wave-uniform and never written by a
// kernel, so the compiler loads them with scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) uint32_t* cparam;
TA_DEV cparam as_cparam(const void* p) { return (cparam)p; }

// Pack two int16 constants into a dot2 operand (lo = a, hi = b).
TA_DEV constexpr uint32_t pk2(int a, int b) {
  return (uint32_t)(uint16_t)(int16_t)a | ((uint32_t)(uint16_t)(int16_t)b << 16);
}

// acc + a.lo*b.lo + a.hi*b.hi, int16 x int16 products, int32 accumulation.
TA_DEV int dot2(uint32_t a, uint32_t b, int acc) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(s2v, a), __builtin_bit_cast(s2v, b), acc, false);
}

// Head of a dot2 chain: the VOP3P form takes the accumulator from a VGPR
// (one register holding the rounding offset serves every chain) and the
// coefficient pair from an SGPR, so starting a chain costs no v_mov.
TA_DEV int dot2h(uint32_t a, uint32_t coef, int acc) {
  int r;
  asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(coef), "v"(acc));
  return r;
}

TA_DEV int dot2h0(uint32_t a, uint32_t coef) {
  int r;
  asm("v_dot2_i32_i16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "s"(coef));
  return r;
}

// acc + a * coef with 24-bit signed operands (|a| < 2^23), one instruction
// per product (the compiler would otherwise split chains into mul + add3).
TA_DEV int mad24(int a, int coef, int acc) {
  int r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(coef), "v"(acc));
  return r;
}

// Saturating pack of two int32 into int16 lanes (lo = a, hi = b): clip16.
TA_DEV uint32_t satpk(int a, int b) {
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pk_i16(a, b));
}

// Packed int16 lanes, wrapping: (a.lo - b.hi, a.hi - b.lo) and
// (a.lo + b.hi, a.hi + b.lo).  One v_pk_sub_i16 / v_pk_add_u16 each: the
// swap of b's halves is an operand selector, not an instruction.
TA_DEV uint32_t pk_sub_x(uint32_t a, uint32_t b) {
  const u2v x = __builtin_bit_cast(u2v, a), y = __builtin_bit_cast(u2v, b);
  return __builtin_bit_cast(uint32_t, x - __builtin_shufflevector(y, y, 1, 0));
}
TA_DEV uint32_t pk_add_x(uint32_t a, uint32_t b) {
  const u2v x = __builtin_bit_cast(u2v, a), y = __builtin_bit_cast(u2v, b);
  return __builtin_bit_cast(uint32_t, x + __builtin_shufflevector(y, y, 1, 0));
}

// Whether every int16 lane of x[0..M) lies in [-2^14, 2^14): then sums and
// differences of any two lanes fit in int16.  v + 2^14 (mod 2^16) has its
// top bit clear exactly for v in that range.
template <int M>
TA_DEV bool lanes_within_14(const uint32_t (&x)[M]) {
  const u2v bias = {16384, 16384};
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < M; ++i) t |= __builtin_bit_cast(uint32_t, __builtin_bit_cast(u2v, x[i]) + bias);
  return (t & 0x80008000u) == 0;
}

// True when `ok` holds in every active lane of the wave (a wave-uniform
// branch condition).
TA_DEV bool wave_all(bool ok) { return __ballot(!ok) == 0; }

// Byte permute: bytes 0-3 of `lo`, 4-7 of `hi`, selector per output byte.
TA_DEV uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

}  // namespace ta
