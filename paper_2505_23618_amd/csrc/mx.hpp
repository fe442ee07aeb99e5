// Exact integer 32-point transforms on the int8 matrix cores (gfx950).
//
// A stage z_k = sum_n M[k][n] x[n] with int16 x and |M| <= 2^10 is computed
// exactly with v_mfma_i32_32x32x32_i8 by splitting both operands into signed
// bytes:  x = 256 xh + xl + 128  (xh = high byte, xl = low byte - 128) and
// M = 256 Mh + Ml  (Ml = ((M + 128) mod 256) - 128).  Then
//   z = 65536 P1 + 256 P2 + P3 + 128 sum_n M[k][n],
//   P1 = sum Mh xh,  P2 = sum (Mh xl + Ml xh),  P3 = sum Ml xl,
// four MFMAs with int32 accumulation, recombined with two shift-adds.
//
// Lane layout of v_mfma_i32_32x32x32_i8 (checked on the device): lane l holds
// 16 int8 of row l%32 of A and of column l%32 of B, for 16 of the 32 values of
// the contraction index; which 16 does not matter as long as A and B agree.
// The result lane l, register r holds D[8(r/4) + 4(l/32) + r%4][l%32].
#pragma once

#include "common.hpp"

namespace ta {
namespace mx {

typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

// Dense integer matrix of a core for N = 32 (row = output, column = input),
// the section 2.1 relations applied to the DCT-2 table:
//   DCT-3 = DCT-2^T, DST-2 = R DCT-2 S, DST-3 = S DCT-2^T R, DCT-8 = S DST-7 R.
// TR selects the transpose (inverse direction).
template <int N>
TA_DEV int core_entry(int core, bool tr, int k, int n) {
  if (tr) {
    const int t = k;
    k = n;
    n = t;
  }
  switch (core) {
    case C_DCT2: return ta_c2_64[k * (64 / N)][n];
    case C_DCT3: return ta_c2_64[n * (64 / N)][k];
    case C_DST2: return ((n & 1) ? -1 : 1) * ta_c2_64[(N - 1 - k) * (64 / N)][n];
    case C_DST3: return ((k & 1) ? -1 : 1) * ta_c2_64[(N - 1 - n) * (64 / N)][k];
    case C_DST7: return s7i<N>(k, n);
    default: return ((k & 1) ? -1 : 1) * s7i<N>(k, N - 1 - n);
  }
}

TA_DEV int lo_byte(int m) { return ((m + 128) & 255) - 128; }
TA_DEV int hi_byte(int m) { return (m - lo_byte(m)) >> 8; }

TA_DEV uint32_t pack4(int a, int b, int c, int d) {
  return (uint32_t)(a & 255) | ((uint32_t)(b & 255) << 8) | ((uint32_t)(c & 255) << 16) |
         ((uint32_t)(d & 255) << 24);
}

// 16 int16 values (8 natural pairs) -> the high-byte and low-byte-minus-128
// planes, 16 int8 each (4 registers), in element order.
TA_DEV void split_planes(const uint32_t (&p)[8], i4v& hi, i4v& lo) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    // bytes of p[2w] = [e0.lo e0.hi e1.lo e1.hi], p[2w+1] = [e2.lo e2.hi e3.lo e3.hi]
    hi[w] = (int)perm(p[2 * w + 1], p[2 * w], 0x07050301u);
    lo[w] = (int)(perm(p[2 * w + 1], p[2 * w], 0x06040200u) ^ 0x80808080u);
  }
}

TA_DEV i16v mfma(const i4v& a, const i4v& b, const i16v& c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// z = 65536 P1 + 256 P2 + P3 + kc for the 16 result registers.
struct Planes {
  i4v h, l;
};

TA_DEV void product(const Planes& x, const Planes& m, int kc, int (&z)[16]) {
  const i16v zero = {};
  const i16v p1 = mfma(x.h, m.h, zero);
  i16v p2 = mfma(x.l, m.h, zero);
  p2 = mfma(x.h, m.l, p2);
  const i16v p3 = mfma(x.l, m.l, zero);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    int t = (p1[r] << 8) + p2[r];
    t = (t << 8) + p3[r];
    z[r] = t + kc;
  }
}

}  // namespace mx
}  // namespace ta
