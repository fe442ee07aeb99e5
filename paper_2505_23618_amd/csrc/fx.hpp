// Fixed-point 1-D stages of the adjusted transforms (int16 data, int32 sums).
//
// Every stage computes sums of int16 x int16 products with v_dot2_i32_i16
// (two products per instruction) or, inside the DCT-2 butterfly where the
// operands are int32 partial sums, with 24-bit multiply-adds.  A stage's
// result is kept as int32 sums that already include the rounding offset
// 2^(s-1); the consumer applies ">> s" and packs two values with the
// saturating v_cvt_pk_i16_i32, which is exactly clip16((sum + 2^(s-1)) >> s)
// and lets the consumer choose the pairing it needs for its own dot2 operands.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace ta {
namespace fx {

// N int16 values held in N/2 packed registers, register s holding elements
// (2s, 2s+1).
template <int N>
struct Packed {
  uint32_t p[N / 2];
  TA_DEV int value(int i) const {
    const uint32_t w = p[i >> 1];
    return (i & 1) ? ((int)w >> 16) : (int)(short)(w & 0xffffu);
  }
  // (value(i), value(j)) packed; an index of -1 stands for zero.
  TA_DEV uint32_t pair(int i, int j) const {
    if (i >= 0 && j == i + 1 && (i & 1) == 0) return p[i >> 1];
    const uint32_t lo = i >= 0 ? p[i >> 1] : 0u;
    const uint32_t hi = j >= 0 ? p[j >> 1] : 0u;
    const uint32_t sl = i >= 0 ? ((i & 1) ? 0x0302u : 0x0100u) : 0x0c0cu;
    const uint32_t sh = j >= 0 ? ((j & 1) ? 0x0706u : 0x0504u) : 0x0c0cu;
    return perm(hi, lo, sl | (sh << 16));
  }
};

// Stage result: pre-shift sums (offset included).  Elements below SPLIT
// shift by s0, the others by s1 (a post-adjustment leaves rows >= B alone).
template <int N, int SPLIT = N>
struct Acc {
  int a[N];
  int s0, s1;
  TA_DEV int value(int i) const { return a[i] >> (i < SPLIT ? s0 : s1); }
  TA_DEV uint32_t pair(int i, int j) const {
    return satpk(i >= 0 ? value(i) : 0, j >= 0 ? value(j) : 0);
  }
};

// Elements < B come from `lo`, the rest from `hi` (inverse sub-block stage).
template <int N, int B, class SL, class SH>
struct Split {
  const SL& lo;
  const SH& hi;
  TA_DEV int value(int i) const { return i < B ? lo.value(i) : hi.value(i); }
  TA_DEV uint32_t pair(int i, int j) const {
    const bool il = i < B, jl = j < B;
    if ((i < 0 || il) && (j < 0 || jl)) return lo.pair(i, j);
    if ((i < 0 || !il) && (j < 0 || !jl)) return hi.pair(i, j);
    return satpk(i >= 0 ? value(i) : 0, j >= 0 ? value(j) : 0);
  }
};

// Input view of a core: w[k] = src[N-1-k] when REV.
template <int N, bool REV, class S>
struct Rev {
  const S& s;
  TA_DEV uint32_t pair(int i, int j) const {
    return REV ? s.pair(i >= 0 ? N - 1 - i : -1, j >= 0 ? N - 1 - j : -1) : s.pair(i, j);
  }
};

// ---------------------------------------------------------------------------
// Band pre-adjustment (K taps per row).  Row i of the forward band A has its
// taps in columns [i - K/2 + ((i + K/2) & 1), +K): the support of K/2 layers
// of Givens rotations on adjacent pairs, even pairs first.  Its transpose
// (used by the inverse) meets the even-pair layer first, so its rows start
// at i - K/2 + 1 - (i & 1).  taps[i*K/2 + t] holds the packed pair
// of columns (start + 2t, start + 2t + 1), zero outside 0..N-1.
// ---------------------------------------------------------------------------
template <int K, bool TR>
TA_DEV constexpr int band_start(int i) {
  return TR ? i - K / 2 + 1 - (i & 1) : i - K / 2 + ((i + K / 2) & 1);
}

template <int N, int K, bool TR, class S>
TA_DEV Acc<N> band(const S& src, cparam taps, int shift) {
  Acc<N> r;
  r.s0 = r.s1 = shift;
  const int off = 1 << (shift - 1);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int st = band_start<K, TR>(i);
    int acc = off;
    bool head = true;
#pragma unroll
    for (int t = 0; t < K / 2; ++t) {
      const int c0 = st + 2 * t, c1 = c0 + 1;
      if (c1 < 0 || c0 >= N) continue;
      const uint32_t pr = src.pair(c0 >= 0 ? c0 : -1, c1 < N ? c1 : -1);
      acc = head ? dot2h(pr, taps[i * (K / 2) + t], off) : dot2(pr, taps[i * (K / 2) + t], acc);
      head = false;
    }
    r.a[i] = acc;
  }
  return r;
}

// ---------------------------------------------------------------------------
// DCT-3 (inverse DCT-2) butterfly: z[n] = sum_k C2_N[k][n] w[k].
// Even part: the N/2-point DCT-3 of w[0], w[2], ...; odd part:
// O[n] = sum_j C2_N[2j+1][n] w[2j+1]; z[n] = E[n] + O[n], z[N-1-n] = E[n] - O[n].
// ---------------------------------------------------------------------------
template <int N, int M, bool OFF, class W>
TA_DEV void c3_even(const W& w, int (&e)[M], int off) {
  constexpr int ST = N / M;
  if constexpr (M == 2) {
    const uint32_t p = w.pair(0, ST);
    const uint32_t c0 = pk2(c2i<2>(0, 0), c2i<2>(1, 0)), c1 = pk2(c2i<2>(0, 1), c2i<2>(1, 1));
    e[0] = OFF ? dot2h(p, c0, off) : dot2h0(p, c0);
    e[1] = OFF ? dot2h(p, c1, off) : dot2h0(p, c1);
  } else {
    int ee[M / 2];
    c3_even<N, M / 2, OFF>(w, ee, off);
#pragma unroll
    for (int n = 0; n < M / 2; ++n) {
      int o = 0;
#pragma unroll
      for (int i = 0; i < M / 4; ++i) {
        const int k1 = 4 * i + 1, k2 = 4 * i + 3;
        const uint32_t pr = w.pair(k1 * ST, k2 * ST), cf = pk2(c2i<M>(k1, n), c2i<M>(k2, n));
        o = i == 0 ? dot2h0(pr, cf) : dot2(pr, cf, o);
      }
      e[n] = ee[n] + o;
      e[M - 1 - n] = ee[n] - o;
    }
  }
}

// OSIGN applies S to the output before rounding (DST-3 = S DCT-3 R);
// IREV reverses the input.  The rounding offset enters once per output.
template <int N, bool IREV, bool OSIGN, class S>
TA_DEV Acc<N> core_c3(const S& src, int shift) {
  const Rev<N, IREV, S> w{src};
  const int off = 1 << (shift - 1);
  Acc<N> r;
  r.s0 = r.s1 = shift;
  int ee[N / 2];
  c3_even<N, N / 2, !OSIGN>(w, ee, off);
#pragma unroll
  for (int n = 0; n < N / 2; ++n) {
    const int sg = (OSIGN && (n & 1)) ? -1 : 1;
    int o = 0;
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const int k1 = 4 * i + 1, k2 = 4 * i + 3;
      const uint32_t pr = w.pair(k1, k2), cf = pk2(sg * c2i<N>(k1, n), sg * c2i<N>(k2, n));
      o = i > 0 ? dot2(pr, cf, o) : (OSIGN ? dot2h(pr, cf, off) : dot2h0(pr, cf));
    }
    if (!OSIGN) {
      r.a[n] = ee[n] + o;
      r.a[N - 1 - n] = ee[n] - o;
    } else if (sg > 0) {      // o = O + off: y_n = E + O + off, y_{N-1-n} = -(E - O) + off
      r.a[n] = ee[n] + o;
      r.a[N - 1 - n] = o - ee[n];
    } else {                  // o = -O + off: y_n = -(E + O) + off, y_{N-1-n} = E - O + off
      r.a[n] = o - ee[n];
      r.a[N - 1 - n] = o + ee[n];
    }
  }
  return r;
}

// ---------------------------------------------------------------------------
// DCT-2 butterfly: z[k] = sum_n C2_N[k][n] u[n].  Odd rows are odd about the
// middle, even rows even, so with d[n] = u[n] - u[N-1-n] and
// e[n] = u[n] + u[N-1-n] (n < N/2):
//   z[k odd] = sum_n C2_N[k][n] d[n],   z[2k] = (N/2-point DCT-2 of e)[k].
// ---------------------------------------------------------------------------
// N/2-point and smaller levels on int32 partial sums (|v| < 2^21) with 24-bit
// multiply-adds.  With NEG_ODD the transform input is u[n] = -v[n] for odd n
// (the sign is folded into the first level's additions and coefficients).
template <int M, bool NEG_ODD = false>
TA_DEV void c2_int(const int (&v)[M], int (&z)[M], int off) {
  if constexpr (M == 2) {
    z[0] = ((NEG_ODD ? v[0] - v[1] : v[0] + v[1]) << 8) + off;     // row 0 = 2^8
    z[1] = ((NEG_ODD ? v[0] + v[1] : v[0] - v[1]) << 8) + off;     // 2-point row 1 = (+2^8, -2^8)
  } else {
    int e[M / 2], o[M / 2];
#pragma unroll
    for (int n = 0; n < M / 2; ++n) {
      if (!NEG_ODD) {
        e[n] = v[n] + v[M - 1 - n];
        o[n] = v[n] - v[M - 1 - n];
      } else if ((n & 1) == 0) {           // u[n] = v[n], u[M-1-n] = -v[M-1-n]
        e[n] = v[n] - v[M - 1 - n];
        o[n] = v[n] + v[M - 1 - n];
      } else {                             // u[n] = -v[n]: o[n] holds -(u[n] - u[M-1-n])
        e[n] = v[M - 1 - n] - v[n];
        o[n] = v[n] + v[M - 1 - n];
      }
    }
#pragma unroll
    for (int k = 1; k < M; k += 2) {
      int acc = off;
#pragma unroll
      for (int n = 0; n < M / 2; ++n)
        acc = mad24(o[n], (NEG_ODD && (n & 1)) ? -c2i<M>(k, n) : c2i<M>(k, n), acc);
      z[k] = acc;
    }
    int ze[M / 2];
    c2_int<M / 2>(e, ze, off);
#pragma unroll
    for (int k = 0; k < M / 2; ++k) z[2 * k] = ze[k];
  }
}

// Unpack natural int16 pairs into int32 values.
template <int M>
TA_DEV void unpack_pairs(const uint32_t (&p)[M / 2], int (&v)[M]) {
#pragma unroll
  for (int s = 0; s < M / 2; ++s) {
    v[2 * s] = (int)(short)(p[s] & 0xffffu);
    v[2 * s + 1] = (int)p[s] >> 16;
  }
}

// M-point DCT-2 of u from natural int16 pairs x of f, u_n = f_n, or
// u_n = (-1)^n f_n with NEG, all |f_n| < 2^14 in the wave.  The first level
// stays in int16: one packed add or subtract of x[s] and the half-swapped
// x[M/2-1-s] gives two values of d_n = u_n - u_{M-1-n} (or of e) at once
// (with NEG, d_n = (-1)^n (f_n + f_{M-1-n}) and e_n = (-1)^n (f_n - f_{M-1-n}):
// the lane signs move into the coefficients or into the next level), so
// each odd row costs M/4 dot2.  With DEEP the even half recurses the same
// way while the wave's e values stay within +-2^14 (forward passes, whose
// inputs are residual-sized); otherwise, and below 4 points, it continues
// on int32 with 24-bit multiply-adds.  z[k] gets the exact sum plus off.
template <int M, bool NEG, bool DEEP>
TA_DEV void c2_packed(const uint32_t (&x)[M / 2], int (&z)[M], int off) {
  constexpr int SG = NEG ? -1 : 1;
  uint32_t dp[M / 4], ep[M / 4];
#pragma unroll
  for (int s = 0; s < M / 4; ++s) {
    const uint32_t a = x[s], b = x[M / 2 - 1 - s];
    dp[s] = NEG ? pk_add_x(a, b) : pk_sub_x(a, b);
    ep[s] = NEG ? pk_sub_x(a, b) : pk_add_x(a, b);
  }
#pragma unroll
  for (int k = 1; k < M; k += 2) {
    int acc = off;
#pragma unroll
    for (int s = 0; s < M / 4; ++s) {
      const uint32_t cf = pk2(c2i<M>(k, 2 * s), SG * c2i<M>(k, 2 * s + 1));
      acc = s == 0 ? dot2h(dp[s], cf, off) : dot2(dp[s], cf, acc);
    }
    z[k] = acc;
  }
  int ze[M / 2];
  bool packed = false;
  if constexpr (DEEP && M / 2 >= 4) {
    if (wave_all(lanes_within_14(ep))) {
      c2_packed<M / 2, NEG, DEEP>(ep, ze, off);
      packed = true;
    }
  }
  if (!packed) {
    int e[M / 2];
    unpack_pairs<M / 2>(ep, e);
    c2_int<M / 2, NEG>(e, ze, off);
  }
#pragma unroll
  for (int k = 0; k < M / 2; ++k) z[2 * k] = ze[k];
}

// ISIGN applies S to the input, OREV reverses the output (DST-2 = R DCT-2 S).
//
// The input arrives as natural int16 pairs x[s] = (x_2s, x_2s+1).  When every
// |x_n| < 2^14 in the whole wave, c2_packed runs the first level (and, with
// DEEP, deeper levels) in int16; otherwise the odd rows are taken as
// full-length dot products of the input pairs and e is formed in int32.
// Both give the same exact integer sums.
template <int N, bool ISIGN, bool OREV, bool DEEP, class S>
TA_DEV Acc<N> core_c2(const S& src, int shift) {
  const int off = 1 << (shift - 1);
  Acc<N> r;
  r.s0 = r.s1 = shift;
  uint32_t x[N / 2];
#pragma unroll
  for (int s = 0; s < N / 2; ++s) x[s] = src.pair(2 * s, 2 * s + 1);
  // With S applied, u_n = (-1)^n x_n: the sign of the odd-n lane moves into
  // the coefficient (odd rows) or into c2_int (even rows).
  constexpr int SG = ISIGN ? -1 : 1;
  int z[N];
  if (wave_all(lanes_within_14(x))) {
    c2_packed<N, ISIGN, DEEP>(x, z, off);
  } else {
#pragma unroll
    for (int k = 1; k < N; k += 2) {
      int acc = off;
#pragma unroll
      for (int s = 0; s < N / 2; ++s) {
        const uint32_t cf = pk2(c2i<N>(k, 2 * s), SG * c2i<N>(k, 2 * s + 1));
        acc = s == 0 ? dot2h(x[s], cf, off) : dot2(x[s], cf, acc);
      }
      z[k] = acc;
    }
    int e[N / 2];
#pragma unroll
    for (int n = 0; n < N / 2; ++n) {
      const int a = (n & 1) ? ((int)x[n >> 1] >> 16) : (int)(short)(x[n >> 1] & 0xffffu);
      const int m = N - 1 - n;
      const int b = (m & 1) ? ((int)x[m >> 1] >> 16) : (int)(short)(x[m >> 1] & 0xffffu);
      e[n] = ISIGN ? a - b : a + b;
    }
    int ze[N / 2];
    c2_int<N / 2, ISIGN>(e, ze, off);
#pragma unroll
    for (int k = 0; k < N / 2; ++k) z[2 * k] = ze[k];
  }
#pragma unroll
  for (int m = 0; m < N; ++m) r.a[m] = z[OREV ? N - 1 - m : m];
  return r;
}

// ---------------------------------------------------------------------------
// Direct DST-7 / DCT-8 (full matrix, the comparison path of Table 1).
// DCT-8[k][n] = (-1)^k DST-7[k][N-1-n] (eq. 3).  TR uses the transpose.
// ---------------------------------------------------------------------------
template <int N, int KIND>
TA_DEV constexpr int dmat(int k, int n) {
  return KIND == C_DST7 ? s7i<N>(k, n) : ((k & 1) ? -s7i<N>(k, N - 1 - n) : s7i<N>(k, N - 1 - n));
}

template <int N, int KIND, bool TR, class S>
TA_DEV Acc<N> core_direct(const S& src, int shift) {
  const int off = 1 << (shift - 1);
  Acc<N> r;
  r.s0 = r.s1 = shift;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int acc = off;
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const int c0 = TR ? dmat<N, KIND>(2 * j, k) : dmat<N, KIND>(k, 2 * j);
      const int c1 = TR ? dmat<N, KIND>(2 * j + 1, k) : dmat<N, KIND>(k, 2 * j + 1);
      const uint32_t pr = src.pair(2 * j, 2 * j + 1);
      acc = j == 0 ? dot2h(pr, pk2(c0, c1), off) : dot2(pr, pk2(c0, c1), acc);
    }
    r.a[k] = acc;
  }
  return r;
}

// DEEP_INV: the inverse's DCT-2 cores also try the deeper packed levels (the
// forward's always do: they see residual-sized inputs); worth it for the
// 32- and 64-point passes of the packed kernels, whose inputs mostly fit
template <int N, int CORE, bool TR, bool DEEP_INV = false, class S>
TA_DEV Acc<N> core(const S& src, int shift) {
  constexpr int C = (CORE == C_DST7 || CORE == C_DCT8) ? CORE : (TR ? core_transpose(CORE) : CORE);
  constexpr bool DEEP = !TR || DEEP_INV;
  if constexpr (C == C_DCT2) return core_c2<N, false, false, DEEP>(src, shift);
  else if constexpr (C == C_DST2) return core_c2<N, true, true, DEEP>(src, shift);
  else if constexpr (C == C_DCT3) return core_c3<N, false, false>(src, shift);
  else if constexpr (C == C_DST3) return core_c3<N, true, true>(src, shift);
  else return core_direct<N, C, TR>(src, shift);
}

// ---------------------------------------------------------------------------
// Sub-block post-adjustment: the first B outputs become Q y_{<B}, the rest
// pass through.  q[i*B/2 + j] holds the packed pair (Q[i][2j], Q[i][2j+1]).
// ---------------------------------------------------------------------------
template <int N, int B, class S>
TA_DEV void post_rows(const S& src, cparam q, int shift, int (&out)[B]) {
  const int off = 1 << (shift - 1);
#pragma unroll
  for (int i = 0; i < B; ++i) {
    int acc = off;
#pragma unroll
    for (int j = 0; j < B / 2; ++j) {
      const uint32_t pr = src.pair(2 * j, 2 * j + 1);
      acc = j == 0 ? dot2h(pr, q[i * (B / 2)], off) : dot2(pr, q[i * (B / 2) + j], acc);
    }
    out[i] = acc;
  }
}

// Both sub-block adjustments of one vector at the cost of one (section
// "Simultaneous transform adjustments", eq. 5): with the even- and
// odd-column halves E_i = sum_{j even} Q[i][j] y_j and O_i = sum_{j odd}
// Q[i][j] y_j, the DST-7 rows are Q y = E + O and the DCT-8 rows are
// S Q S y = (-1)^i (E - O).  q holds, for row i, the pairs
// (Q[i][4t], Q[i][4t+2]), t < B/4, then (Q[i][4t+1], Q[i][4t+3]).  The
// rounding offset enters the chain whose sign stays positive, so z7/z8 are
// the exact pre-shift sums of the two adjusted stages.
template <int B, class S>
TA_DEV void post_both(const S& y, cparam q, int shift, int (&z7)[B], int (&z8)[B]) {
  const int off = 1 << (shift - 1);
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const bool even = (i & 1) == 0;
    int e = 0, o = 0;
#pragma unroll
    for (int t = 0; t < B / 4; ++t) {
      const uint32_t pe = y.pair(4 * t, 4 * t + 2), po = y.pair(4 * t + 1, 4 * t + 3);
      const uint32_t qe = q[i * (B / 2) + t], qo = q[i * (B / 2) + B / 4 + t];
      if (t == 0) {
        e = even ? dot2h(pe, qe, off) : dot2h0(pe, qe);
        o = even ? dot2h0(po, qo) : dot2h(po, qo, off);
      } else {
        e = dot2(pe, qe, e);
        o = dot2(po, qo, o);
      }
    }
    z7[i] = e + o;
    z8[i] = even ? e - o : o - e;
  }
}

// One axis: compile-time core, adjustment and K (taps) or B (block).
template <int CORE_, int ADJ_, int KB_>
struct Axis {
  static constexpr int CORE = CORE_, ADJ = ADJ_, KB = KB_;
};

// Run the forward (INV = false) or inverse pass of axis AX on `in`.
// pf: forward parameters (band taps / Q pairs), pi: transposed parameters.
template <int N, class AX, bool INV, bool DEEP_INV = false, class S>
TA_DEV auto run_pass(const S& in, cparam pf, cparam pi,
                     int s_core, int a) {
  if constexpr (AX::ADJ == ADJ_NONE) {
    return core<N, AX::CORE, INV, DEEP_INV>(in, s_core);
  } else if constexpr (AX::ADJ == ADJ_BAND) {
    if constexpr (!INV) {
      const Acc<N> u = band<N, AX::KB, false>(in, pf, a);
      return core<N, AX::CORE, false>(u, s_core);
    } else {
      const Acc<N> u = core<N, AX::CORE, true, DEEP_INV>(in, s_core);
      return band<N, AX::KB, true>(u, pi, a);
    }
  } else {
    constexpr int B = AX::KB;
    if constexpr (!INV) {
      const Acc<N> y = core<N, AX::CORE, false>(in, s_core);
      Acc<N, B> r;
      r.s0 = a;
      r.s1 = s_core;
      int z[B];
      post_rows<N, B>(y, pf, a, z);
#pragma unroll
      for (int i = 0; i < N; ++i) r.a[i] = i < B ? z[i] : y.a[i];
      return r;
    } else {
      Acc<B> z;
      z.s0 = z.s1 = a;
      post_rows<N, B>(in, pi, a, z.a);
      const Split<N, B, Acc<B>, S> comp{z, in};
      return core<N, AX::CORE, true, DEEP_INV>(comp, s_core);
    }
  }
}

// ---------------------------------------------------------------------------
// Scaled-result variants of the butterfly cores and of run_pass, for the
// packed kernels: the same arithmetic with the integer tables multiplied by
// 2^SC so that a stage's shift becomes 16.  They are kept apart from the
// unscaled functions above, which the batched kernels instantiate, so that
// those kernels compile exactly as before.
// ---------------------------------------------------------------------------
// Stage result scaled so that its shift is 16: the rounded value is the high
// half of each sum, and a pair packs with one byte permute instead of two
// shifts and a saturating pack.  Only for stages whose sums provably stay
// below 2^31 and whose rounded values provably fit int16 (no clamp here).
template <int N>
struct AccHi {
  int a[N];
  TA_DEV int value(int i) const { return a[i] >> 16; }
  TA_DEV uint32_t pair(int i, int j) const {
    return perm(j >= 0 ? (uint32_t)a[j] : 0u, i >= 0 ? (uint32_t)a[i] : 0u, 0x07060302u);
  }
};

// SC scales every table entry by 2^SC (see core_c3_sc).
template <int N, int M, bool OFF, int SC, class W>
TA_DEV void c3_even_sc(const W& w, int (&e)[M], int off) {
  constexpr int ST = N / M, F = 1 << SC;
  if constexpr (M == 2) {
    const uint32_t p = w.pair(0, ST);
    const uint32_t c0 = pk2(F * c2i<2>(0, 0), F * c2i<2>(1, 0)), c1 = pk2(F * c2i<2>(0, 1), F * c2i<2>(1, 1));
    e[0] = OFF ? dot2h(p, c0, off) : dot2h0(p, c0);
    e[1] = OFF ? dot2h(p, c1, off) : dot2h0(p, c1);
  } else {
    int ee[M / 2];
    c3_even_sc<N, M / 2, OFF, SC>(w, ee, off);
#pragma unroll
    for (int n = 0; n < M / 2; ++n) {
      int o = 0;
#pragma unroll
      for (int i = 0; i < M / 4; ++i) {
        const int k1 = 4 * i + 1, k2 = 4 * i + 3;
        const uint32_t pr = w.pair(k1 * ST, k2 * ST), cf = pk2(F * c2i<M>(k1, n), F * c2i<M>(k2, n));
        o = i == 0 ? dot2h0(pr, cf) : dot2(pr, cf, o);
      }
      e[n] = ee[n] + o;
      e[M - 1 - n] = ee[n] - o;
    }
  }
}

// OSIGN applies S to the output before rounding (DST-3 = S DCT-3 R);
// IREV reverses the input.  The rounding offset enters once per output.
// SC > 0 (with shift + SC = 16) scales the table by 2^SC and returns an
// AccHi: RS(2^SC v, 16) = RS(v, shift) exactly.  The caller guarantees the
// bounds: |2^SC v| < 2^31 and |RS(v, shift)| < 2^15 for its inputs.
template <int N, bool IREV, bool OSIGN, int SC = 0, class S>
TA_DEV auto core_c3_sc(const S& src, int shift) {
  constexpr int F = 1 << SC;
  const Rev<N, IREV, S> w{src};
  const int off = 1 << (shift + SC - 1);
  std::conditional_t<(SC > 0), AccHi<N>, Acc<N>> r;
  if constexpr (SC == 0) r.s0 = r.s1 = shift;
  int ee[N / 2];
  c3_even_sc<N, N / 2, !OSIGN, SC>(w, ee, off);
#pragma unroll
  for (int n = 0; n < N / 2; ++n) {
    const int sg = (OSIGN && (n & 1)) ? -F : F;
    int o = 0;
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const int k1 = 4 * i + 1, k2 = 4 * i + 3;
      const uint32_t pr = w.pair(k1, k2), cf = pk2(sg * c2i<N>(k1, n), sg * c2i<N>(k2, n));
      o = i > 0 ? dot2(pr, cf, o) : (OSIGN ? dot2h(pr, cf, off) : dot2h0(pr, cf));
    }
    if (!OSIGN) {
      r.a[n] = ee[n] + o;
      r.a[N - 1 - n] = ee[n] - o;
    } else if (sg > 0) {      // o = O + off: y_n = E + O + off, y_{N-1-n} = -(E - O) + off
      r.a[n] = ee[n] + o;
      r.a[N - 1 - n] = o - ee[n];
    } else {                  // o = -O + off: y_n = -(E + O) + off, y_{N-1-n} = E - O + off
      r.a[n] = o - ee[n];
      r.a[N - 1 - n] = o + ee[n];
    }
  }
  return r;
}

// SC scales every table entry by 2^SC (see core_c2_sc).
template <int M, bool NEG_ODD = false, int SC = 0>
TA_DEV void c2_int_sc(const int (&v)[M], int (&z)[M], int off) {
  constexpr int F = 1 << SC;
  if constexpr (M == 2) {
    z[0] = ((NEG_ODD ? v[0] - v[1] : v[0] + v[1]) << (8 + SC)) + off;     // row 0 = 2^8
    z[1] = ((NEG_ODD ? v[0] + v[1] : v[0] - v[1]) << (8 + SC)) + off;     // 2-point row 1 = (+2^8, -2^8)
  } else {
    int e[M / 2], o[M / 2];
#pragma unroll
    for (int n = 0; n < M / 2; ++n) {
      if (!NEG_ODD) {
        e[n] = v[n] + v[M - 1 - n];
        o[n] = v[n] - v[M - 1 - n];
      } else if ((n & 1) == 0) {           // u[n] = v[n], u[M-1-n] = -v[M-1-n]
        e[n] = v[n] - v[M - 1 - n];
        o[n] = v[n] + v[M - 1 - n];
      } else {                             // u[n] = -v[n]: o[n] holds -(u[n] - u[M-1-n])
        e[n] = v[M - 1 - n] - v[n];
        o[n] = v[n] + v[M - 1 - n];
      }
    }
#pragma unroll
    for (int k = 1; k < M; k += 2) {
      int acc = off;
#pragma unroll
      for (int n = 0; n < M / 2; ++n)
        acc = mad24(o[n], (NEG_ODD && (n & 1)) ? -F * c2i<M>(k, n) : F * c2i<M>(k, n), acc);
      z[k] = acc;
    }
    int ze[M / 2];
    c2_int_sc<M / 2, false, SC>(e, ze, off);
#pragma unroll
    for (int k = 0; k < M / 2; ++k) z[2 * k] = ze[k];
  }
}

template <int M, bool NEG, bool DEEP, int SC = 0>
TA_DEV void c2_packed_sc(const uint32_t (&x)[M / 2], int (&z)[M], int off) {
  constexpr int SG = NEG ? -1 : 1, F = 1 << SC;
  uint32_t dp[M / 4], ep[M / 4];
#pragma unroll
  for (int s = 0; s < M / 4; ++s) {
    const uint32_t a = x[s], b = x[M / 2 - 1 - s];
    dp[s] = NEG ? pk_add_x(a, b) : pk_sub_x(a, b);
    ep[s] = NEG ? pk_sub_x(a, b) : pk_add_x(a, b);
  }
#pragma unroll
  for (int k = 1; k < M; k += 2) {
    int acc = off;
#pragma unroll
    for (int s = 0; s < M / 4; ++s) {
      const uint32_t cf = pk2(F * c2i<M>(k, 2 * s), SG * F * c2i<M>(k, 2 * s + 1));
      acc = s == 0 ? dot2h(dp[s], cf, off) : dot2(dp[s], cf, acc);
    }
    z[k] = acc;
  }
  int ze[M / 2];
  bool packed = false;
  if constexpr (DEEP && M / 2 >= 4) {
    if (wave_all(lanes_within_14(ep))) {
      c2_packed_sc<M / 2, NEG, DEEP, SC>(ep, ze, off);
      packed = true;
    }
  }
  if (!packed) {
    int e[M / 2];
    unpack_pairs<M / 2>(ep, e);
    c2_int_sc<M / 2, NEG, SC>(e, ze, off);
  }
#pragma unroll
  for (int k = 0; k < M / 2; ++k) z[2 * k] = ze[k];
}

// SC > 0 (with shift + SC = 16) scales the table by 2^SC and returns an
// AccHi, under the same caller guarantees as core_c3_sc.
template <int N, bool ISIGN, bool OREV, bool DEEP, int SC = 0, class S>
TA_DEV auto core_c2_sc(const S& src, int shift) {
  constexpr int F = 1 << SC;
  const int off = 1 << (shift + SC - 1);
  std::conditional_t<(SC > 0), AccHi<N>, Acc<N>> r;
  if constexpr (SC == 0) r.s0 = r.s1 = shift;
  uint32_t x[N / 2];
#pragma unroll
  for (int s = 0; s < N / 2; ++s) x[s] = src.pair(2 * s, 2 * s + 1);
  // With S applied, u_n = (-1)^n x_n: the sign of the odd-n lane moves into
  // the coefficient (odd rows) or into c2_int (even rows).
  constexpr int SG = ISIGN ? -1 : 1;
  int z[N];
  if (wave_all(lanes_within_14(x))) {
    c2_packed_sc<N, ISIGN, DEEP, SC>(x, z, off);
  } else {
#pragma unroll
    for (int k = 1; k < N; k += 2) {
      int acc = off;
#pragma unroll
      for (int s = 0; s < N / 2; ++s) {
        const uint32_t cf = pk2(F * c2i<N>(k, 2 * s), SG * F * c2i<N>(k, 2 * s + 1));
        acc = s == 0 ? dot2h(x[s], cf, off) : dot2(x[s], cf, acc);
      }
      z[k] = acc;
    }
    int e[N / 2];
#pragma unroll
    for (int n = 0; n < N / 2; ++n) {
      const int a = (n & 1) ? ((int)x[n >> 1] >> 16) : (int)(short)(x[n >> 1] & 0xffffu);
      const int m = N - 1 - n;
      const int b = (m & 1) ? ((int)x[m >> 1] >> 16) : (int)(short)(x[m >> 1] & 0xffffu);
      e[n] = ISIGN ? a - b : a + b;
    }
    int ze[N / 2];
    c2_int_sc<N / 2, ISIGN, SC>(e, ze, off);
#pragma unroll
    for (int k = 0; k < N / 2; ++k) z[2 * k] = ze[k];
  }
#pragma unroll
  for (int m = 0; m < N; ++m) r.a[m] = z[OREV ? N - 1 - m : m];
  return r;
}

// SC: see core_c3_sc and core_c2_sc (butterfly cores only).
template <int N, int CORE, bool TR, bool DEEP_INV = false, int SC = 0, class S>
TA_DEV auto core_sc(const S& src, int shift) {
  constexpr int C = (CORE == C_DST7 || CORE == C_DCT8) ? CORE : (TR ? core_transpose(CORE) : CORE);
  constexpr bool DEEP = !TR || DEEP_INV;
  static_assert(SC == 0 || C == C_DCT2 || C == C_DST2 || C == C_DCT3 || C == C_DST3,
                "scaled results are built for the butterfly cores only");
  if constexpr (C == C_DCT2) return core_c2_sc<N, false, false, DEEP, SC>(src, shift);
  else if constexpr (C == C_DST2) return core_c2_sc<N, true, true, DEEP, SC>(src, shift);
  else if constexpr (C == C_DCT3) return core_c3_sc<N, false, false, SC>(src, shift);
  else if constexpr (C == C_DST3) return core_c3_sc<N, true, true, SC>(src, shift);
  else return core_direct<N, C, TR>(src, shift);
}

// SC (band or plain passes with a butterfly core): the core's result is
// scaled to a shift of 16 (see core_c3_sc, core_c2_sc); 0 leaves it as is.  The
// caller guarantees s_core + SC = 16 and the bounds for its inputs.
template <int N, class AX, bool INV, bool DEEP_INV = false, int SC = 0, class S>
TA_DEV auto run_pass_sc(const S& in, cparam pf, cparam pi,
                     int s_core, int a) {
  static_assert(SC == 0 || AX::ADJ != ADJ_POST, "scaled results: band or plain passes only");
  if constexpr (AX::ADJ == ADJ_NONE) {
    return core_sc<N, AX::CORE, INV, DEEP_INV, SC>(in, s_core);
  } else if constexpr (AX::ADJ == ADJ_BAND) {
    if constexpr (!INV) {
      const Acc<N> u = band<N, AX::KB, false>(in, pf, a);
      return core_sc<N, AX::CORE, false, false, SC>(u, s_core);
    } else {
      const auto u = core_sc<N, AX::CORE, true, DEEP_INV, SC>(in, s_core);
      return band<N, AX::KB, true>(u, pi, a);
    }
  } else {
    constexpr int B = AX::KB;
    if constexpr (!INV) {
      const Acc<N> y = core_sc<N, AX::CORE, false>(in, s_core);
      Acc<N, B> r;
      r.s0 = a;
      r.s1 = s_core;
      int z[B];
      post_rows<N, B>(y, pf, a, z);
#pragma unroll
      for (int i = 0; i < N; ++i) r.a[i] = i < B ? z[i] : y.a[i];
      return r;
    } else {
      Acc<B> z;
      z.s0 = z.s1 = a;
      post_rows<N, B>(in, pi, a, z.a);
      const Split<N, B, Acc<B>, S> comp{z, in};
      return core_sc<N, AX::CORE, true, DEEP_INV>(comp, s_core);
    }
  }
}

}  // namespace fx
}  // namespace ta
