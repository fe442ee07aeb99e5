// Stages of the general transforms (gen_kernels.hip, bwd_kernels.hip): one
// 1-D stage of an axis program applied to a vector in registers, and one
// vector of a tile in LDS run through its program.
#pragma once

#include "fp.hpp"
#include "fx.hpp"
#include "kernels.hpp"

namespace ta {
namespace gen {

// A stage's parameters live in the constant address space: they are
// wave-uniform and arrive by scalar loads.
TA_DEV GenStage load_stage(const GenProg* pr, int i) {
  typedef const __attribute__((address_space(4))) int32_t* cint;
  typedef const __attribute__((address_space(4))) uint64_t* cu64;
  const cint w = (cint)&pr->st[i];
  GenStage s;
  s.op = w[0];
  s.arg = w[1];
  s.tr = w[2];
  s.adj = w[3];
  s.p = reinterpret_cast<const void*>(*(cu64)&pr->st[i].p);
  return s;
}
TA_DEV int load_nst(const GenProg* pr) {
  typedef const __attribute__((address_space(4))) int32_t* cint;
  return *(cint)&pr->nst;
}

// ---------------------------------------------------------------- int16 stages
template <int N, class A>
TA_DEV void pack_into(const A& acc, fx::Packed<N>& x) {
#pragma unroll
  for (int s = 0; s < N / 2; ++s) x.p[s] = acc.pair(2 * s, 2 * s + 1);
}

// z = M x for a dense N x N integer matrix, row k of m holding the packed
// pairs (M[k][2j], M[k][2j+1]).
template <int N, class S>
TA_DEV fx::Acc<N> dense(const S& src, cparam m, int shift) {
  fx::Acc<N> r;
  r.s0 = r.s1 = shift;
  const int off = 1 << (shift - 1);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int acc = off;
#pragma unroll
    for (int j = 0; j < N / 2; ++j) acc = dot2(src.p[j], m[k * (N / 2) + j], acc);
    r.a[k] = acc;
  }
  return r;
}

template <int N, int K>
TA_DEV void band_fx(fx::Packed<N>& x, cparam taps, int tr, int shift) {
  if (tr)
    pack_into<N>(fx::band<N, K, true>(x, taps, shift), x);
  else
    pack_into<N>(fx::band<N, K, false>(x, taps, shift), x);
}

// First B entries become RS(Q x_{<B}, a), the rest pass through.
template <int N, int B>
TA_DEV void post_fx(fx::Packed<N>& x, cparam q, int a) {
  if constexpr (B <= N) {
    int z[B];
    fx::post_rows<N, B>(x, q, a, z);
#pragma unroll
    for (int s = 0; s < B / 2; ++s) x.p[s] = satpk(z[2 * s] >> a, z[2 * s + 1] >> a);
  }
}

template <int N>
TA_DEV void apply_fx(const GenStage& st, fx::Packed<N>& x, int s_core, int a) {
  const int sh = st.adj ? a : s_core;
  const cparam p = as_cparam(st.p);
  switch (st.op) {
    case GS_C2: pack_into<N>(fx::core_c2<N, false, false, false>(x, sh), x); break;
    case GS_S2: pack_into<N>(fx::core_c2<N, true, true, false>(x, sh), x); break;
    case GS_C3: pack_into<N>(fx::core_c3<N, false, false>(x, sh), x); break;
    case GS_S3: pack_into<N>(fx::core_c3<N, true, true>(x, sh), x); break;
    case GS_DENSE: pack_into<N>(dense<N>(x, p, sh), x); break;
    case GS_BAND:
      switch (st.arg) {
        case 2: band_fx<N, 2>(x, p, st.tr, sh); break;
        case 4: band_fx<N, 4>(x, p, st.tr, sh); break;
        case 6: band_fx<N, 6>(x, p, st.tr, sh); break;
        default: band_fx<N, 8>(x, p, st.tr, sh); break;
      }
      break;
    default:   // GS_POST
      switch (st.arg) {
        case 4: post_fx<N, 4>(x, p, sh); break;
        case 8: post_fx<N, 8>(x, p, sh); break;
        default: post_fx<N, 16>(x, p, sh); break;
      }
      break;
  }
}

// One vector of a tile in LDS: N int16 at base + i * stride halfwords (a row
// when stride == 1: dword-aligned, read and written as dwords; a column
// otherwise).  Runs the program's stages and writes the result in place.
template <int N>
TA_DEV void vec_fx(uint16_t* lds, int base, int stride, const GenProg* pr, int s_core, int a) {
  fx::Packed<N> x;
  if (stride == 1) {
    const uint32_t* s = reinterpret_cast<const uint32_t*>(lds + base);
#pragma unroll
    for (int j = 0; j < N / 2; ++j) x.p[j] = s[j];
  } else {
#pragma unroll
    for (int j = 0; j < N / 2; ++j)
      x.p[j] = (uint32_t)lds[base + 2 * j * stride] | ((uint32_t)lds[base + (2 * j + 1) * stride] << 16);
  }
  const int nst = load_nst(pr);
#pragma unroll 1
  for (int i = 0; i < nst; ++i) apply_fx<N>(load_stage(pr, i), x, s_core, a);
  if (stride == 1) {
    uint32_t* d = reinterpret_cast<uint32_t*>(lds + base);
#pragma unroll
    for (int j = 0; j < N / 2; ++j) d[j] = x.p[j];
  } else {
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      lds[base + 2 * j * stride] = (uint16_t)x.p[j];
      lds[base + (2 * j + 1) * stride] = (uint16_t)(x.p[j] >> 16);
    }
  }
}

// ---------------------------------------------------------------- fp32 stages
template <int N>
TA_DEV fp::Vec<N> dense_f(const fp::Vec<N>& x, const float* __restrict__ m) {
  typedef const __attribute__((address_space(4))) float* cfl;
  const cfl c = (cfl)m;
  fp::Vec<N> z;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int n = 0; n < N; ++n) acc = __builtin_fmaf(c[k * N + n], x.v[n], acc);
    z.v[k] = acc;
  }
  return z;
}

template <int N, int K>
TA_DEV void band_f(fp::Vec<N>& x, const float* taps, int tr) {
  x = tr ? fp::band<N, K, true>(x, taps) : fp::band<N, K, false>(x, taps);
}

template <int N, int B>
TA_DEV void post_f(fp::Vec<N>& x, const float* q) {
  if constexpr (B <= N) x = fp::post<N, B>(x, q);
}

template <int N>
TA_DEV void apply_f(const GenStage& st, fp::Vec<N>& x) {
  const float* p = static_cast<const float*>(st.p);
  switch (st.op) {
    case GS_C2: x = fp::core_c2<N, false, false>(x); break;
    case GS_S2: x = fp::core_c2<N, true, true>(x); break;
    case GS_C3: x = fp::core_c3<N, false, false>(x); break;
    case GS_S3: x = fp::core_c3<N, true, true>(x); break;
    case GS_DENSE: x = dense_f<N>(x, p); break;
    case GS_BAND:
      switch (st.arg) {
        case 2: band_f<N, 2>(x, p, st.tr); break;
        case 4: band_f<N, 4>(x, p, st.tr); break;
        case 6: band_f<N, 6>(x, p, st.tr); break;
        default: band_f<N, 8>(x, p, st.tr); break;
      }
      break;
    default:   // GS_POST
      switch (st.arg) {
        case 4: post_f<N, 4>(x, p); break;
        case 8: post_f<N, 8>(x, p); break;
        default: post_f<N, 16>(x, p); break;
      }
      break;
  }
}

template <int N>
TA_DEV void vec_f(float* lds, int base, int stride, const GenProg* pr) {
  fp::Vec<N> x;
#pragma unroll
  for (int i = 0; i < N; ++i) x.v[i] = lds[base + i * stride];
  const int nst = load_nst(pr);
#pragma unroll 1
  for (int i = 0; i < nst; ++i) apply_f<N>(load_stage(pr, i), x);
#pragma unroll
  for (int i = 0; i < N; ++i) lds[base + i * stride] = x.v[i];
}

}  // namespace gen
}  // namespace ta
