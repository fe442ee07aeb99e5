// FP32 1-D stages of the adjusted transforms (orthonormal, no rounding).
//
// Same structure as the fixed-point stages: band (K taps per row, runtime
// fp32 parameters), DCT-2 / DCT-3 butterflies with the section 2.1 R/S maps
// for DST-2 / DST-3, direct DST-7 / DCT-8, and the B x B sub-block.  All
// butterfly constants are the N-point DCT-2 entries C[k][n] = s_k cos(pi k
// (2n+1) / 2N) (s_0 = 1/sqrt N, s_k = sqrt(2/N)); every level of the even/odd
// recursion uses entries of the original N-point matrix, so no rescaling is
// needed between levels.
#pragma once

#include "common.hpp"

namespace ta {
namespace fp {

template <int N>
TA_DEV constexpr double c2_scale(int k) {
  // 1/sqrt(N) and sqrt(2/N) for N = 4..64
  constexpr double inv_sqrt[7] = {1.0, 0.70710678118654752, 0.5, 0.35355339059327376, 0.25,
                                  0.17677669529663688, 0.125};
  constexpr double sqrt2_over[7] = {1.41421356237309505, 1.0, 0.70710678118654752, 0.5,
                                    0.35355339059327376, 0.25, 0.17677669529663688};
  return k == 0 ? inv_sqrt[ilog2(N)] : sqrt2_over[ilog2(N)];
}

template <int N>
TA_DEV constexpr float c2f(int k, int n) {
  return (float)(c2_scale<N>(k) * ta_cos_64[k * (64 / N)][n]);
}

template <int N>
struct Vec {
  float v[N];
};

// band: u[i] = sum_t A[i][start_i + t] x[start_i + t]; taps[i*K + t]
template <int K, bool TR>
TA_DEV constexpr int band_start(int i) {
  return TR ? i - K / 2 + 1 - (i & 1) : i - K / 2 + ((i + K / 2) & 1);
}

template <int N, int K, bool TR>
TA_DEV Vec<N> band(const Vec<N>& x, const float* __restrict__ taps) {
  Vec<N> u;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int st = band_start<K, TR>(i);
    float acc = 0.0f;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int c = st + t;
      if (c < 0 || c >= N) continue;
      acc = __builtin_fmaf(taps[i * K + t], x.v[c], acc);
    }
    u.v[i] = acc;
  }
  return u;
}

// DCT-3 butterfly on w[k] = x[IREV ? N-1-k : k]: z[n] = sum_k C[k][n] w[k];
// OSIGN negates odd outputs (DST-3 = S DCT-3 R).
template <int N, int M, bool IREV>
TA_DEV void c3_level(const Vec<N>& x, float (&e)[M]) {
  constexpr int ST = N / M;
  auto w = [&](int k) { return x.v[IREV ? N - 1 - k : k]; };
  if constexpr (M == 2) {
    e[0] = c2f<N>(0, 0) * w(0) + c2f<N>(ST, 0) * w(ST);
    e[1] = c2f<N>(0, 1) * w(0) + c2f<N>(ST, 1) * w(ST);
  } else {
    float ee[M / 2];
    c3_level<N, M / 2, IREV>(x, ee);
#pragma unroll
    for (int n = 0; n < M / 2; ++n) {
      float o = 0.0f;
#pragma unroll
      for (int i = 0; i < M / 2; ++i) o = __builtin_fmaf(c2f<N>((2 * i + 1) * ST, n), w((2 * i + 1) * ST), o);
      e[n] = ee[n] + o;
      e[M - 1 - n] = ee[n] - o;
    }
  }
}

template <int N, bool IREV, bool OSIGN>
TA_DEV Vec<N> core_c3(const Vec<N>& x) {
  float e[N];
  c3_level<N, N, IREV>(x, e);
  Vec<N> z;
#pragma unroll
  for (int n = 0; n < N; ++n) z.v[n] = (OSIGN && (n & 1)) ? -e[n] : e[n];
  return z;
}

// DCT-2 butterfly on x'[n] = (ISIGN ? (-1)^n : 1) x[n]; output reversed when OREV.
template <int N, int M>
TA_DEV void c2_level(const float (&v)[M], float (&z)[M]) {
  constexpr int ST = N / M;   // v holds the level's inputs; output k corresponds to C row k*ST
  if constexpr (M == 2) {
    z[0] = c2f<N>(0, 0) * (v[0] + v[1]);
    z[1] = c2f<N>(ST, 0) * (v[0] - v[1]);
  } else {
    float e[M / 2], o[M / 2];
#pragma unroll
    for (int n = 0; n < M / 2; ++n) {
      e[n] = v[n] + v[M - 1 - n];
      o[n] = v[n] - v[M - 1 - n];
    }
#pragma unroll
    for (int k = 1; k < M; k += 2) {
      float acc = 0.0f;
#pragma unroll
      for (int n = 0; n < M / 2; ++n) acc = __builtin_fmaf(c2f<N>(k * ST, n), o[n], acc);
      z[k] = acc;
    }
    float ze[M / 2];
    c2_level<N, M / 2>(e, ze);
#pragma unroll
    for (int k = 0; k < M / 2; ++k) z[2 * k] = ze[k];
  }
}

template <int N, bool ISIGN, bool OREV>
TA_DEV Vec<N> core_c2(const Vec<N>& x) {
  float v[N], z[N];
#pragma unroll
  for (int n = 0; n < N; ++n) v[n] = (ISIGN && (n & 1)) ? -x.v[n] : x.v[n];
  c2_level<N, N>(v, z);
  Vec<N> r;
#pragma unroll
  for (int m = 0; m < N; ++m) r.v[m] = z[OREV ? N - 1 - m : m];
  return r;
}

template <int N, int KIND>
TA_DEV constexpr float dmatf(int k, int n) {
  return KIND == C_DST7 ? (float)s7f<N>(k, n)
                        : (float)((k & 1) ? -s7f<N>(k, N - 1 - n) : s7f<N>(k, N - 1 - n));
}

template <int N, int KIND, bool TR>
TA_DEV Vec<N> core_direct(const Vec<N>& x) {
  Vec<N> z;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int n = 0; n < N; ++n) acc = __builtin_fmaf(TR ? dmatf<N, KIND>(n, k) : dmatf<N, KIND>(k, n), x.v[n], acc);
    z.v[k] = acc;
  }
  return z;
}

template <int N, int CORE, bool TR>
TA_DEV Vec<N> core(const Vec<N>& x) {
  constexpr int C = (CORE == C_DST7 || CORE == C_DCT8) ? CORE : (TR ? core_transpose(CORE) : CORE);
  if constexpr (C == C_DCT2) return core_c2<N, false, false>(x);
  else if constexpr (C == C_DST2) return core_c2<N, true, true>(x);
  else if constexpr (C == C_DCT3) return core_c3<N, false, false>(x);
  else if constexpr (C == C_DST3) return core_c3<N, true, true>(x);
  else return core_direct<N, C, TR>(x);
}

// first B entries replaced by Q y_{<B}; q row-major B x B (already transposed
// for the inverse by the host)
template <int N, int B>
TA_DEV Vec<N> post(const Vec<N>& y, const float* __restrict__ q) {
  Vec<N> z = y;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < B; ++j) acc = __builtin_fmaf(q[i * B + j], y.v[j], acc);
    z.v[i] = acc;
  }
  return z;
}

template <int N, class AX, bool INV>
TA_DEV Vec<N> run_pass(const Vec<N>& x, const float* __restrict__ pf, const float* __restrict__ pi) {
  if constexpr (AX::ADJ == ADJ_NONE) {
    return core<N, AX::CORE, INV>(x);
  } else if constexpr (AX::ADJ == ADJ_BAND) {
    if constexpr (!INV) return core<N, AX::CORE, false>(band<N, AX::KB, false>(x, pf));
    else return band<N, AX::KB, true>(core<N, AX::CORE, true>(x), pi);
  } else {
    if constexpr (!INV) return post<N, AX::KB>(core<N, AX::CORE, false>(x), pf);
    else return core<N, AX::CORE, true>(post<N, AX::KB>(x, pi));
  }
}

}  // namespace fp
}  // namespace ta
