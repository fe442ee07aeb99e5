// Batched adjustment design search (section 2, Fig. 1): many independent
// candidates (base B, target D, pre or post adjustment, random start), each
// minimising
//   f(M) = lam sum_ij M_ij^2 / (0.05 + |M_ij|) + sum_ij w_i (H_ij - D_ij)^2,
//   w_i = exp(-i ln(100) / N),  H = B M (pre) or M B (post),
// over orthogonal M = G(theta) J, where G is N layers of parallel Givens
// rotations on adjacent pairs (layer l on the pairs starting at l mod 2, angle
// order layer by layer) and J = diag(sigma, 1, ..., 1).  Each candidate runs
// `steps` Adam updates and a final evaluation inside one launch.
//
// One workgroup per candidate; thread t is (pair slot r, column group jg) =
// (t mod N/2, t div N/2) and owns rows 2r, 2r+1 of its CW columns (jg + q N/CW).
// The N/2 slots of a column group are consecutive lanes inside one 16-lane
// DPP row, so the matrices of the layer chain stay in registers: an even
// layer rotates rows (2r, 2r+1), both the thread's own; an odd layer rotates
// rows (2r+1, 2r+2), and the row owned by the next slot arrives by a
// row_shl:1 DPP move (row 2r-1 of the previous slot by row_shr:1).  The 2N
// layers of a step (forward, and backward recovering each layer's input by
// the transposed rotation, orthogonal so nothing is stored) touch no LDS.
// LDS holds what is shared: the products with B (M and the error adjoint X),
// the angle tables, and each thread's angle-gradient terms, summed per angle
// over the column groups in a fixed order once the backward pass is done.
// Everything is FP64.
#include <math.h>

#include "kernels.hpp"

namespace ta {
namespace {

constexpr double kSparseEps = 0.05;

// first angle of layer l: even layers have N/2 pairs, odd layers N/2 - 1
template <int N>
__device__ inline int layer_start(int l) {
  return (l >> 1) * (N - 1) + ((l & 1) ? N / 2 : 0);
}

// Workgroup-wide barrier; a one-wave workgroup only needs its LDS traffic
// ordered, which a wavefront-scope fence gives.
template <int T>
__device__ inline void group_sync() {
  if constexpr (T <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Two columns a thread: the second column gives each thread independent
// work between the dependent steps of the chain, which measured faster than
// one column a thread on twice the waves (N = 16: 3.6 against 5.3 ms).

constexpr int kRowShl1 = 0x101;   // DPP: lane i reads lane i + 1 of its row
constexpr int kRowShr1 = 0x111;   // DPP: lane i reads lane i - 1 of its row

template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int N, int CW>
__global__ __launch_bounds__((N / 2) * (N / CW)) void design_search(DesignArgs a) {
  constexpr int HN = N / 2;                  // pair slots
  constexpr int NC = N / CW;                 // column groups (threads per slot)
  constexpr int T = HN * NC;
  static_assert((T <= 1024 && T % 64 == 0) || T < 64, "whole waves, or one partial wave");
  static_assert(16 % HN == 0, "the slots of a column group inside one DPP row");
  constexpr int NA = N * (N - 1) / 2;
  // Row pitch N + 1 doubles: the 16 lanes an LDS access serves together are
  // up to 16 slots r of one or two column groups, and rows 2r then start
  // 4r dwords (mod 64) apart, in distinct banks
  constexpr int LP = N + 1;
  __shared__ double Ms[N * LP], Bs[N * LP], Xs[N * LP];
  // cs_c / cs_s hold one more entry, the identity rotation (1, 0), which the
  // threads of a missing pair slot (the ends of an odd layer) apply: the
  // layers then run without selects
  __shared__ double th[NA], mo[NA], ve[NA], cs_c[NA + 1], cs_s[NA + 1], gr[NA];
  // angle-gradient term of each (column group g, angle k) at g * TP + k:
  // the slots of a group write consecutive angles, and TP = 8 mod 32 doubles
  // puts a second group's run right after the first in the banks
  constexpr int TP = NA + (40 - NA % 32) % 32;
  __shared__ double terms[NC * TP];
  __shared__ double part[T >= 64 ? 2 * (T / 64) : 2];   // per-wave objective partials
  __shared__ int bad;

  const int cand = blockIdx.x;
  const int t = threadIdx.x, r = t % HN, jg = t / HN;
  const int i0 = 2 * r, i1 = 2 * r + 1;      // rows owned in each of the thread's columns

  if (t == 0) {
    const int* c = a.cands + 4 * (int64_t)cand;
    const int b = c[0], d = c[1], mode = c[2], sg = c[3];
    bad = (b < 0 || b >= a.nmat || d < 0 || d >= a.nmat || (mode != 0 && mode != 1) || (sg != 1 && sg != -1));
  }
  group_sync<T>();
  if (bad) {
    if (t == 0) {
      const double nan = __builtin_nan("");
      for (int k = 0; k < 3; ++k) a.obj[3 * (int64_t)cand + k] = nan;
    }
    return;
  }
  const int* c = a.cands + 4 * (int64_t)cand;
  const int mode = c[2];
  const double sigma = (double)c[3];
  const double* bm = a.mats + (int64_t)c[0] * N * N;
  const double* dm = a.mats + (int64_t)c[1] * N * N;
  double* theta = a.theta + (int64_t)cand * NA;
  for (int k = t; k < N * N; k += T) Bs[(k / N) * LP + k % N] = bm[k];
  double d0[CW], d1[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) {
    const int j = jg + q * NC;
    d0[q] = dm[i0 * N + j];
    d1[q] = dm[i1 * N + j];
  }
  for (int k = t; k < NA; k += T) {
    th[k] = theta[k];
    mo[k] = 0.0;
    ve[k] = 0.0;
  }
  if (t == 0) {
    cs_c[NA] = 1.0;
    cs_s[NA] = 0.0;
  }
  const double alpha = log(100.0) / N;
  const double w0 = exp(-alpha * i0), w1 = exp(-alpha * i1);
  double b1t = 1.0, b2t = 1.0;   // beta1^t, beta2^t
  group_sync<T>();

  for (int step = 0; step <= a.steps; ++step) {
    const bool last = step == a.steps;
    for (int k = t; k < NA; k += T) sincos(th[k], &cs_s[k], &cs_c[k]);
    group_sync<T>();
    // forward: M = G_{N-1} ... G_0 I, rows i0, i1 of the thread's columns
    double m0[CW], m1[CW];
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int j = jg + q * NC;
      m0[q] = (i0 == j) ? 1.0 : 0.0;
      m1[q] = (i1 == j) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const int k = layer_start<N>(l) + r;
      if ((l & 1) == 0) {
        const double cc = cs_c[k], ss = cs_s[k];
#pragma unroll
        for (int q = 0; q < CW; ++q) {
          const double u0 = m0[q], u1 = m1[q];
          m0[q] = cc * u0 - ss * u1;
          m1[q] = ss * u0 + cc * u1;
        }
      } else {
        // straight-line code so that the angle loads of later layers can be
        // issued early; a missing slot rotates by the identity entry
        const int ku = r + 1 < HN ? k : NA, kl = r >= 1 ? k - 1 : NA;   // upper row of slot r, lower of r - 1
        const double cu = cs_c[ku], su = cs_s[ku], cl = cs_c[kl], sl = cs_s[kl];
#pragma unroll
        for (int q = 0; q < CW; ++q) {
          const double below = dpp_f64<kRowShl1>(m0[q]);   // row 2r + 2
          const double above = dpp_f64<kRowShr1>(m1[q]);   // row 2r - 1
          const double n1 = cu * m1[q] - su * below, n0 = sl * above + cl * m0[q];
          m1[q] = n1;
          m0[q] = n0;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int j = jg + q * NC;
      Ms[i0 * LP + j] = m0[q];
      Ms[i1 * LP + j] = m1[q];
    }
    group_sync<T>();
    // M = G J, J = diag(sigma, 1, ...): the J factor is applied where M is
    // read (column 0 times sigma).  Per column: H rows i0, i1, the error and
    // its adjoint 2 w (H - D)
    double mm0[CW], mm1[CW], sp = 0.0, er = 0.0;
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int j = jg + q * NC;
      const double js = j == 0 ? sigma : 1.0;
      double h0 = 0.0, h1 = 0.0;
      if (mode == 0) {   // H = B M
#pragma unroll 8
        for (int k = 0; k < N; ++k) {
          const double mk = Ms[k * LP + j];
          h0 += Bs[i0 * LP + k] * mk;
          h1 += Bs[i1 * LP + k] * mk;
        }
        h0 *= js;
        h1 *= js;
      } else {           // H = M B: H[i][j] = sum_k M[i][k] B[k][j], M[i][0] scaled by sigma
#pragma unroll 8
        for (int k = 0; k < N; ++k) {
          const double bk = Bs[k * LP + j];
          const double sk = k == 0 ? sigma : 1.0;
          h0 += sk * Ms[i0 * LP + k] * bk;
          h1 += sk * Ms[i1 * LP + k] * bk;
        }
      }
      const double e0 = h0 - d0[q], e1 = h1 - d1[q];
      mm0[q] = js * m0[q];   // entries of M = G J
      mm1[q] = js * m1[q];
      if (last) {
        sp += mm0[q] * mm0[q] / (kSparseEps + fabs(mm0[q])) + mm1[q] * mm1[q] / (kSparseEps + fabs(mm1[q]));
        er += w0 * e0 * e0 + w1 * e1 * e1;
        if (a.adj) {
          double* out = a.adj + (int64_t)cand * N * N;
          out[i0 * N + j] = mm0[q];
          out[i1 * N + j] = mm1[q];
        }
      }
      Xs[i0 * LP + j] = 2.0 * w0 * e0;
      Xs[i1 * LP + j] = 2.0 * w1 * e1;
    }
    if (last) {
      // objective: sparsity of M and weighted error, reduced in a fixed order
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) {
        if (m < T) {
          sp += __shfl_xor(sp, m);
          er += __shfl_xor(er, m);
        }
      }
      if ((t & 63) == 0) {
        part[2 * (t >> 6)] = sp;
        part[2 * (t >> 6) + 1] = er;
      }
    }
    group_sync<T>();
    if (last && t == 0) {
      double sps = 0.0, ers = 0.0;
      for (int w = 0; w < (T + 63) / 64; ++w) {
        sps += part[2 * w];
        ers += part[2 * w + 1];
      }
      a.obj[3 * (int64_t)cand] = a.lam * sps + ers;
      a.obj[3 * (int64_t)cand + 1] = sps;
      a.obj[3 * (int64_t)cand + 2] = ers;
    }
    // adjoint of M = G J at (i, j): lam phi'(M) + (B^T X or X B^T), then times J
    double g0[CW], g1[CW];
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int j = jg + q * NC;
      const double js = j == 0 ? sigma : 1.0;
      double x0 = 0.0, x1 = 0.0;
      if (mode == 0) {   // dM = B^T X: dM[i][j] = sum_k B[k][i] X[k][j]
#pragma unroll 8
        for (int k = 0; k < N; ++k) {
          const double xk = Xs[k * LP + j];
          x0 += Bs[k * LP + i0] * xk;
          x1 += Bs[k * LP + i1] * xk;
        }
      } else {           // dM = X B^T: dM[i][j] = sum_k X[i][k] B[j][k]
#pragma unroll 8
        for (int k = 0; k < N; ++k) {
          const double bj = Bs[j * LP + k];
          x0 += Xs[i0 * LP + k] * bj;
          x1 += Xs[i1 * LP + k] * bj;
        }
      }
      const double a0 = fabs(mm0[q]), a1 = fabs(mm1[q]);
      x0 += a.lam * mm0[q] * (2.0 * kSparseEps + a0) / ((kSparseEps + a0) * (kSparseEps + a0));
      x1 += a.lam * mm1[q] * (2.0 * kSparseEps + a1) / ((kSparseEps + a1) * (kSparseEps + a1));
      g0[q] = js * x0;
      g1[q] = js * x1;
    }
    // backward through the layers: each layer's angle term from its outputs,
    // then both the activations and the adjoint stepped back through it
#pragma unroll
    for (int l = N - 1; l >= 0; --l) {
      const int k = layer_start<N>(l) + r;
      if ((l & 1) == 0) {
        const double cc = cs_c[k], ss = cs_s[k];
        double term = 0.0;
#pragma unroll
        for (int q = 0; q < CW; ++q) {
          const double vp = m0[q], vq = m1[q], gp = g0[q], gq = g1[q];
          term += -gp * vq + gq * vp;
          m0[q] = cc * vp + ss * vq;
          m1[q] = -ss * vp + cc * vq;
          g0[q] = cc * gp + ss * gq;
          g1[q] = -ss * gp + cc * gq;
        }
        terms[jg * TP + k] = term;
      } else {
        const bool up = r + 1 < HN;             // upper row of slot r; lower row of slot r - 1 if r >= 1
        const int ku = up ? k : NA, kl = r >= 1 ? k - 1 : NA;
        const double cu = cs_c[ku], su = cs_s[ku], cl = cs_c[kl], sl = cs_s[kl];
        double term = 0.0;
#pragma unroll
        for (int q = 0; q < CW; ++q) {
          const double bm_ = dpp_f64<kRowShl1>(m0[q]), bg_ = dpp_f64<kRowShl1>(g0[q]);   // rows 2r + 2
          const double am_ = dpp_f64<kRowShr1>(m1[q]), ag_ = dpp_f64<kRowShr1>(g1[q]);   // rows 2r - 1
          const double vp = m1[q], gp = g1[q];
          term += -gp * bm_ + bg_ * vp;
          m1[q] = cu * vp + su * bm_;
          g1[q] = cu * gp + su * bg_;
          m0[q] = -sl * am_ + cl * m0[q];
          g0[q] = -sl * ag_ + cl * g0[q];
        }
        if (up) terms[jg * TP + k] = term;
      }
    }
    group_sync<T>();
    // each angle's gradient: its terms summed over the column groups, in order
    for (int k = t; k < NA; k += T) {
      double s = 0.0;
#pragma unroll
      for (int g = 0; g < NC; ++g) s += terms[g * TP + k];
      gr[k] = s;
    }
    if (last) break;
    // Adam (Kingma and Ba) with bias correction
    b1t *= a.beta1;
    b2t *= a.beta2;
    for (int k = t; k < NA; k += T) {
      const double g = gr[k];
      mo[k] = a.beta1 * mo[k] + (1.0 - a.beta1) * g;
      ve[k] = a.beta2 * ve[k] + (1.0 - a.beta2) * g * g;
      const double mh = mo[k] / (1.0 - b1t);
      const double vh = ve[k] / (1.0 - b2t);
      th[k] -= a.lr * mh / (sqrt(vh) + a.eps);
    }
    group_sync<T>();
  }
  for (int k = t; k < NA; k += T) {
    theta[k] = th[k];
    if (a.grad) a.grad[(int64_t)cand * NA + k] = gr[k];
  }
}

}  // namespace

// threads per workgroup: (n / 2) x (n / CW); n = 16 and 32 run two columns
// a thread (one wave, four waves a candidate)
const void* design_kernel(int n, int* threads) {
  switch (n) {
    case 4: *threads = 8; return reinterpret_cast<const void*>(&design_search<4, 1>);
    case 8: *threads = 32; return reinterpret_cast<const void*>(&design_search<8, 1>);
    case 16: *threads = 64; return reinterpret_cast<const void*>(&design_search<16, 2>);
    case 32: *threads = 256; return reinterpret_cast<const void*>(&design_search<32, 2>);
    default: return nullptr;
  }
}

}  // namespace ta
