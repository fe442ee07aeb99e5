// Backward of the fp32 block-list transform (ta_transform_bwd).
//
// Forward, per block: Y = H_v X H_h^T, every axis a program of stages (a
// band A before the base, or a sub-block C after it; flipped axes as the
// host folds them: core' = S B R, A' = R A R, Q' = S Q S).  For dL/dY = G_Y:
//   dL/dX = H_v^T G_Y H_h: the columns of G_Y through the vertical inverse
//           program (G_W = H_v^T G_Y), then the rows of G_W through the
//           horizontal inverse program;
//   for an axis on the angle set, the gradient of its adjustment matrix,
//   summed over the vectors it transforms:
//     band      dL/dA  += g_v u^T on the K-tap support, u = R^f x the input
//               of A and g_v = R^f core'^T g the gradient at its output;
//     sub-block dL/dQ  += S^f (g_z u'^T) S^f on the B x B block, u' = core' x;
//   the rows of X with the rows of G_W for the horizontal axis, the columns
//   of W = X H_h^T with the columns of G_Y for the vertical one.
// One workgroup runs one block at a time (a persistent grid over the list);
// per matrix entry, each wave sums its vectors' products with a fixed
// butterfly of shuffles and the four wave sums are added in wave order into
// the workgroup's accumulator, written as one partial row per workgroup.
// bwd_chain sums the rows in a fixed order (FP64) and applies the chain rule
// through the rotations (section 2: sequential sets of Givens rotations):
// with m_l = left_l^T Gbar right_l^T (left_l the rotations after l, right_l
// the ones before), the angle of rotation (p, q) in step l has gradient
// -s m[p][p] - c m[p][q] + c m[q][p] - s m[q][q], and m_{l+1} =
// G_{l+1} m_l G_l^T.  All results are bitwise repeatable.
#include "gen.hpp"

namespace ta {
namespace {

using gen::apply_f;
using gen::load_stage;
using gen::vec_f;

constexpr int kBwdMaxSide = 64;
constexpr int kBwdPitch = kBwdMaxSide + 1;

// Workgroup sum of v (zero in inactive threads) into acc[e], fixed order.
TA_DEV void wg_accumulate(float v, int e, float* red, int ne) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * kBwdMaxEntries + e] = v;
  (void)ne;
}

TA_DEV void wg_fold(float* red, float* acc, int ne) {
  __syncthreads();
  for (int e = threadIdx.x; e < ne; e += 256)
    acc[e] += ((red[e] + red[kBwdMaxEntries + e]) + red[2 * kBwdMaxEntries + e]) + red[3 * kBwdMaxEntries + e];
  __syncthreads();
}

// band: entry (i, t) = g[i] * u[s_i + t], s_i = i - K/2 + ((i + K/2) & 1)
template <int N, int K>
TA_DEV void band_entries(const float (&u)[N], const float (&g)[N], float* red, float* acc) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int st = i - K / 2 + ((i + K / 2) & 1);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int j = st + t;
      if (j >= 0 && j < N)
        wg_accumulate(g[i] * u[j], i * K + t, red, N * K);
      else if ((threadIdx.x & 63) == 0)
        red[(threadIdx.x >> 6) * kBwdMaxEntries + i * K + t] = 0.0f;   // outside the vector: no entry
    }
  }
  wg_fold(red, acc, N * K);
}

// sub-block: entry (i, j) = sign * g[i] * u[j], i, j < B
template <int N, int B>
TA_DEV void post_entries(const float (&u)[N], const float (&g)[N], bool flip, float* red, float* acc) {
  if constexpr (B <= N) {
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const float v = g[i] * u[j];
        wg_accumulate((flip && ((i + j) & 1)) ? -v : v, i * B + j, red, B * B);
      }
    wg_fold(red, acc, B * B);
  }
}

// One axis of one block on the angle set: vectors of length N at base +
// i * stride (x from lx, g from lg), thread t < nvec holding vector t.
template <int N>
TA_DEV void axis_grad(const BwdArgs& a, const float* lx, const float* lg, int vbase, int vstep, int stride,
                      int nvec, const GenProg* pf, const GenProg* pi, bool flip, float* red, float* acc) {
  const bool act = (int)threadIdx.x < nvec;
  fp::Vec<N> x, g;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    x.v[i] = act ? lx[vbase + threadIdx.x * vstep + i * stride] : 0.0f;
    g.v[i] = act ? lg[vbase + threadIdx.x * vstep + i * stride] : 0.0f;
  }
  float u[N], gv[N];
  if (a.kind == TA_ADJ_BAND) {
    apply_f<N>(load_stage(pi, 0), g);          // core'^T g: first stage of the inverse program
#pragma unroll
    for (int i = 0; i < N; ++i) {
      u[i] = flip ? x.v[N - 1 - i] : x.v[i];
      gv[i] = flip ? g.v[N - 1 - i] : g.v[i];
    }
    switch (a.k_or_b) {
      case 2: band_entries<N, 2>(u, gv, red, acc); break;
      case 4: band_entries<N, 4>(u, gv, red, acc); break;
      case 6: band_entries<N, 6>(u, gv, red, acc); break;
      default: band_entries<N, 8>(u, gv, red, acc); break;
    }
  } else {
    apply_f<N>(load_stage(pf, 0), x);          // u' = core' x: first stage of the forward program
#pragma unroll
    for (int i = 0; i < N; ++i) {
      u[i] = x.v[i];
      gv[i] = g.v[i];
    }
    switch (a.k_or_b) {
      case 4: post_entries<N, 4>(u, gv, flip, red, acc); break;
      case 8: post_entries<N, 8>(u, gv, flip, red, acc); break;
      default: post_entries<N, 16>(u, gv, flip, red, acc); break;
    }
  }
}

TA_DEV const GenProg* prog_of(const BwdArgs& a, int axis, int l, int inv) {
  return a.progs + ((size_t)axis * kAxisSizes + l) * 2 + inv;
}

// Whether axis `axis` (at log2 size l) uses the angle set, and flipped.
TA_DEV bool uses_set(const BwdArgs& a, int axis, int l, bool* flip) {
  const int u = a.axis_use[axis];
  *flip = (u >> 8) & 1;
  return u >= 0 && (u & 0xff) == a.pid && (u >> 9) == a.kind && (1 << l) == a.n;
}

// One side of length `n` through the run of vec_f: all vectors of a pass.
TA_DEV void pass_f(float* l, int nlog, int nvec, int vstep, int stride, const GenProg* pr) {
  if ((int)threadIdx.x < nvec) {
    const int base = threadIdx.x * vstep;
    switch (nlog) {
      case 2: vec_f<4>(l, base, stride, pr); break;
      case 3: vec_f<8>(l, base, stride, pr); break;
      case 4: vec_f<16>(l, base, stride, pr); break;
      case 5: vec_f<32>(l, base, stride, pr); break;
      default: vec_f<64>(l, base, stride, pr); break;
    }
  }
}

TA_DEV void grad_side(const BwdArgs& a, int nlog, const float* lx, const float* lg, int nvec, int vstep, int stride,
                      const GenProg* pf, const GenProg* pi, bool flip, float* red, float* acc) {
  switch (nlog) {
    case 2: axis_grad<4>(a, lx, lg, 0, vstep, stride, nvec, pf, pi, flip, red, acc); break;
    case 3: axis_grad<8>(a, lx, lg, 0, vstep, stride, nvec, pf, pi, flip, red, acc); break;
    case 4: axis_grad<16>(a, lx, lg, 0, vstep, stride, nvec, pf, pi, flip, red, acc); break;
    case 5: axis_grad<32>(a, lx, lg, 0, vstep, stride, nvec, pf, pi, flip, red, acc); break;
    default: axis_grad<64>(a, lx, lg, 0, vstep, stride, nvec, pf, pi, flip, red, acc); break;
  }
}

__global__ __launch_bounds__(256) void bwd_blocks(BwdArgs a) {
  __shared__ float lx[kBwdMaxSide * kBwdPitch];    // X, row pitch W + 1
  __shared__ float lg[kBwdMaxSide * kBwdPitch];    // G_Y
  __shared__ float lw[kBwdMaxSide * kBwdPitch];    // G_W = H_v^T G_Y, then dL/dX
  __shared__ float lt[kBwdMaxSide * kBwdPitch];    // W = X H_h^T (vertical axis on the set)
  __shared__ float red[4 * kBwdMaxEntries];
  __shared__ float acc[kBwdMaxEntries];
  const int tid = threadIdx.x;
  for (int e = tid; e < a.ne; e += 256) acc[e] = 0.0f;
  for (int64_t bi = blockIdx.x; bi < a.nblocks; bi += gridDim.x) {
    const ta_block d = a.blocks[bi];
    // descriptors the transforms would skip are skipped here too
    if (d.log2w < 2 || d.log2w > 6 || d.log2h < 2 || d.log2h > 6 || d.in_off < 0 || d.out_off < 0 ||
        d.in_stride < (1 << d.log2w) || d.out_stride < (1 << d.log2w) || d.axis_h >= kAxisIds || d.axis_v >= kAxisIds)
      continue;
    const int lwg = d.log2w, lhg = d.log2h, w = 1 << lwg, h = 1 << lhg, p = w + 1;
    const GenProg* hf = prog_of(a, d.axis_h, lwg, 0);
    const GenProg* hi = prog_of(a, d.axis_h, lwg, 1);
    const GenProg* vf = prog_of(a, d.axis_v, lhg, 0);
    const GenProg* vi = prog_of(a, d.axis_v, lhg, 1);
    if (hf->nst <= 0 || vf->nst <= 0) continue;
    bool fh, fv;
    const bool uh = uses_set(a, d.axis_h, lwg, &fh), uv = uses_set(a, d.axis_v, lhg, &fv);
    for (int k = tid; k < w * h; k += 256) {
      const int r = k >> lwg, c = k & (w - 1);
      const float xv = a.x[d.in_off + (int64_t)r * d.in_stride + c];
      const float gvv = a.gy[d.out_off + (int64_t)r * d.out_stride + c];
      lx[r * p + c] = xv;
      lt[r * p + c] = xv;
      lg[r * p + c] = gvv;
      lw[r * p + c] = gvv;
    }
    __syncthreads();
    pass_f(lw, lhg, w, 1, p, vi);            // columns: G_W = H_v^T G_Y
    if (uv) pass_f(lt, lwg, h, p, 1, hf);    // rows: W = X H_h^T
    __syncthreads();
    if (uh) grad_side(a, lwg, lx, lw, h, p, 1, hf, hi, fh, red, acc);   // rows of X, rows of G_W
    if (uv) grad_side(a, lhg, lt, lg, w, 1, p, vf, vi, fv, red, acc);   // columns of W, columns of G_Y
    pass_f(lw, lwg, h, p, 1, hi);            // rows: dL/dX = G_W H_h
    __syncthreads();
    for (int k = tid; k < w * h; k += 256) {
      const int r = k >> lwg, c = k & (w - 1);
      a.gx[d.in_off + (int64_t)r * d.in_stride + c] = lw[r * p + c];
    }
    __syncthreads();
  }
  __syncthreads();
  for (int e = tid; e < a.ne; e += 256) a.part[(int64_t)blockIdx.x * a.ne + e] = acc[e];
}

// ---------------------------------------------------------------- chain rule
// Rotation (p, q) by angle t applied to rows p, q of m (n x n, row-major in
// LDS) from the left, or its transpose (tr), one thread per column.
TA_DEV void rot_rows(double* m, int n, int p, int q, double c, double s, bool tr) {
  const int j = threadIdx.x;
  if (j < n) {
    const double a = m[p * n + j], b = m[q * n + j];
    m[p * n + j] = tr ? c * a + s * b : c * a - s * b;
    m[q * n + j] = tr ? -s * a + c * b : s * a + c * b;
  }
}
// m G^T for rotation (p, q): columns p, q, one thread per row.
TA_DEV void rot_cols_t(double* m, int n, int p, int q, double c, double s) {
  const int i = threadIdx.x;
  if (i < n) {
    const double a = m[i * n + p], b = m[i * n + q];
    m[i * n + p] = c * a - s * b;
    m[i * n + q] = s * a + c * b;
  }
}

// Rotations of step l of the set (band: layer l, pairs (l mod 2 + 2j,
// l mod 2 + 2j + 1); sub-block: the single rotation l, pairs (p, q), p < q
// in lexicographic order); first angle index in *r0, count in *cnt.
TA_DEV void step_pairs(int kind, int n, int l, int* r0, int* cnt) {
  if (kind == TA_ADJ_BAND) {
    int r = 0;
    for (int k = 0; k < l; ++k) r += (n - 2 - (k & 1)) / 2 + 1;
    *r0 = r;
    *cnt = (n - 2 - (l & 1)) / 2 + 1;
  } else {
    *r0 = l;
    *cnt = 1;
  }
}
TA_DEV void pair_of(int kind, int n, int l, int k, int* p, int* q) {
  if (kind == TA_ADJ_BAND) {
    *p = (l & 1) + 2 * k;
    *q = *p + 1;
  } else {
    int idx = l, a = 0;              // lexicographic pair number l of (a, b), a < b < n
    while (idx >= n - 1 - a) {
      idx -= n - 1 - a;
      ++a;
    }
    *p = a;
    *q = a + 1 + idx;
  }
}

// Applies step l of the set (all its rotations) to the rows of m, or the
// transposed step.
TA_DEV void apply_step_rows(double* m, const double* cs, const double* sn, int kind, int n, int l, bool tr) {
  int r0, cnt;
  step_pairs(kind, n, l, &r0, &cnt);
  for (int k = 0; k < cnt; ++k) {
    int p, q;
    pair_of(kind, n, l, k, &p, &q);
    rot_rows(m, n, p, q, cs[r0 + k], sn[r0 + k], tr);
    if (kind != TA_ADJ_BAND) __syncthreads();   // a single rotation per step: rows may repeat across steps
  }
  __syncthreads();
}
TA_DEV void apply_step_cols_t(double* m, const double* cs, const double* sn, int kind, int n, int l) {
  int r0, cnt;
  step_pairs(kind, n, l, &r0, &cnt);
  for (int k = 0; k < cnt; ++k) {
    int p, q;
    pair_of(kind, n, l, k, &p, &q);
    rot_cols_t(m, n, p, q, cs[r0 + k], sn[r0 + k]);
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void bwd_chain(BwdChainArgs a) {
  __shared__ double m[kBwdMaxSide * kBwdMaxSide];
  __shared__ double q0[16 * 16];
  __shared__ double cs[kBwdMaxAngles], sn[kBwdMaxAngles];
  __shared__ double gsum[kBwdMaxEntries];
  const int tid = threadIdx.x;
  const int n = a.kind == TA_ADJ_BAND ? a.n : a.k_or_b;      // side of the matrix the angles act on
  // fixed-order sums of the partial rows
  for (int e = tid; e < a.ne; e += 256) {
    double s = 0.0;
    for (int64_t g = 0; g < a.groups; ++g) s += (double)a.part[g * a.ne + e];
    gsum[e] = s;
  }
  for (int r = tid; r < a.nang; r += 256) {
    double s, c;
    sincos(a.angles[r], &s, &c);
    cs[r] = c;
    sn[r] = s;
  }
  for (int k = tid; k < n * n; k += 256) m[k] = 0.0;
  if (a.kind != TA_ADJ_BAND)
    for (int k = tid; k < n * n; k += 256) q0[k] = a.q0 ? a.q0[k] : ((k / n) == (k % n) ? 1.0 : 0.0);
  __syncthreads();
  if (a.kind == TA_ADJ_BAND) {
    // Gbar on the band support: entry (i, t) at column s_i + t
    const int kk = a.k_or_b;
    for (int e = tid; e < a.ne; e += 256) {
      const int i = e / kk, t = e % kk, j = i - kk / 2 + ((i + kk / 2) & 1) + t;
      if (j >= 0 && j < n) m[i * n + j] = gsum[e];
    }
  } else {
    // Gbar = Q0^T dL/dQ
    for (int k = tid; k < n * n; k += 256) {
      const int i = k / n, j = k % n;
      double s = 0.0;
      for (int r = 0; r < n; ++r) s += q0[r * n + i] * gsum[r * n + j];
      m[k] = s;
    }
  }
  __syncthreads();
  const int steps = a.kind == TA_ADJ_BAND ? a.k_or_b / 2 : a.nang;
  // m_0 = (R_{L-1} ... R_1)^T Gbar: transposed steps L-1 first, 1 last
  for (int l = steps - 1; l >= 1; --l) apply_step_rows(m, cs, sn, a.kind, n, l, true);
  for (int l = 0; l < steps; ++l) {
    int r0, cnt;
    step_pairs(a.kind, n, l, &r0, &cnt);
    for (int k = tid; k < cnt; k += 256) {
      int p, q;
      pair_of(a.kind, n, l, k, &p, &q);
      const double c = cs[r0 + k], s = sn[r0 + k];
      a.gtheta[r0 + k] = (float)(-s * m[p * n + p] - c * m[p * n + q] + c * m[q * n + p] - s * m[q * n + q]);
    }
    __syncthreads();
    if (l + 1 < steps) {
      apply_step_rows(m, cs, sn, a.kind, n, l + 1, false);     // m <- R_{l+1} m
      apply_step_cols_t(m, cs, sn, a.kind, n, l);             // m <- m R_l^T
    }
  }
}

}  // namespace

const void* bwd_kernel(int which) {
  return which == 0 ? reinterpret_cast<const void*>(&bwd_blocks) : reinterpret_cast<const void*>(&bwd_chain);
}

}  // namespace ta
