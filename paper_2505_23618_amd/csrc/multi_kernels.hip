// Encoder evaluation of one residual block under the five separable
// transforms a VVC-style encoder compares (section "Simultaneous transform
// adjustments for the DCT-8 and DST-7"): DCT-2 x DCT-2 and every
// (vertical, horizontal) pair of adjusted DST-7 / DCT-8, where both adjusted
// transforms are the DCT-2 followed by a B x B sub-block adjustment, Q for
// DST-7 and S Q S for DCT-8 (eq. 5).
//
// The DCT-2 core is shared by all five, and in fixed point exactly so: the
// flipped design's core S T R equals T entry by entry.  Per block:
//   rows:    one DCT-2 per row; the first B outputs are also adjusted both
//            ways at the cost of one adjustment (fx::post_both).  The tile in
//            LDS gets W + 2B columns per block: the N DCT-2 columns, then the
//            B DST-7-adjusted and the B DCT-8-adjusted leading columns.
//   columns: one DCT-2 per stored column (N + 2B per block instead of 5N),
//            then both vertical adjustments of its first B outputs.
//   output:  five rounds; in round k every column thread writes the part it
//            owns of output k into a row-major LDS tile, which leaves with
//            coalesced 16-byte stores.
// Which column feeds which output (c = column index within the block):
//   c <  B            DCT-2 rows' leading columns   -> output 0 only
//   B <= c < N        shared columns               -> all five outputs
//   N <= c < N+B      DST-7 rows' leading columns   -> outputs 1 and 3
//   N+B <= c          DCT-8 rows' leading columns   -> outputs 2 and 4
// and outputs 1..4 take the DST-7 (1, 2) or DCT-8 (3, 4) vertical adjustment.
#include "fx.hpp"
#include "kernels.hpp"

namespace ta {
namespace {

template <int LN, int B>
struct MTile {
  static constexpr int N = 1 << LN;
  static constexpr int NB = 256 / N;            // blocks per tile
  static constexpr int WX = N + 2 * B;          // stored columns per block
  static constexpr int THREADS = NB * WX;       // one thread per stored column
  static constexpr int PP = WX + 1;             // pair-column pitch (dwords)
  static constexpr int PCB = (N / 2) * PP;      // dwords per block, PC
  static constexpr int RMB = N * N + 32;        // halfwords per block, RM (padded)
  static constexpr int CPB = N * N / 8;         // 16-byte chunks per block
  static constexpr int CPT = (NB * CPB + THREADS - 1) / THREADS;
  static constexpr int LDS = (NB * PCB) > (NB * RMB + 1) / 2 ? (NB * PCB) : (NB * RMB + 1) / 2;
};

template <int LN, int B>
__global__ __launch_bounds__(384) void multi_fwd(MultiArgs a) {
  using T = MTile<LN, B>;
  constexpr int N = T::N, NB = T::NB, WX = T::WX;
  static_assert(T::THREADS == 384, "one thread per stored column");
  __shared__ __align__(16) uint32_t lds[T::LDS];
  uint32_t* pc = lds;
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  uint16_t* rm = reinterpret_cast<uint16_t*>(lds);

  const int tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * NB;
  const int nbh = (int)min<int64_t>(NB, a.nblocks - blk0);
  const int16_t* __restrict__ in = a.in + blk0 * (N * N);
  const cparam q = as_cparam(a.q_eo);

  // row pass: DCT-2 of every row, both adjustments of its leading outputs
  if (tid < NB * N) {
    const int b = tid / N, r = tid % N;
    fx::Packed<N> x;
    const int16_t* src = in + (min(b, nbh - 1) * N + r) * N;
#pragma unroll
    for (int k = 0; k < N / 8; ++k) {
      const uint4 v = reinterpret_cast<const uint4*>(src)[k];
      x.p[4 * k] = v.x; x.p[4 * k + 1] = v.y; x.p[4 * k + 2] = v.z; x.p[4 * k + 3] = v.w;
    }
    const fx::Acc<N> y = fx::core<N, C_DCT2, false>(x, a.s_row);
    int z7[B], z8[B];
    fx::post_both<B>(y, q, a.a, z7, z8);
    const int base = (b * T::PCB + (r >> 1) * T::PP) * 2 + (r & 1);
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const uint32_t v = y.pair(2 * j, 2 * j + 1);
      pch[base + (2 * j) * 2] = (uint16_t)v;
      pch[base + (2 * j + 1) * 2] = (uint16_t)(v >> 16);
    }
#pragma unroll
    for (int j = 0; j < B / 2; ++j) {
      const uint32_t v7 = satpk(z7[2 * j] >> a.a, z7[2 * j + 1] >> a.a);
      const uint32_t v8 = satpk(z8[2 * j] >> a.a, z8[2 * j + 1] >> a.a);
      pch[base + (N + 2 * j) * 2] = (uint16_t)v7;
      pch[base + (N + 2 * j + 1) * 2] = (uint16_t)(v7 >> 16);
      pch[base + (N + B + 2 * j) * 2] = (uint16_t)v8;
      pch[base + (N + B + 2 * j + 1) * 2] = (uint16_t)(v8 >> 16);
    }
  }
  __syncthreads();

  // column pass: DCT-2 of every stored column, both vertical adjustments
  const int b = tid / WX, c = tid % WX;
  fx::Packed<N> z;
#pragma unroll
  for (int i = 0; i < N / 2; ++i) z.p[i] = pc[b * T::PCB + i * T::PP + c];
  const fx::Acc<N> y = fx::core<N, C_DCT2, false>(z, a.s_col);
  int v7[B], v8[B];
  fx::post_both<B>(y, q, a.a, v7, v8);
  uint32_t yc[N / 2], w7[B / 2], w8[B / 2];
#pragma unroll
  for (int i = 0; i < N / 2; ++i) yc[i] = y.pair(2 * i, 2 * i + 1);
#pragma unroll
  for (int i = 0; i < B / 2; ++i) {
    w7[i] = satpk(v7[2 * i] >> a.a, v7[2 * i + 1] >> a.a);
    w8[i] = satpk(v8[2 * i] >> a.a, v8[2 * i + 1] >> a.a);
  }
  // destination column of this thread in the outputs it feeds
  const int cls = c < B ? 0 : c < N ? 1 : c < N + B ? 2 : 3;
  const int oc = cls == 2 ? c - N : cls == 3 ? c - N - B : c;
  __syncthreads();   // PC is dead: the same LDS holds RM from here on

#pragma unroll
  for (int k = 0; k < 5; ++k) {
    // does this column feed output k, and with which leading rows?
    const bool feeds = k == 0 ? cls <= 1
                              : cls == 1 || (cls == 2 && (k == 1 || k == 3)) || (cls == 3 && (k == 2 || k == 4));
    if (feeds) {
      const int base = b * T::RMB + oc;
#pragma unroll
      for (int i = 0; i < N / 2; ++i) {
        uint32_t v = yc[i];
        if (i < B / 2 && k > 0) v = k <= 2 ? w7[i] : w8[i];
        rm[base + (2 * i) * N] = (uint16_t)v;
        rm[base + (2 * i + 1) * N] = (uint16_t)(v >> 16);
      }
    }
    __syncthreads();
    int16_t* __restrict__ out = a.out + (int64_t)k * a.nblocks * (N * N) + blk0 * (N * N);
    const int nch = nbh * T::CPB;
#pragma unroll
    for (int j = 0; j < T::CPT; ++j) {
      const int ch = tid + T::THREADS * j;
      if (ch < nch) {
        const int bb = ch / T::CPB, qq = ch % T::CPB;
        reinterpret_cast<uint4*>(out)[ch] = *reinterpret_cast<const uint4*>(rm + bb * T::RMB + qq * 8);
      }
    }
    __syncthreads();
  }
}

}  // namespace

// (log2 n, b) in {(5, 8), (6, 16)}; threads per workgroup in *threads,
// blocks per workgroup in *blocks.
const void* multi_kernel(int log2n, int b, int* threads, int* blocks) {
  if (log2n == 5 && b == 8) {
    *threads = MTile<5, 8>::THREADS;
    *blocks = MTile<5, 8>::NB;
    return reinterpret_cast<const void*>(&multi_fwd<5, 8>);
  }
  if (log2n == 6 && b == 16) {
    *threads = MTile<6, 16>::THREADS;
    *blocks = MTile<6, 16>::NB;
    return reinterpret_cast<const void*>(&multi_fwd<6, 16>);
  }
  return nullptr;
}

}  // namespace ta
