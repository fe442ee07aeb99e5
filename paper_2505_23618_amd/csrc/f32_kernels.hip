// FP32 packed-batch kernels: forward (rows, then columns) and inverse
// (columns, then rows) of W x H fp32 blocks.  One 256-thread workgroup per
// tile of NB = 256 / max(W, H) blocks; one thread per row in the row pass and
// per column in the column pass.  LDS holds the tile column-major (pitch
// H + 1, for the column threads) or row-major (pitch W + 1, for the row
// threads); odd pitches keep the per-element accesses of a wave in distinct
// banks.  Forward: global rows -> row pass -> LDS (col-major) -> column pass
// -> LDS (row-major) -> coalesced stores.  Inverse: coalesced loads -> LDS
// (col-major) -> column pass -> LDS (row-major) -> row pass -> global rows.
#include "fp.hpp"
#include "kernels.hpp"

namespace ta {
namespace {

template <int LW, int LH>
struct FTile {
  static constexpr int W = 1 << LW, H = 1 << LH;
  static constexpr int NB = 256 / (W > H ? W : H);
  static constexpr int CM = W * (H + 1);   // floats per block, column-major
  static constexpr int RM = H * (W + 1);   // floats per block, row-major
  static constexpr int BS = CM > RM ? CM : RM;
  static constexpr int Q4 = W * H / 4;     // float4 chunks per block
  static constexpr int CPT = (NB * Q4 + 255) / 256;   // chunks per thread (full tile)
};

template <int W>
TA_DEV void load_rowf(const float* __restrict__ src, fp::Vec<W>& x) {
  if constexpr (W >= 4) {
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
      const float4 v = reinterpret_cast<const float4*>(src)[q];
      x.v[4 * q] = v.x; x.v[4 * q + 1] = v.y; x.v[4 * q + 2] = v.z; x.v[4 * q + 3] = v.w;
    }
  }
}

// Coalesced float4 stores of a tile held row-major (pitch W + 1) in LDS.
template <class T>
TA_DEV void store_tile(const float* lds, float* __restrict__ out, int nbh, int tid) {
  constexpr int W = T::W;
  const int nch = nbh * T::Q4;
#pragma unroll
  for (int k = 0; k < T::CPT; ++k) {
    const int c = tid + 256 * k;
    if (c < nch) {
      const int b = c / T::Q4, q = c % T::Q4;
      const float* s = lds + b * T::BS + (q / (W / 4)) * (W + 1) + (q % (W / 4)) * 4;
      reinterpret_cast<float4*>(out)[c] = make_float4(s[0], s[1], s[2], s[3]);
    }
  }
}

template <int LW, int LH, class AH, class AV>
__global__ __launch_bounds__(256) void f32_fwd(PackedArgs p) {
  using T = FTile<LW, LH>;
  constexpr int W = T::W, H = T::H, NB = T::NB;
  __shared__ float lds[NB * T::BS];
  const int tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * NB;
  const int nbh = (int)min<int64_t>(NB, p.nblocks - blk0);
  const float* __restrict__ in = static_cast<const float*>(p.in) + blk0 * (W * H);
  float* __restrict__ out = static_cast<float*>(p.out) + blk0 * (W * H);
  const float* ph_f = static_cast<const float*>(p.ph_f);
  const float* ph_i = static_cast<const float*>(p.ph_i);
  const float* pv_f = static_cast<const float*>(p.pv_f);
  const float* pv_i = static_cast<const float*>(p.pv_i);

  // row pass: rows of blocks past the batch end repeat the last block (never stored)
  if (tid < NB * H) {
    const int b = tid / H, r = tid % H;
    fp::Vec<W> x;
    load_rowf<W>(in + (min(b, nbh - 1) * H + r) * W, x);
    const fp::Vec<W> y = fp::run_pass<W, AH, false>(x, ph_f, ph_i);
#pragma unroll
    for (int c = 0; c < W; ++c) lds[b * T::BS + c * (H + 1) + r] = y.v[c];
  }
  __syncthreads();
  fp::Vec<H> z;
  if (tid < NB * W) {
    const int b = tid / W, c = tid % W;
#pragma unroll
    for (int r = 0; r < H; ++r) z.v[r] = lds[b * T::BS + c * (H + 1) + r];
    z = fp::run_pass<H, AV, false>(z, pv_f, pv_i);
  }
  __syncthreads();
  if (tid < NB * W) {
    const int b = tid / W, c = tid % W;
#pragma unroll
    for (int r = 0; r < H; ++r) lds[b * T::BS + r * (W + 1) + c] = z.v[r];
  }
  __syncthreads();
  store_tile<T>(lds, out, nbh, tid);
}

template <int LW, int LH, class AH, class AV>
__global__ __launch_bounds__(256) void f32_inv(PackedArgs p) {
  using T = FTile<LW, LH>;
  constexpr int W = T::W, H = T::H, NB = T::NB;
  __shared__ float lds[NB * T::BS];
  const int tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * NB;
  const int nbh = (int)min<int64_t>(NB, p.nblocks - blk0);
  const float* __restrict__ in = static_cast<const float*>(p.in) + blk0 * (W * H);
  float* __restrict__ out = static_cast<float*>(p.out) + blk0 * (W * H);
  const float* ph_f = static_cast<const float*>(p.ph_f);
  const float* ph_i = static_cast<const float*>(p.ph_i);
  const float* pv_f = static_cast<const float*>(p.pv_f);
  const float* pv_i = static_cast<const float*>(p.pv_i);

  // coalesced float4 loads into the column-major layout, in groups of G
  // chunks per thread whose loads are all issued before any is written to
  // LDS (a load followed by its own scatter would wait for each in turn)
  const int nch = nbh * T::Q4;
  constexpr int G = T::CPT < 8 ? T::CPT : 8;
#pragma unroll
  for (int k0 = 0; k0 < T::CPT; k0 += G) {
    float4 v[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int c = tid + 256 * (k0 + g);
      if (c < nch) v[g] = reinterpret_cast<const float4*>(in)[c];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int c = tid + 256 * (k0 + g);
      if (c < nch) {
        const int b = c / T::Q4, q = c % T::Q4;
        const int r = q / (W / 4), c0 = (q % (W / 4)) * 4;
        float* d = lds + b * T::BS + c0 * (H + 1) + r;
        d[0] = v[g].x; d[H + 1] = v[g].y; d[2 * (H + 1)] = v[g].z; d[3 * (H + 1)] = v[g].w;
      }
    }
  }
  __syncthreads();
  fp::Vec<H> z;
  if (tid < NB * W) {
    const int b = tid / W, c = tid % W;
#pragma unroll
    for (int r = 0; r < H; ++r) z.v[r] = lds[b * T::BS + c * (H + 1) + r];
    z = fp::run_pass<H, AV, true>(z, pv_f, pv_i);
  }
  __syncthreads();
  if (tid < NB * W) {
    const int b = tid / W, c = tid % W;
#pragma unroll
    for (int r = 0; r < H; ++r) lds[b * T::BS + r * (W + 1) + c] = z.v[r];
  }
  __syncthreads();
  // row pass; each thread writes its result back over its own row, then the
  // tile leaves with coalesced stores
  if (tid < NB * H) {
    const int b = tid / H, r = tid % H;
    fp::Vec<W> x;
    float* row = lds + b * T::BS + r * (W + 1);
#pragma unroll
    for (int c = 0; c < W; ++c) x.v[c] = row[c];
    const fp::Vec<W> y = fp::run_pass<W, AH, true>(x, ph_f, ph_i);
#pragma unroll
    for (int c = 0; c < W; ++c) row[c] = y.v[c];
  }
  __syncthreads();
  store_tile<T>(lds, out, nbh, tid);
}

template <int CORE_, int ADJ_, int KB_>
struct FAx {
  static constexpr int CORE = CORE_, ADJ = ADJ_, KB = KB_;
};
using F_S3B4 = FAx<C_DST3, ADJ_BAND, 4>;
using F_C3B4 = FAx<C_DCT3, ADJ_BAND, 4>;
using F_C2B4 = FAx<C_DCT2, ADJ_BAND, 4>;
using F_C2P16 = FAx<C_DCT2, ADJ_POST, 16>;
using F_C2P8 = FAx<C_DCT2, ADJ_POST, 8>;
using F_C2 = FAx<C_DCT2, ADJ_NONE, 0>;
using F_S7 = FAx<C_DST7, ADJ_NONE, 0>;
using F_C8 = FAx<C_DCT8, ADJ_NONE, 0>;
using F_S2 = FAx<C_DST2, ADJ_NONE, 0>;

#define TA_F32(LW, LH, AH, AV)                                                                    \
  {{0, 1, LW, LH, AH::CORE, AH::ADJ, AH::KB, AV::CORE, AV::ADJ, AV::KB},                          \
   reinterpret_cast<const void*>(&f32_fwd<LW, LH, AH, AV>), FTile<LW, LH>::NB, 256, 0, false},   \
  {{1, 1, LW, LH, AH::CORE, AH::ADJ, AH::KB, AV::CORE, AV::ADJ, AV::KB},                          \
   reinterpret_cast<const void*>(&f32_inv<LW, LH, AH, AV>), FTile<LW, LH>::NB, 256, 0, false}

const KernelEntry kTable[] = {
    TA_F32(6, 6, F_C2P16, F_C2P16),   // 64x64 DCT-2 + 16x16 sub-block (DCT-8 rows, DST-7 columns)
    TA_F32(6, 6, F_S7, F_S7),         // 64x64 direct DST-7
    TA_F32(5, 5, F_S3B4, F_S3B4),     // 32x32 adjusted DST-7
    TA_F32(5, 5, F_C3B4, F_C3B4),     // 32x32 adjusted DCT-8
    TA_F32(5, 5, F_S7, F_S7),         // 32x32 direct DST-7
    TA_F32(5, 5, F_C2P8, F_C2P8),     // 32x32 DCT-2 + 8x8 sub-block
    TA_F32(4, 4, F_C2B4, F_C2B4),     // 16x16 DCT-2 + 4-tap band
    TA_F32(3, 4, F_S2, F_C8),         // 8x16 DST-2 / direct DCT-8
};

}  // namespace

const KernelEntry* f32_kernels(int* count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

}  // namespace ta
