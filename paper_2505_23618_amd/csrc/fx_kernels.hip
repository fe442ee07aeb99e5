// Fixed-point packed-batch kernels: forward (rows, then columns) and inverse
// (columns, then rows) of W x H int16 blocks.
//
// One 256-thread workgroup transforms a tile of NB = 256 / max(W, H) blocks.
// Each thread owns one row in the row pass and one column in the column pass
// and keeps the whole 1-D vector in registers.  The row/column exchange goes
// through LDS in two layouts, chosen so that every LDS read is a full dword
// or wider and all scattering happens on the write side (ds_write_b16 and
// ds_write_b16_d16_hi cost no VALU work):
//   PC ("pair-column"): dword s*PP + c of a block holds two elements of
//      column c, so a column thread reads its vector as packed int16 pairs;
//      PP = W + 1 keeps the pair-rows of a column in distinct banks.
//   RM ("row-major"): row pitch W + 8 halfwords so that ds_read_b128 of
//      consecutive rows hits distinct banks.
// A dword always holds the natural pair (2s, 2s+1) of its vector.
// Forward: global rows -> registers -> row pass -> PC -> column pass -> RM ->
// coalesced 16-byte stores.  Inverse: coalesced 16-byte loads -> PC ->
// column pass -> RM -> row pass -> RM -> coalesced 16-byte stores.  PC and RM alias the same
// LDS (a barrier separates the last PC read from the first RM write), which
// halves the LDS per workgroup and doubles the resident waves per CU.
#include "fx.hpp"
#include "kernels.hpp"

namespace ta {
namespace {

template <int LW, int LH>
struct Tile {
  static constexpr int W = 1 << LW, H = 1 << LH;
  static constexpr int NB = 256 / (W > H ? W : H);
  // whether every thread owns a row (a column) of the tile
  static constexpr bool ROWS_ALL = NB * H == 256, COLS_ALL = NB * W == 256;
  static constexpr int PP = W + 1;
  // XCOL (64-wide tiles of 4 blocks): in the column pass wave w takes
  // columns [16w, 16w + 16) of all 4 blocks instead of all columns of one
  // block.  The large values of a block's rows sit in its first few columns,
  // so only wave 0 then leaves the packed int16 butterfly (the wave-uniform
  // range check fails for a whole wave when any of its lanes is out of
  // range).  Its PC block pitch is padded to 16 mod 64 dwords so that the 4
  // blocks a wave reads fall in distinct banks.
  static constexpr bool XCOL = W == 64 && NB == 4;
  static constexpr int PCB = (H / 2) * PP + (XCOL ? 48 : 0);   // dwords per block, PC
  // RM row pitch: the inverse reads whole rows with ds_read_b128 and pads each
  // row by 16 bytes; the forward reads consecutive 16-byte chunks and needs no
  // row padding.  Each block is padded by 64 bytes so that the two blocks a
  // wave writes in the column pass use different banks.
  static constexpr int RPF = W;
  static constexpr int RPI = W >= 8 ? W + 8 : W;
  static constexpr int RMBF = H * RPF + (W >= 8 ? 32 : 0);
  static constexpr int RMBI = H * RPI + (W >= 8 ? 32 : 0);
  static constexpr int CH = W >= 8 ? 8 : 4;                // halfwords per global chunk
  static constexpr int CPB = W * H / CH;                   // chunks per block
  static constexpr int CPT = (NB * CPB + 255) / 256;       // chunks per thread (full tile)
  // PC and RM share one LDS buffer (sized in dwords)
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int LDS_F = cmax(NB * PCB, (NB * RMBF + 1) / 2);
  static constexpr int LDS_I = cmax(NB * PCB, (NB * RMBI + 1) / 2);
};

template <int W>
TA_DEV void load_row(const int16_t* __restrict__ src, fx::Packed<W>& x) {
  if constexpr (W >= 8) {
#pragma unroll
    for (int q = 0; q < W / 8; ++q) {
      const uint4 v = reinterpret_cast<const uint4*>(src)[q];
      x.p[4 * q + 0] = v.x;
      x.p[4 * q + 1] = v.y;
      x.p[4 * q + 2] = v.z;
      x.p[4 * q + 3] = v.w;
    }
  } else {
    const uint2 v = *reinterpret_cast<const uint2*>(src);
    x.p[0] = v.x;
    x.p[1] = v.y;
  }
}

template <int LW, int LH, class AH, class AV>
__global__ __launch_bounds__(256) void fx_fwd(PackedArgs p) {
  using T = Tile<LW, LH>;
  constexpr int W = T::W, H = T::H, NB = T::NB;
  __shared__ __align__(16) uint32_t lds[T::LDS_F];
  uint32_t* pc = lds;
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  uint16_t* rm = reinterpret_cast<uint16_t*>(lds);

  const int tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * NB;
  const int nbh = (int)min<int64_t>(NB, p.nblocks - blk0);
  const int16_t* __restrict__ in = static_cast<const int16_t*>(p.in) + blk0 * (W * H);
  int16_t* __restrict__ out = static_cast<int16_t*>(p.out) + blk0 * (W * H);
  const cparam ph_f = as_cparam(p.ph_f), ph_i = as_cparam(p.ph_i);
  const cparam pv_f = as_cparam(p.pv_f), pv_i = as_cparam(p.pv_i);

  using PV = fx::Packed<H>;

  // row pass (horizontal transform of every row) -> PC.  Rows of blocks
  // past the end of the batch repeat the last block's rows (computed, never
  // stored), so no thread needs a separate zero-fill path.
  if (T::ROWS_ALL || tid < NB * H) {
    const int b = tid / H, r = tid % H;
    fx::Packed<W> x;
    load_row<W>(in + (min(b, nbh - 1) * H + r) * W, x);
    const auto y = fx::run_pass<W, AH, false>(x, ph_f, ph_i, p.s_row, p.a);
    const int base = (b * T::PCB + (r >> 1) * T::PP) * 2 + (r & 1);
#pragma unroll
    for (int j = 0; j < W / 2; ++j) {
      const uint32_t v = y.pair(2 * j, 2 * j + 1);
      pch[base + (2 * j) * 2] = (uint16_t)v;
      pch[base + (2 * j + 1) * 2] = (uint16_t)(v >> 16);
    }
  }
  __syncthreads();

  // column pass (vertical transform of every column); PC is dead once every
  // thread has read its column, then the same LDS holds RM
  // The column pass ends the forward.  With a DCT-3 / DST-3 core (band or no
  // adjustment) its table is scaled by 2^(8 - LH), so that its shift
  // s_col = LH + m becomes 16 (the contexts fix m = 8) and each output pair
  // packs with one permute: for every int16 input the scaled sums stay below
  // 2^31 and the results inside int16, because a column of the integer DCT-2
  // has an L1 norm below H * 2^8 (7449 < 8192 at H = 32).
  // (A DCT-2 core cannot be scaled so: its rows reach an L1 norm of H * 2^8,
  // and with inputs of matching signs at +32767 / -32768 the scaled sum
  // reaches 2^31.)
  constexpr bool SCALED = (AV::CORE == C_DCT3 || AV::CORE == C_DST3) && AV::ADJ != ADJ_POST;
  constexpr int SCV = SCALED ? 8 - LH : 0;
  uint32_t o[H / 2];
  const int cb = T::XCOL ? (tid >> 4) & 3 : tid / W;                  // column thread -> block
  const int cc = T::XCOL ? ((tid >> 6) << 4) | (tid & 15) : tid % W;  // and column
  if (T::COLS_ALL || tid < NB * W) {
    PV z;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) z.p[i] = pc[cb * T::PCB + i * T::PP + cc];
    const auto y = fx::run_pass_sc<H, AV, false, false, SCV>(z, pv_f, pv_i, p.s_col, p.a);
#pragma unroll
    for (int i = 0; i < H / 2; ++i) o[i] = y.pair(2 * i, 2 * i + 1);
  }
  __syncthreads();
  if (T::COLS_ALL || tid < NB * W) {
    const int base = cb * T::RMBF + cc;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) {
      rm[base + (2 * i) * T::RPF] = (uint16_t)o[i];
      rm[base + (2 * i + 1) * T::RPF] = (uint16_t)(o[i] >> 16);
    }
  }
  __syncthreads();

  // coalesced store of the tile: chunk tid + 256 k, k < CPT
  const int nch = nbh * T::CPB;
#pragma unroll
  for (int k = 0; k < T::CPT; ++k) {
    const int c = tid + 256 * k;
    if (c < nch) {
      const int b = c / T::CPB, q = c % T::CPB;
      const uint16_t* s = rm + b * T::RMBF + q * T::CH;
      if constexpr (T::CH == 8)
        reinterpret_cast<uint4*>(out)[c] = *reinterpret_cast<const uint4*>(s);
      else
        reinterpret_cast<uint2*>(out)[c] = *reinterpret_cast<const uint2*>(s);
    }
  }
}

// The inverse holds more live values than the forward (84 VGPRs at the
// compiler's choice, five waves per SIMD); asking for six waves fits the
// 32-point kernels in 80 without spills, about 1.4 % faster in interleaved
// timing.  Larger instantiations keep what they need.
template <int LW, int LH, class AH, class AV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void fx_inv(PackedArgs p) {
  using T = Tile<LW, LH>;
  constexpr int W = T::W, H = T::H, NB = T::NB;
  __shared__ __align__(16) uint32_t lds[T::LDS_I];
  uint32_t* pc = lds;
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  uint16_t* rm = reinterpret_cast<uint16_t*>(lds);

  const int tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * NB;
  const int nbh = (int)min<int64_t>(NB, p.nblocks - blk0);
  const int16_t* __restrict__ in = static_cast<const int16_t*>(p.in) + blk0 * (W * H);
  int16_t* __restrict__ out = static_cast<int16_t*>(p.out) + blk0 * (W * H);
  const cparam ph_f = as_cparam(p.ph_f), ph_i = as_cparam(p.ph_i);
  const cparam pv_f = as_cparam(p.pv_f), pv_i = as_cparam(p.pv_i);

  using PV = fx::Packed<H>;
  using PH = fx::Packed<W>;

  // coalesced load of the tile into the pair-column layout: chunk
  // tid + 256 k, k < CPT.  All of a thread's loads are issued before any of
  // them is written to LDS, so they are in flight together (a load followed
  // by its own scatter would wait for each load in turn).
  const int nch = nbh * T::CPB;
  uint32_t w[T::CPT][T::CH / 2];
#pragma unroll
  for (int k = 0; k < T::CPT; ++k) {
    const int c = tid + 256 * k;
    if (c < nch) {
      if constexpr (T::CH == 8) {
        const uint4 v = reinterpret_cast<const uint4*>(in)[c];
        w[k][0] = v.x; w[k][1] = v.y; w[k][2] = v.z; w[k][3] = v.w;
      } else {
        const uint2 v = reinterpret_cast<const uint2*>(in)[c];
        w[k][0] = v.x; w[k][1] = v.y;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < T::CPT; ++k) {
    const int c = tid + 256 * k;
    if (c < nch) {
      const int b = c / T::CPB, q = c % T::CPB;
      const int r = q / (W / T::CH), c0 = (q % (W / T::CH)) * T::CH;
      const int base = (b * T::PCB + (r >> 1) * T::PP + c0) * 2 + (r & 1);
#pragma unroll
      for (int j = 0; j < T::CH / 2; ++j) {
        pch[base + (2 * j) * 2] = (uint16_t)w[k][j];
        pch[base + (2 * j + 1) * 2] = (uint16_t)(w[k][j] >> 16);
      }
    }
  }
  __syncthreads();

  // column pass (inverse vertical transform first); then PC is dead and the
  // same LDS holds RM
  uint32_t o[H / 2];
  if (T::COLS_ALL || tid < NB * W) {
    const int b = tid / W, c = tid % W;
    PV z;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) z.p[i] = pc[b * T::PCB + i * T::PP + c];
    const auto y = fx::run_pass<H, AV, true, (H >= 32)>(z, pv_f, pv_i, p.s_col, p.a);
#pragma unroll
    for (int i = 0; i < H / 2; ++i) o[i] = y.pair(2 * i, 2 * i + 1);
  }
  __syncthreads();
  if (T::COLS_ALL || tid < NB * W) {
    const int b = tid / W, c = tid % W;
    const int base = b * T::RMBI + c;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) {
      rm[base + (2 * i) * T::RPI] = (uint16_t)o[i];
      rm[base + (2 * i + 1) * T::RPI] = (uint16_t)(o[i] >> 16);
    }
  }
  __syncthreads();

  // row pass (inverse horizontal transform); the rows go back to RM and
  // leave the tile with coalesced 16-byte stores.  At bit depth 8 the row
  // shift m + 14 - bd is 14 (the contexts fix m = 8): a butterfly core of
  // up to 32 points then runs with its table scaled by 4 (shift 16, see
  // core_c2 / core_c3): the sums stay within 4 * W * 2^8 * 2^15 <= 2^30 and
  // the results within W * 2^8 * 2^15 / 2^14 <= 2^14 for every int16 input.
  constexpr bool ROW_SC = W <= 32 && AH::ADJ != ADJ_POST &&
                          (AH::CORE == C_DCT2 || AH::CORE == C_DST2 || AH::CORE == C_DCT3 || AH::CORE == C_DST3);
  auto row_pass = [&](auto sc) {
  constexpr int SC = decltype(sc)::value;
  if (T::ROWS_ALL || tid < NB * H) {
    const int b = tid / H, r = tid % H;
    PH x;
    const uint16_t* s = rm + b * T::RMBI + r * T::RPI;
    if constexpr (W >= 8) {
#pragma unroll
      for (int q = 0; q < W / 8; ++q) {
        const uint4 v = reinterpret_cast<const uint4*>(s)[q];
        x.p[4 * q + 0] = v.x; x.p[4 * q + 1] = v.y; x.p[4 * q + 2] = v.z; x.p[4 * q + 3] = v.w;
      }
    } else {
      const uint2 v = *reinterpret_cast<const uint2*>(s);
      x.p[0] = v.x; x.p[1] = v.y;
    }
    const auto y = fx::run_pass_sc<W, AH, true, (W >= 32), SC>(x, ph_f, ph_i, p.s_row, p.a);
    // the result goes back over this thread's own row of RM
    uint16_t* d = rm + b * T::RMBI + r * T::RPI;
    uint32_t o2[W / 2];
#pragma unroll
    for (int j = 0; j < W / 2; ++j) o2[j] = y.pair(2 * j, 2 * j + 1);
    if constexpr (W >= 8) {
#pragma unroll
      for (int q = 0; q < W / 8; ++q)
        reinterpret_cast<uint4*>(d)[q] = make_uint4(o2[4 * q], o2[4 * q + 1], o2[4 * q + 2], o2[4 * q + 3]);
    } else {
      *reinterpret_cast<uint2*>(d) = make_uint2(o2[0], o2[1]);
    }
  }
  };
  if constexpr (ROW_SC) {
    if (p.s_row == 14)
      row_pass(std::integral_constant<int, 2>{});
    else
      row_pass(std::integral_constant<int, 0>{});
  } else {
    row_pass(std::integral_constant<int, 0>{});
  }
  __syncthreads();
  // coalesced store of the tile from RM: the chunks tid + 256 k, with the
  // lanes of a wave permuted inside their 64 consecutive chunks (the same
  // 1 KiB of the output per store instruction) so that 8 consecutive lanes
  // read the same column chunk of 8 consecutive rows: with the row pitch of
  // RPI / 2 = 4 mod 8 dwords their 16-byte reads then fall in distinct banks
  // (in row order, 4 chunks of one row and 4 of the next collide once).
  constexpr int CR = W / T::CH;                       // chunks per row
  constexpr int RW = CR < 64 ? 64 / CR : 1;           // rows per 64 chunks
  const int lane = tid & 63;
  const int tperm = (tid & ~63) | (CR < 64 ? (lane % RW) * CR + lane / RW : lane);
#pragma unroll
  for (int k = 0; k < T::CPT; ++k) {
    const int c = tperm + 256 * k;
    if (c < nch) {
      const int b = c / T::CPB, q = c % T::CPB;
      const int r = q / CR, c0 = (q % CR) * T::CH;
      const uint16_t* s = rm + b * T::RMBI + r * T::RPI + c0;
      if constexpr (T::CH == 8)
        reinterpret_cast<uint4*>(out)[c] = *reinterpret_cast<const uint4*>(s);
      else
        reinterpret_cast<uint2*>(out)[c] = *reinterpret_cast<const uint2*>(s);
    }
  }
}

using fx::Axis;
// Axis shorthands: core, adjustment, K taps or B block.
using A_S3B4 = Axis<C_DST3, ADJ_BAND, 4>;
using A_C3B4 = Axis<C_DCT3, ADJ_BAND, 4>;
using A_S3B6 = Axis<C_DST3, ADJ_BAND, 6>;
using A_C2B4 = Axis<C_DCT2, ADJ_BAND, 4>;
using A_C2P16 = Axis<C_DCT2, ADJ_POST, 16>;
using A_C2P8 = Axis<C_DCT2, ADJ_POST, 8>;
using A_C2 = Axis<C_DCT2, ADJ_NONE, 0>;
using A_C3 = Axis<C_DCT3, ADJ_NONE, 0>;
using A_S2 = Axis<C_DST2, ADJ_NONE, 0>;
using A_S3 = Axis<C_DST3, ADJ_NONE, 0>;
using A_S7 = Axis<C_DST7, ADJ_NONE, 0>;
using A_C8 = Axis<C_DCT8, ADJ_NONE, 0>;

#define TA_FX(LW, LH, AH, AV)                                                                     \
  {{0, 0, LW, LH, AH::CORE, AH::ADJ, AH::KB, AV::CORE, AV::ADJ, AV::KB},                          \
   reinterpret_cast<const void*>(&fx_fwd<LW, LH, AH, AV>), Tile<LW, LH>::NB, 256, 0, false},               \
  {{1, 0, LW, LH, AH::CORE, AH::ADJ, AH::KB, AV::CORE, AV::ADJ, AV::KB},                          \
   reinterpret_cast<const void*>(&fx_inv<LW, LH, AH, AV>), Tile<LW, LH>::NB, 256, 0, false}

const KernelEntry kTable[] = {
    TA_FX(5, 5, A_S3B4, A_S3B4),     // 32x32 adjusted DST-7 (DST-3 + 4-tap band)
    TA_FX(5, 5, A_C3B4, A_C3B4),     // 32x32 adjusted DCT-8
    TA_FX(5, 5, A_S3B6, A_S3B6),     // 32x32 DST-3 + 6-tap band
    TA_FX(5, 5, A_S7, A_S7),         // 32x32 direct DST-7 (VALU)
    TA_FX(5, 5, A_C2, A_C2),         // 32x32 DCT-2
    TA_FX(5, 5, A_C2P8, A_C2P8),     // 32x32 DCT-2 + 8x8 sub-block
    TA_FX(4, 4, A_C2B4, A_C2B4),     // 16x16 DCT-2 + 4-tap band
    TA_FX(6, 6, A_C2P16, A_C2P16),   // 64x64 DCT-2 + 16x16 sub-block
    TA_FX(6, 6, A_C2P8, A_C2P8),     // 64x64 DCT-2 + 8x8 sub-block (Table 1, 64 points)
    TA_FX(6, 6, A_S3B4, A_S3B4),     // 64x64 adjusted DST-7, 4-tap band
    TA_FX(6, 6, A_S3B6, A_S3B6),     // 64x64 DST-3 + 6-tap band
    TA_FX(6, 6, A_S7, A_S7),         // 64x64 direct DST-7
    TA_FX(2, 2, A_S3B4, A_S3B4),     // 4x4 adjusted DST-7
    TA_FX(3, 3, A_S3, A_C3),         // 8x8 plain DST-3 / DCT-3
    TA_FX(4, 3, A_S2, A_C8),         // 16x8 DST-2 / direct DCT-8 (rectangular)
    TA_FX(3, 5, A_C2, A_S3B4),       // 8x32 DCT-2 / adjusted DST-7 (rectangular)
};

}  // namespace

const KernelEntry* fx_kernels(int* count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

}  // namespace ta
