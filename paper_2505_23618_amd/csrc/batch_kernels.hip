// Batched uneven blocks: one persistent launch over a planned list of tiles.
//
// The host planner groups blocks by (frame region, W, H, horizontal kind,
// vertical kind) and cuts the groups into tiles of BatchGeo::nb_for blocks.
// Each workgroup walks its XCD's tile list with a grid stride.  Within a
// tile the forward runs the phases of the packed kernels (rows -> pair-row
// LDS -> columns -> row-major LDS -> coalesced stores) and the inverse the
// reverse, but block addresses come from the block descriptors (offsets and
// row strides into frame buffers) and the block size and kinds are
// wave-uniform runtime values: the row phase dispatches on (W, row kind),
// the column phase on (H, column kind), 15 row and 15 column bodies per
// direction.
//
// LDS layout (BatchGeo): the tile's blocks sit side by side, block b at
// column b * W; pair-row i (rows 2i, 2i+1 packed in dwords) has pitch
// pc_pitch(H) and row r (halfwords) has pitch rm_pitch(H).  A column thread
// with index t = b * W + c therefore reads and writes at t plus compile-time
// offsets, and a row thread only adds its block's column offset.
//
// Kinds: 0 = DCT-2, 1 = DST-3 + 4-tap band (adjusted DST-7),
//        2 = DCT-3 + 4-tap band with flipped taps (adjusted DCT-8, eq. 3).
//
// The same tile walk runs on fp32 data with the orthonormal fp32 stages
// (batch_f32, BatchGeoF32 layout), and both data types also run unplanned,
// straight from a device array of descriptors (batch_desc).
#include <type_traits>

#include "fp.hpp"
#include "fx.hpp"
#include "kernels.hpp"
#include "window_sort.hpp"

namespace ta {
namespace {

using fx::Axis;
using KC2 = Axis<C_DCT2, ADJ_NONE, 0>;
using KS3 = Axis<C_DST3, ADJ_BAND, 4>;
using KC3 = Axis<C_DCT3, ADJ_BAND, 4>;

constexpr int kBatchLds = BatchGeo::max_lds_dwords();

// Offsets and strides of the blocks of the current tile, in LDS: the chunk
// loops look them up there instead of loading a descriptor per chunk.
struct BDesc {
  int64_t in_off, out_off;
  int32_t in_stride, out_stride;
};
constexpr int kMaxTileBlocks = 64;
static_assert(kBatchLds * 4 <= 20480, "tile LDS above 20 KiB");

// The tile loads issue all of a thread's chunks at once: at most 4 chunks
// (8 halfwords, 4 for 4-wide blocks) per thread for int16 tiles and 8 float4
// per thread for fp32 tiles.
constexpr bool tile_chunks_fit() {
  for (int lw = 2; lw <= 6; ++lw)
    for (int lh = 2; lh <= 6; ++lh) {
      const int elems = BatchGeo::nb_for(lw, lh) << (lw + lh);
      if (elems / (lw >= 3 ? 8 : 4) > 4 * 256) return false;
      if ((BatchGeoF32::nb_for(lw, lh) << (lw + lh)) / 4 > 8 * 256) return false;
    }
  return true;
}
static_assert(tile_chunks_fit(), "a tile has more chunks than the loads issue");

// Workgroup barrier that orders LDS only.  The planned kernels keep global
// loads into LDS (the LDS DMA path) in flight across the barriers of the
// tile before; the workgroup-scope fence of __syncthreads would wait for
// them (they write LDS), this waits for the wave's own LDS accesses alone.
TA_DEV void tile_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int W>
TA_DEV void load_strided_row(const int16_t* __restrict__ src, fx::Packed<W>& x) {
  if constexpr (W >= 8) {
#pragma unroll
    for (int q = 0; q < W / 8; ++q) {
      const uint4 v = reinterpret_cast<const uint4*>(src)[q];
      x.p[4 * q] = v.x; x.p[4 * q + 1] = v.y; x.p[4 * q + 2] = v.z; x.p[4 * q + 3] = v.w;
    }
  } else {
    const uint2 v = *reinterpret_cast<const uint2*>(src);
    x.p[0] = v.x; x.p[1] = v.y;
  }
}

// ---------------------------------------------------------------- forward
// row phase of one tile for kind KH at width W (H = 2^lh rows per block)
template <int W, class KH>
TA_DEV void fwd_rows(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, uint16_t* pch, BDesc* desc,
                      int s_row) {
  const int tid = threadIdx.x;
  if (tid >= (t.count << t.lh)) return;
  const int b = tid >> t.lh, r = tid & ((1 << t.lh) - 1);
  const ta_block d = blocks[t.first + b];
  if (r == 0) desc[b] = BDesc{d.in_off, d.out_off, d.in_stride, d.out_stride};
  fx::Packed<W> x;
  load_strided_row<W>(a.in + d.in_off + (int64_t)r * d.in_stride, x);
  const auto y = fx::run_pass<W, KH, false>(x, as_cparam(t.ph_f), as_cparam(t.ph_i), s_row, a.a);
  const int base = ((r >> 1) * BatchGeo::pc_pitch(t.lh) + b * W) * 2 + (r & 1);
#pragma unroll
  for (int j = 0; j < W / 2; ++j) {
    const uint32_t v = y.pair(2 * j, 2 * j + 1);
    pch[base + (2 * j) * 2] = (uint16_t)v;
    pch[base + (2 * j + 1) * 2] = (uint16_t)(v >> 16);
  }
}

// column phase: read the pair-rows, transform, barrier (they are dead), write
// the row-major layout
template <int H, class KV, int LH>
TA_DEV void fwd_cols(const BatchArgs& a, const BatchTile& t, uint32_t* lds, int s_col) {
  constexpr int P = BatchGeo::pc_pitch(LH), Q = BatchGeo::rm_pitch(LH);
  const int tid = threadIdx.x;
  const bool act = tid < (t.count << t.lw);
  uint32_t o[H / 2];
  if (act) {
    fx::Packed<H> z;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) z.p[i] = lds[i * P + tid];
    const auto y = fx::run_pass<H, KV, false>(z, as_cparam(t.pv_f), as_cparam(t.pv_i), s_col, a.a);
#pragma unroll
    for (int i = 0; i < H / 2; ++i) o[i] = y.pair(2 * i, 2 * i + 1);
  }
  tile_sync();
  if (act) {
    uint16_t* rm = reinterpret_cast<uint16_t*>(lds);
#pragma unroll
    for (int i = 0; i < H / 2; ++i) {
      rm[(2 * i) * Q + tid] = (uint16_t)o[i];
      rm[(2 * i + 1) * Q + tid] = (uint16_t)(o[i] >> 16);
    }
  }
}

template <class KH>
TA_DEV void fwd_rows_w(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, uint16_t* pch, BDesc* desc,
                        int s) {
  switch (t.lw) {
    case 2: fwd_rows<4, KH>(a, t, blocks, pch, desc, s); break;
    case 3: fwd_rows<8, KH>(a, t, blocks, pch, desc, s); break;
    case 4: fwd_rows<16, KH>(a, t, blocks, pch, desc, s); break;
    case 5: fwd_rows<32, KH>(a, t, blocks, pch, desc, s); break;
    default: fwd_rows<64, KH>(a, t, blocks, pch, desc, s); break;
  }
}

template <class KV>
TA_DEV void fwd_cols_h(const BatchArgs& a, const BatchTile& t, uint32_t* lds, int s) {
  switch (t.lh) {
    case 2: fwd_cols<4, KV, 2>(a, t, lds, s); break;
    case 3: fwd_cols<8, KV, 3>(a, t, lds, s); break;
    case 4: fwd_cols<16, KV, 4>(a, t, lds, s); break;
    case 5: fwd_cols<32, KV, 5>(a, t, lds, s); break;
    default: fwd_cols<64, KV, 6>(a, t, lds, s); break;
  }
}

// Chunks of a tile in memory order: chunk ch of 2^lch halfwords belongs to
// block b, row r, and starts at column c0.
struct Chunk {
  int b, r, c0;
  TA_DEV Chunk(int ch, int lw, int lh, int lch) {
    const int lq = lw - lch;                      // log2 chunks per row
    b = ch >> (lq + lh);
    r = (ch >> lq) & ((1 << lh) - 1);
    c0 = (ch & ((1 << lq) - 1)) << lch;
  }
};

// One tile of the forward: rows -> pair-row LDS -> columns -> row-major LDS
// -> coalesced stores.  Ends with a barrier (LDS free for the next tile).
TA_DEV void fwd_tile(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, uint32_t* lds, BDesc* desc) {
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  const int s_row = t.lw + a.bd + a.m - 15, s_col = t.lh + a.m;
  switch (t.kind_h) {
    case 0: fwd_rows_w<KC2>(a, t, blocks, pch, desc, s_row); break;
    case 1: fwd_rows_w<KS3>(a, t, blocks, pch, desc, s_row); break;
    default: fwd_rows_w<KC3>(a, t, blocks, pch, desc, s_row); break;
  }
  __syncthreads();
  switch (t.kind_v) {
    case 0: fwd_cols_h<KC2>(a, t, lds, s_col); break;
    case 1: fwd_cols_h<KS3>(a, t, lds, s_col); break;
    default: fwd_cols_h<KC3>(a, t, lds, s_col); break;
  }
  __syncthreads();
  // coalesced store of the tile (row-major layout, chunks of 2^lch halfwords)
  const int lch = t.lw >= 3 ? 3 : 2;
  const int q = BatchGeo::rm_pitch(t.lh);
  const int nch = t.count << (t.lw + t.lh - lch);
  for (int ch = threadIdx.x; ch < nch; ch += 256) {
    const Chunk k(ch, t.lw, t.lh, lch);
    const BDesc d = desc[k.b];
    int16_t* dst = a.out + d.out_off + (int64_t)k.r * d.out_stride + k.c0;
    const uint16_t* src = pch + k.r * q + (k.b << t.lw) + k.c0;
    if (lch == 3)
      *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(src);
    else
      *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(src);
  }
  __syncthreads();
}

// ---------------------------------------------------------------- inverse
template <int H, class KV, int LH>
TA_DEV void inv_cols(const BatchArgs& a, const BatchTile& t, uint32_t* lds, int s_col) {
  constexpr int P = BatchGeo::pc_pitch(LH), Q = BatchGeo::rm_pitch(LH);
  const int tid = threadIdx.x;
  const bool act = tid < (t.count << t.lw);
  uint32_t o[H / 2];
  if (act) {
    fx::Packed<H> z;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) z.p[i] = lds[i * P + tid];
    const auto y = fx::run_pass<H, KV, true>(z, as_cparam(t.pv_f), as_cparam(t.pv_i), s_col, a.a);
#pragma unroll
    for (int i = 0; i < H / 2; ++i) o[i] = y.pair(2 * i, 2 * i + 1);
  }
  tile_sync();
  if (act) {
    uint16_t* rm = reinterpret_cast<uint16_t*>(lds);
#pragma unroll
    for (int i = 0; i < H / 2; ++i) {
      rm[(2 * i) * Q + tid] = (uint16_t)o[i];
      rm[(2 * i + 1) * Q + tid] = (uint16_t)(o[i] >> 16);
    }
  }
}

// row phase of the inverse: each thread transforms its row and writes the
// result back over the same row of the row-major layout
template <int W, class KH>
TA_DEV void inv_rows(const BatchArgs& a, const BatchTile& t, uint16_t* rm, int s_row) {
  const int tid = threadIdx.x;
  if (tid >= (t.count << t.lh)) return;
  const int b = tid >> t.lh, r = tid & ((1 << t.lh) - 1);
  uint16_t* s = rm + r * BatchGeo::rm_pitch(t.lh) + b * W;
  fx::Packed<W> x;
  if constexpr (W >= 8) {
#pragma unroll
    for (int q = 0; q < W / 8; ++q) {
      const uint4 v = reinterpret_cast<const uint4*>(s)[q];
      x.p[4 * q] = v.x; x.p[4 * q + 1] = v.y; x.p[4 * q + 2] = v.z; x.p[4 * q + 3] = v.w;
    }
  } else {
    const uint2 v = *reinterpret_cast<const uint2*>(s);
    x.p[0] = v.x; x.p[1] = v.y;
  }
  const auto y = fx::run_pass<W, KH, true>(x, as_cparam(t.ph_f), as_cparam(t.ph_i), s_row, a.a);
  uint32_t o[W / 2];
#pragma unroll
  for (int j = 0; j < W / 2; ++j) o[j] = y.pair(2 * j, 2 * j + 1);
  if constexpr (W >= 8) {
#pragma unroll
    for (int q = 0; q < W / 8; ++q)
      reinterpret_cast<uint4*>(s)[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
  } else {
    *reinterpret_cast<uint2*>(s) = make_uint2(o[0], o[1]);
  }
}

template <class KV>
TA_DEV void inv_cols_h(const BatchArgs& a, const BatchTile& t, uint32_t* lds, int s) {
  switch (t.lh) {
    case 2: inv_cols<4, KV, 2>(a, t, lds, s); break;
    case 3: inv_cols<8, KV, 3>(a, t, lds, s); break;
    case 4: inv_cols<16, KV, 4>(a, t, lds, s); break;
    case 5: inv_cols<32, KV, 5>(a, t, lds, s); break;
    default: inv_cols<64, KV, 6>(a, t, lds, s); break;
  }
}

template <class KH>
TA_DEV void inv_rows_w(const BatchArgs& a, const BatchTile& t, uint16_t* rm, int s) {
  switch (t.lw) {
    case 2: inv_rows<4, KH>(a, t, rm, s); break;
    case 3: inv_rows<8, KH>(a, t, rm, s); break;
    case 4: inv_rows<16, KH>(a, t, rm, s); break;
    case 5: inv_rows<32, KH>(a, t, rm, s); break;
    default: inv_rows<64, KH>(a, t, rm, s); break;
  }
}

// One tile of the inverse: coalesced loads -> pair-row LDS -> columns ->
// row-major LDS -> rows in place -> coalesced stores.  Ends with a barrier.
TA_DEV void inv_tile(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, uint32_t* lds, BDesc* desc) {
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  const int s_col = a.m + 1, s_row = a.m + 14 - a.bd;
  const int lch = t.lw >= 3 ? 3 : 2;
  const int nch = t.count << (t.lw + t.lh - lch);
  if ((int)threadIdx.x < t.count) {
    const ta_block d = blocks[t.first + threadIdx.x];
    desc[threadIdx.x] = BDesc{d.in_off, d.out_off, d.in_stride, d.out_stride};
  }
  __syncthreads();
  // coalesced load of the tile into the pair-row layout: a tile holds at
  // most 1024 chunks, so each thread's (at most 4) loads are issued together
  // before any is written to LDS (a load followed by its own scatter would
  // wait for each in turn)
  {
    const int p = BatchGeo::pc_pitch(t.lh);
    uint4 v[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int ch = threadIdx.x + 256 * g;
      if (ch < nch) {
        const Chunk k(ch, t.lw, t.lh, lch);
        const BDesc d = desc[k.b];
        const int16_t* src = a.in + d.in_off + (int64_t)k.r * d.in_stride + k.c0;
        if (lch == 3) {
          v[g] = *reinterpret_cast<const uint4*>(src);
        } else {
          const uint2 h = *reinterpret_cast<const uint2*>(src);
          v[g] = make_uint4(h.x, h.y, 0, 0);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int ch = threadIdx.x + 256 * g;
      if (ch < nch) {
        const Chunk k(ch, t.lw, t.lh, lch);
        const uint32_t w[4] = {v[g].x, v[g].y, v[g].z, v[g].w};
        const int base = ((k.r >> 1) * p + (k.b << t.lw) + k.c0) * 2 + (k.r & 1);
        for (int j = 0; j < (1 << lch) / 2; ++j) {
          pch[base + (2 * j) * 2] = (uint16_t)w[j];
          pch[base + (2 * j + 1) * 2] = (uint16_t)(w[j] >> 16);
        }
      }
    }
  }
  __syncthreads();
  switch (t.kind_v) {
    case 0: inv_cols_h<KC2>(a, t, lds, s_col); break;
    case 1: inv_cols_h<KS3>(a, t, lds, s_col); break;
    default: inv_cols_h<KC3>(a, t, lds, s_col); break;
  }
  __syncthreads();
  switch (t.kind_h) {
    case 0: inv_rows_w<KC2>(a, t, pch, s_row); break;
    case 1: inv_rows_w<KS3>(a, t, pch, s_row); break;
    default: inv_rows_w<KC3>(a, t, pch, s_row); break;
  }
  __syncthreads();
  // coalesced store of the tile (row-major layout)
  {
    const int q = BatchGeo::rm_pitch(t.lh);
    for (int ch = threadIdx.x; ch < nch; ch += 256) {
      const Chunk k(ch, t.lw, t.lh, lch);
      const BDesc d = desc[k.b];
      int16_t* dst = a.out + d.out_off + (int64_t)k.r * d.out_stride + k.c0;
      const uint16_t* src = pch + k.r * q + (k.b << t.lw) + k.c0;
      if (lch == 3)
        *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(src);
      else
        *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(src);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- planned, pipelined
// The planned int16 kernels run tiles of up to 8192 coefficients
// (BatchGeo::nb_planned blocks) and overlap each tile's global loads with
// the work on the tile before.  Loads go straight to LDS (global_load_lds,
// the LDS DMA path) and complete on their own: while tile k runs its column
// phase and stores, the data of tile k+1 streams into the staging buffer and
// the block deltas of tile k+2 into the delta staging slot.  One vmcnt(0)
// wait and barrier at the head of each tile publishes all of it.
//
// Staging layout: the tile's rows in order (row = b * H + r), in 16-byte
// units (4-byte units for 4-wide blocks), so one wave's loads cover whole
// rows; the units of a row are XOR-permuted by swz(row) so that the wide
// LDS reads of the forward row phase (thread = row) fall in distinct banks
// for 8- and 16-unit bank periods alike.
//
// Compute layout: as the smaller tiles (pair rows, then rows, block b at
// column b * W) with the pitches BatchGeo::pl_pc(H) dwords and pl_rm(H)
// halfwords; the phases loop over rows (at most 4 a thread) and columns (at
// most 8 a thread, H = 4).
using lds_void = __attribute__((address_space(3))) void;
constexpr int kStageDwords = 4096;             // 8192 halfwords
constexpr int kPB = BatchGeo::kPlannedBlocks;

constexpr bool planned_fits() {
  for (int lw = 2; lw <= 6; ++lw)
    for (int lh = 2; lh <= 6; ++lh) {
      const int nb = BatchGeo::nb_planned(lw, lh), elems = nb << (lw + lh);
      if (nb < 1 || elems > 2 * kStageDwords) return false;
      if (lw == 2 && elems / 2 > 8 * 256) return false;     // eight rounds of 4-byte units
      if (lw >= 3 && elems / 8 > 4 * 256) return false;     // four rounds of 16-byte units
      if ((nb << lh) > 4 * 256) return false;                // rows: four a thread
      if (lw >= 5 && (nb << lh) > 256) return false;         // one for W >= 32
      if ((nb << lw) > (32 >> lh) * 256 && lh < 5) return false;   // columns: 32 / H a thread
      if ((nb << lw) > 256 && lh >= 5) return false;
      if (elems / (lw >= 3 ? 8 : 4) > 4 * 256) return false;        // store chunks: four a thread
      if ((nb << lw) > (8192 >> lh)) return false;                   // within the pitches
      if (BatchGeo::planned_lds_dwords(lh) > kBatchLds) return false;
    }
  return true;
}
static_assert(planned_fits(), "a planned tile does not fit its buffers or loops");

TA_DEV int swz(int row, int lcpr) { return ((row >> (4 - lcpr)) ^ (row >> (3 - lcpr))) & ((1 << lcpr) - 1); }

TA_DEV void dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

// LDS DMA loads of 16 or 4 bytes a lane from base (scalar) + voff (bytes,
// per lane, below 2^31) into the wave's LDS window at lds (wave-uniform byte
// address; lane i lands at lds + i * size).  Issued from inline assembly so
// that the compiler, which does not see them, inserts no waits of its own
// for them (it would wait on every LDS store it cannot tell apart from the
// window); dma_wait() and the tile barrier order them.  No other code of
// these kernels uses M0.
TA_DEV uint32_t lds_addr(const void* p) { return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)p); }
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"   // M0 is reserved: it is named as clobbered on purpose
TA_DEV void dma16(const void* base, uint32_t voff, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(voff), "s"(base), "s"(lds)
               : "memory", "m0");
}
TA_DEV void dma4(const void* base, uint32_t voff, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dword %0, %1" ::"v"(voff), "s"(base), "s"(lds)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// The thread index, rebuilt where it is used from the wave's base (a scalar)
// and the lane number (computed in place by an opaque instruction pair), so
// that neither it nor the addresses derived from it are kept across the
// tile loop and spilled: a spill reload waits on vmcnt, that is, on the
// loads in flight into LDS.
TA_DEV int tid_here(int wb) {
  int lane;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lane));
  return wb + lane;
}

// What the loads of a tile need.  Tile records are read through the
// constant address space (the kernel never writes them): scalar loads,
// counted apart from the vector loads and stores, so fetching the next
// record waits on neither.
struct TileHead {
  int lw, lh, count, in_stride;
  int64_t first, in_base;
};

typedef const __attribute__((address_space(4))) uint32_t* ConstWords;

TA_DEV uint32_t sload(ConstWords w, int i) { return __builtin_amdgcn_readfirstlane(w[i]); }
TA_DEV int64_t sload64(ConstWords w, int i) { return (int64_t)(((uint64_t)sload(w, i + 1) << 32) | sload(w, i)); }

TA_DEV TileHead tile_head(const BatchTile* p) {
  static_assert(offsetof(BatchTile, lw) == 0 && offsetof(BatchTile, lh) == 4 && offsetof(BatchTile, first) == 16 &&
                    offsetof(BatchTile, count) == 24 && offsetof(BatchTile, in_stride) == 28 &&
                    offsetof(BatchTile, in_base) == 64,
                "tile record layout");
  const ConstWords w = (ConstWords)p;
  return TileHead{(int)sload(w, 0), (int)sload(w, 1), (int)sload(w, 6), (int)sload(w, 7), sload64(w, 4), sload64(w, 16)};
}
TA_DEV TileHead tile_head(const BatchTile& t) { return TileHead{t.lw, t.lh, t.count, t.in_stride, t.first, t.in_base}; }
TA_DEV BatchTile uniform_tile(const BatchTile* p) {
  const ConstWords w = (ConstWords)p;
  BatchTile t;
  uint32_t* d = reinterpret_cast<uint32_t*>(&t);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(BatchTile) / 4); ++i) d[i] = sload(w, i);
  return t;
}

// block deltas of tile t -> dst (two 4-byte units per block)
TA_DEV void stage_deltas(const BatchArgs& a, const TileHead& t, int2* dst, int wb) {
  const int tx = tid_here(wb);
  const int32_t* src = a.deltas + 2 * t.first;
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int s = tx + 256 * g;
    if (s < 2 * t.count) dma4(src, 4 * s, lds_addr(reinterpret_cast<uint32_t*>(dst) + 256 * g + wb));
  }
}

// data of tile t -> stage, through its deltas dl (in LDS); a block's rows
// lie within 2^30 elements of the tile's base (the planner's rule)
TA_DEV void stage_data(const BatchArgs& a, const TileHead& t, const int2* dl, uint32_t* stage, int wb) {
  const int tx = tid_here(wb), lane = tx & 63;
  const int hm = (1 << t.lh) - 1;
  const int16_t* base = a.in + t.in_base;
  if (t.lw >= 3) {
    const int lcpr = t.lw - 3, nu = t.count << (t.lh + lcpr);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int s = g * 256 + wb + lane;
      if (s < nu) {
        const int row = s >> lcpr;
        const int c = (s & ((1 << lcpr) - 1)) ^ swz(row, lcpr);
        const uint32_t e = (uint32_t)dl[row >> t.lh].x + (uint32_t)((row & hm) * t.in_stride) + c * 8;
        dma16(base, 2 * e, lds_addr(stage + (g * 256 + wb) * 4));
      }
    }
  } else {
    const int nu = t.count << (t.lh + 1);
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const int s = g * 256 + wb + lane;
      if (s < nu) {
        const int row = s >> 1;
        const uint32_t e = (uint32_t)dl[row >> t.lh].x + (uint32_t)((row & hm) * t.in_stride) + (s & 1) * 2;
        dma4(base, 2 * e, lds_addr(stage + g * 256 + wb));
      }
    }
  }
}

TA_DEV void copy_deltas(const TileHead& t, const int2* src, int2* dst, int wb) {
  const int tx = tid_here(wb);
  if (2 * tx < t.count) reinterpret_cast<int4*>(dst)[tx] = reinterpret_cast<const int4*>(src)[tx];
}

// forward row phase from the staged rows
template <int W, class KH>
TA_DEV void fwd_rows_pl(const BatchArgs& a, const BatchTile& t, const uint32_t* stage, uint16_t* pch, int P,
                        int s_row, int wb) {
  constexpr int LC = W == 4 ? 0 : W == 8 ? 0 : W == 16 ? 1 : W == 32 ? 2 : 3;
  const int nrows = t.count << t.lh;
  // rows: at most 8192 / W, so one round for W >= 32
#pragma unroll 1
  for (int row = tid_here(wb); row < nrows; row += (W >= 32 ? 1 << 30 : 256)) {
    const int b = row >> t.lh, r = row & ((1 << t.lh) - 1);
    fx::Packed<W> x;
    if constexpr (W >= 8) {
      const uint4* src = reinterpret_cast<const uint4*>(stage) + (row << LC);
      const int f = swz(row, LC);
#pragma unroll
      for (int q = 0; q < W / 8; ++q) {
        const uint4 v = src[q ^ f];
        x.p[4 * q] = v.x; x.p[4 * q + 1] = v.y; x.p[4 * q + 2] = v.z; x.p[4 * q + 3] = v.w;
      }
    } else {
      const uint2 v = reinterpret_cast<const uint2*>(stage)[row];
      x.p[0] = v.x; x.p[1] = v.y;
    }
    const auto y = fx::run_pass<W, KH, false>(x, as_cparam(t.ph_f), as_cparam(t.ph_i), s_row, a.a);
    const int base = ((r >> 1) * P + b * W) * 2 + (r & 1);
#pragma unroll
    for (int j = 0; j < W / 2; ++j) {
      const uint32_t v = y.pair(2 * j, 2 * j + 1);
      pch[base + (2 * j) * 2] = (uint16_t)v;
      pch[base + (2 * j + 1) * 2] = (uint16_t)(v >> 16);
    }
  }
}

template <class KH>
TA_DEV void fwd_rows_pl_w(const BatchArgs& a, const BatchTile& t, const uint32_t* stage, uint16_t* pch, int P, int s,
                          int wb) {
  switch (t.lw) {
    case 2: fwd_rows_pl<4, KH>(a, t, stage, pch, P, s, wb); break;
    case 3: fwd_rows_pl<8, KH>(a, t, stage, pch, P, s, wb); break;
    case 4: fwd_rows_pl<16, KH>(a, t, stage, pch, P, s, wb); break;
    case 5: fwd_rows_pl<32, KH>(a, t, stage, pch, P, s, wb); break;
    default: fwd_rows_pl<64, KH>(a, t, stage, pch, P, s, wb); break;
  }
}

// column phase (either direction): pair rows -> transform -> barrier (they
// are dead) -> rows; a thread holds the results of its (up to 32 / H)
// columns across the barrier
template <int H, class KV, bool INV, int LH>
TA_DEV void cols_pl(const BatchArgs& a, const BatchTile& t, uint32_t* lds, int s_col, int wb) {
  constexpr int K = H >= 32 ? 1 : 32 / H;
  constexpr int P = BatchGeo::pl_pc(LH), Q = BatchGeo::pl_rm(LH);
  const int cols = t.count << t.lw, tx = tid_here(wb);
  uint32_t o[K][H / 2];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int c = tx + 256 * k;
    if (c < cols) {
      fx::Packed<H> z;
#pragma unroll
      for (int i = 0; i < H / 2; ++i) z.p[i] = lds[i * P + c];
      const auto y = fx::run_pass<H, KV, INV>(z, as_cparam(t.pv_f), as_cparam(t.pv_i), s_col, a.a);
#pragma unroll
      for (int i = 0; i < H / 2; ++i) o[k][i] = y.pair(2 * i, 2 * i + 1);
    }
  }
  tile_sync();
  uint16_t* rm = reinterpret_cast<uint16_t*>(lds);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int c = tx + 256 * k;
    if (c < cols) {
#pragma unroll
      for (int i = 0; i < H / 2; ++i) {
        rm[(2 * i) * Q + c] = (uint16_t)o[k][i];
        rm[(2 * i + 1) * Q + c] = (uint16_t)(o[k][i] >> 16);
      }
    }
  }
}

template <class KV, bool INV>
TA_DEV void cols_pl_h(const BatchArgs& a, const BatchTile& t, uint32_t* lds, int s, int wb) {
  switch (t.lh) {
    case 2: cols_pl<4, KV, INV, 2>(a, t, lds, s, wb); break;
    case 3: cols_pl<8, KV, INV, 3>(a, t, lds, s, wb); break;
    case 4: cols_pl<16, KV, INV, 4>(a, t, lds, s, wb); break;
    case 5: cols_pl<32, KV, INV, 5>(a, t, lds, s, wb); break;
    default: cols_pl<64, KV, INV, 6>(a, t, lds, s, wb); break;
  }
}

// inverse row phase, in place in the row layout
template <int W, class KH>
TA_DEV void inv_rows_pl(const BatchArgs& a, const BatchTile& t, uint16_t* rm, int Q, int s_row, int wb) {
  const int nrows = t.count << t.lh;
#pragma unroll 1
  for (int row = tid_here(wb); row < nrows; row += (W >= 32 ? 1 << 30 : 256)) {
    const int b = row >> t.lh, r = row & ((1 << t.lh) - 1);
    uint16_t* s = rm + r * Q + b * W;
    fx::Packed<W> x;
    if constexpr (W >= 8) {
#pragma unroll
      for (int q = 0; q < W / 8; ++q) {
        const uint4 v = reinterpret_cast<const uint4*>(s)[q];
        x.p[4 * q] = v.x; x.p[4 * q + 1] = v.y; x.p[4 * q + 2] = v.z; x.p[4 * q + 3] = v.w;
      }
    } else {
      const uint2 v = *reinterpret_cast<const uint2*>(s);
      x.p[0] = v.x; x.p[1] = v.y;
    }
    const auto y = fx::run_pass<W, KH, true>(x, as_cparam(t.ph_f), as_cparam(t.ph_i), s_row, a.a);
    uint32_t o[W / 2];
#pragma unroll
    for (int j = 0; j < W / 2; ++j) o[j] = y.pair(2 * j, 2 * j + 1);
    if constexpr (W >= 8) {
#pragma unroll
      for (int q = 0; q < W / 8; ++q)
        reinterpret_cast<uint4*>(s)[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
      *reinterpret_cast<uint2*>(s) = make_uint2(o[0], o[1]);
    }
  }
}

template <class KH>
TA_DEV void inv_rows_pl_w(const BatchArgs& a, const BatchTile& t, uint16_t* rm, int Q, int s, int wb) {
  switch (t.lw) {
    case 2: inv_rows_pl<4, KH>(a, t, rm, Q, s, wb); break;
    case 3: inv_rows_pl<8, KH>(a, t, rm, Q, s, wb); break;
    case 4: inv_rows_pl<16, KH>(a, t, rm, Q, s, wb); break;
    case 5: inv_rows_pl<32, KH>(a, t, rm, Q, s, wb); break;
    default: inv_rows_pl<64, KH>(a, t, rm, Q, s, wb); break;
  }
}

// inverse: the staged rows -> pair-row layout
TA_DEV void inv_scatter(const BatchTile& t, const uint32_t* stage, uint16_t* pch, int P, int wb) {
  const int hm = (1 << t.lh) - 1, tx = tid_here(wb);
  if (t.lw >= 3) {
    const int lcpr = t.lw - 3, nu = t.count << (t.lh + lcpr);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int s = tx + 256 * g;
      if (s < nu) {
        const uint4 v = reinterpret_cast<const uint4*>(stage)[s];
        const int row = s >> lcpr;
        const int c0 = ((s & ((1 << lcpr) - 1)) ^ swz(row, lcpr)) * 8;
        const int r = row & hm;
        const int base = ((r >> 1) * P + ((row >> t.lh) << t.lw) + c0) * 2 + (r & 1);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          pch[base + 4 * j] = (uint16_t)w[j];
          pch[base + 4 * j + 2] = (uint16_t)(w[j] >> 16);
        }
      }
    }
  } else {
    const int nu = t.count << (t.lh + 1);
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const int s = tx + 256 * g;
      if (s < nu) {
        const uint32_t v = stage[s];
        const int row = s >> 1, r = row & hm;
        const int base = ((r >> 1) * P + ((row >> t.lh) << 2) + (s & 1) * 2) * 2 + (r & 1);
        pch[base] = (uint16_t)v;
        pch[base + 2] = (uint16_t)(v >> 16);
      }
    }
  }
}

// coalesced store of the row layout through the deltas dl (LDS); a tile has
// at most 1024 chunks: four rounds, the LDS reads issued first
template <int LCH>
TA_DEV void store_chunks(const BatchArgs& a, const BatchTile& t, const uint16_t* rm, int Q, const int2* dl, int tx) {
  typedef typename std::conditional<LCH == 3, uint4, uint2>::type V;
  const int nch = t.count << (t.lw + t.lh - LCH);
  // every round reads a valid chunk (threads past the end repeat the last)
  // and stores only its own, so nothing is defined conditionally
  V v[4];
  int64_t off[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const Chunk k(min(tx + 256 * g, nch - 1), t.lw, t.lh, LCH);
    off[g] = t.out_base + dl[k.b].y + (int64_t)k.r * t.out_stride + k.c0;
    v[g] = *reinterpret_cast<const V*>(rm + k.r * Q + (k.b << t.lw) + k.c0);
  }
#pragma unroll
  for (int g = 0; g < 4; ++g)
    if (tx + 256 * g < nch) *reinterpret_cast<V*>(a.out + off[g]) = v[g];
}

TA_DEV void store_tile(const BatchArgs& a, const BatchTile& t, const uint16_t* rm, int Q, const int2* dl, int wb) {
  if (t.lw >= 3)
    store_chunks<3>(a, t, rm, Q, dl, tid_here(wb));
  else
    store_chunks<2>(a, t, rm, Q, dl, tid_here(wb));
}

// The walk of one workgroup over its XCD's tile list (grid stride P):
// tile k is processed while the data of k+1 and the deltas of k+2 load.
// Dynamic tile schedule.  Workgroup w of an XCD starts with tile w of its
// XCD's list; the later tiles of the list are handed out in list order by
// that list's counter, so a workgroup that draws small tiles takes more of
// them and all finish together.  A workgroup takes its next tile two tiles
// ahead of use (the pipeline stages the deltas of tile k+2 while running
// tile k) and only once the one before exists; the last workgroup to finish
// sets the counters back to zero for the next launch.  Two launches that use
// the same counters must therefore not run at the same time.
// The counters sit kSchedPitch dwords apart (own cache lines): counter x
// at sched[x * kSchedPitch], the finished-workgroup count after the eight.
TA_DEV int sched_take(int32_t* sched, int xcd, int k) {
  return __hip_atomic_fetch_add(sched + xcd * kSchedPitch, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// one lane per workgroup, after the last take of the workgroup has returned
TA_DEV void sched_done(int32_t* sched) {
  if (__hip_atomic_fetch_add(sched + kXcds * kSchedPitch, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
      (int)gridDim.x - 1) {
#pragma unroll
    for (int x = 0; x <= kXcds; ++x)
      __hip_atomic_store(sched + x * kSchedPitch, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <bool INV>
TA_DEV void planned_tiles(const BatchArgs& a, uint32_t* lds, uint32_t* stage, int2 (*ring)[kPB], int2* dnext,
                          int* slot) {
  // tile indices fit int32 (the planner's rule), so the loop tests are scalar
  const int xcd = blockIdx.x % kXcds;
  const int P = (gridDim.x + kXcds - 1 - xcd) / kXcds;
  const int end = a.xcount ? (int)a.xstart[xcd] + a.xcount[xcd] : (int)a.xstart[xcd + 1];
  const int dyn0 = (int)a.xstart[xcd] + P;     // the first tile the counter hands out
  int32_t* const sched = a.sched;
  int ti = (int)a.xstart[xcd] + blockIdx.x / kXcds;
  const int wb = __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63;   // this wave's first thread
  if (ti >= end) {
    if (sched && tid_here(wb) == 0) sched_done(sched);
    return;
  }
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  // n1, n2: the next two tiles (end or beyond: none)
  int n1, n2;
  // prologue: deltas and data of the first tile, deltas of the second
  {
    int got = 0;
    if (sched && tid_here(wb) == 0) got = sched_take(sched, xcd, 2);
    const TileHead h0 = tile_head(a.tiles + ti);
    stage_deltas(a, h0, ring[0], wb);
    dma_wait();
    if (sched && tid_here(wb) == 0) *slot = got;
    tile_sync();
    if (sched) {
      n1 = dyn0 + __builtin_amdgcn_readfirstlane(*slot);
      n2 = n1 + 1;
    } else {
      n1 = ti + P;
      n2 = ti + 2 * P;
    }
    stage_data(a, h0, ring[0], stage, wb);
    if (n1 < end) stage_deltas(a, tile_head(a.tiles + n1), dnext, wb);
  }
  int cur = 0;
  bool pending = false;   // the take of n2 has landed in *slot
  for (;;) {
    // tile records are re-read each step (scalar loads, cheap) rather than
    // carried across the loop in scalar registers
    const BatchTile t = uniform_tile(a.tiles + ti);
    dma_wait();                          // this tile's data, the next deltas, the last stores
    tile_sync();
    if (pending) n2 = dyn0 + __builtin_amdgcn_readfirstlane(*slot);
    const bool has_n = n1 < end, has_nn = n2 < end;
    // the tile after n2 (once n2 exists), taken a whole tile ahead of use so
    // that its round trip overlaps this tile's work
    // The take goes out where its result costs least: in the inverse at the
    // tile head, its result written to *slot after the stores (a whole tile
    // later); in the forward, whose phases hold every register, after the
    // stores, written at once (the wait then also covers the loads and stores
    // in flight, which the next tile head waits for anyway).
    [[maybe_unused]] int got = 0;
    if constexpr (INV) {
      if (sched && has_nn && tid_here(wb) == 0) got = sched_take(sched, xcd, 1);
    }
    if (has_n) copy_deltas(tile_head(a.tiles + n1), dnext, ring[cur ^ 1], wb);
    const int PP = BatchGeo::pl_pc(t.lh), Q = BatchGeo::pl_rm(t.lh);
    if (INV) {
      inv_scatter(t, stage, pch, PP, wb);
    } else {
      const int s_row = t.lw + a.bd + a.m - 15;
      switch (t.kind_h) {
        case 0: fwd_rows_pl_w<KC2>(a, t, stage, pch, PP, s_row, wb); break;
        case 1: fwd_rows_pl_w<KS3>(a, t, stage, pch, PP, s_row, wb); break;
        default: fwd_rows_pl_w<KC3>(a, t, stage, pch, PP, s_row, wb); break;
      }
    }
    tile_sync();                         // stage and dnext are free
    if (has_n) stage_data(a, tile_head(a.tiles + n1), ring[cur ^ 1], stage, wb);
    if (has_nn) stage_deltas(a, tile_head(a.tiles + n2), dnext, wb);
    const int s_col = INV ? a.m + 1 : t.lh + a.m;
    switch (t.kind_v) {
      case 0: cols_pl_h<KC2, INV>(a, t, lds, s_col, wb); break;
      case 1: cols_pl_h<KS3, INV>(a, t, lds, s_col, wb); break;
      default: cols_pl_h<KC3, INV>(a, t, lds, s_col, wb); break;
    }
    tile_sync();
    if (INV) {
      const int s_row = a.m + 14 - a.bd;
      switch (t.kind_h) {
        case 0: inv_rows_pl_w<KC2>(a, t, pch, Q, s_row, wb); break;
        case 1: inv_rows_pl_w<KS3>(a, t, pch, Q, s_row, wb); break;
        default: inv_rows_pl_w<KC3>(a, t, pch, Q, s_row, wb); break;
      }
      tile_sync();
    }
    store_tile(a, t, pch, Q, ring[cur], wb);
    if constexpr (INV) {
      if (sched && has_nn && tid_here(wb) == 0) *slot = got;
    }
    if (!has_n) break;   // (then n2 does not exist either and nothing was taken)
    ti = n1;
    n1 = n2;
    if (sched) {
      pending = n1 < end;
      if constexpr (!INV) {
        if (pending && tid_here(wb) == 0) *slot = sched_take(sched, xcd, 1);
      }
      if (!pending) n2 = end;   // the counter only grows: once past the end, always past it
    } else {
      n2 = n1 + P;
    }
    cur ^= 1;
  }
  if (sched && tid_here(wb) == 0) sched_done(sched);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_fwd(BatchArgs a) {
  __shared__ __align__(16) uint32_t lds[kBatchLds];
  __shared__ __align__(16) uint32_t stage[kStageDwords];
  __shared__ __align__(16) int2 ring[2][kPB];
  __shared__ __align__(16) int2 dnext[kPB];
  __shared__ int slot;
  planned_tiles<false>(a, lds, stage, ring, dnext, &slot);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_inv(BatchArgs a) {
  __shared__ __align__(16) uint32_t lds[kBatchLds];
  __shared__ __align__(16) uint32_t stage[kStageDwords];
  __shared__ __align__(16) int2 ring[2][kPB];
  __shared__ __align__(16) int2 dnext[kPB];
  __shared__ int slot;
  planned_tiles<true>(a, lds, stage, ring, dnext, &slot);
}

// ---------------------------------------------------------------- fp32 tiles
// The same phases on fp32 data with the orthonormal fp32 stages (no
// rounding), in the BatchGeoF32 layout: block b at b * BS, column-major
// (pitch H + 1) between the row and column phases, row-major (pitch W + 1)
// for the second phase's output and the coalesced float4 loads and stores.
constexpr int kBatchLdsF32 = BatchGeoF32::kLds;

TA_DEV const float* fparam(const uint32_t* p) { return reinterpret_cast<const float*>(p); }

template <int W>
TA_DEV void load_rowf(const float* __restrict__ src, fp::Vec<W>& x) {
#pragma unroll
  for (int q = 0; q < W / 4; ++q) {
    const float4 v = reinterpret_cast<const float4*>(src)[q];
    x.v[4 * q] = v.x; x.v[4 * q + 1] = v.y; x.v[4 * q + 2] = v.z; x.v[4 * q + 3] = v.w;
  }
}

// descriptor of block b of an fp32 tile: entry first + b of the list, or of
// the list's index when one is given (device-planned lists)
TA_DEV ta_block tile_block_f(const BatchArgs& a, const ta_block* blocks, const BatchTile& t, int b) {
  return a.order ? blocks[a.order[t.first + b]] : blocks[t.first + b];
}

// forward row phase: global row -> transform -> column-major LDS
template <int W, class KH>
TA_DEV void fwd_rows_f(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, float* lds, BDesc* desc) {
  const int tid = threadIdx.x;
  if (tid >= (t.count << t.lh)) return;
  const int b = tid >> t.lh, r = tid & ((1 << t.lh) - 1), h1 = (1 << t.lh) + 1;
  const ta_block d = tile_block_f(a, blocks, t, b);
  if (r == 0) desc[b] = BDesc{d.in_off, d.out_off, d.in_stride, d.out_stride};
  fp::Vec<W> x;
  load_rowf<W>(reinterpret_cast<const float*>(a.in) + d.in_off + (int64_t)r * d.in_stride, x);
  const fp::Vec<W> y = fp::run_pass<W, KH, false>(x, fparam(t.ph_f), fparam(t.ph_i));
  float* blk = lds + b * BatchGeoF32::bs(t.lw, t.lh) + r;
#pragma unroll
  for (int c = 0; c < W; ++c) blk[c * h1] = y.v[c];
}

// column phase (either direction): column-major LDS -> transform -> barrier
// -> row-major LDS
template <int H, class KV, bool INV>
TA_DEV void cols_f(const BatchTile& t, float* lds) {
  const int tid = threadIdx.x;
  const bool act = tid < (t.count << t.lw);
  const int b = tid >> t.lw, c = tid & ((1 << t.lw) - 1), w1 = (1 << t.lw) + 1;
  float* blk = lds + b * BatchGeoF32::bs(t.lw, t.lh);
  fp::Vec<H> z;
  if (act) {
#pragma unroll
    for (int r = 0; r < H; ++r) z.v[r] = blk[c * (H + 1) + r];
    z = fp::run_pass<H, KV, INV>(z, fparam(t.pv_f), fparam(t.pv_i));
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < H; ++r) blk[r * w1 + c] = z.v[r];
  }
}

// inverse row phase: row-major LDS row -> transform -> back over the row
template <int W, class KH>
TA_DEV void inv_rows_f(const BatchTile& t, float* lds) {
  const int tid = threadIdx.x;
  if (tid >= (t.count << t.lh)) return;
  const int b = tid >> t.lh, r = tid & ((1 << t.lh) - 1);
  float* row = lds + b * BatchGeoF32::bs(t.lw, t.lh) + r * (W + 1);
  fp::Vec<W> x;
#pragma unroll
  for (int c = 0; c < W; ++c) x.v[c] = row[c];
  const fp::Vec<W> y = fp::run_pass<W, KH, true>(x, fparam(t.ph_f), fparam(t.ph_i));
#pragma unroll
  for (int c = 0; c < W; ++c) row[c] = y.v[c];
}

template <class KH>
TA_DEV void fwd_rows_fw(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, float* lds, BDesc* desc) {
  switch (t.lw) {
    case 2: fwd_rows_f<4, KH>(a, t, blocks, lds, desc); break;
    case 3: fwd_rows_f<8, KH>(a, t, blocks, lds, desc); break;
    case 4: fwd_rows_f<16, KH>(a, t, blocks, lds, desc); break;
    case 5: fwd_rows_f<32, KH>(a, t, blocks, lds, desc); break;
    default: fwd_rows_f<64, KH>(a, t, blocks, lds, desc); break;
  }
}

template <class KH>
TA_DEV void inv_rows_fw(const BatchTile& t, float* lds) {
  switch (t.lw) {
    case 2: inv_rows_f<4, KH>(t, lds); break;
    case 3: inv_rows_f<8, KH>(t, lds); break;
    case 4: inv_rows_f<16, KH>(t, lds); break;
    case 5: inv_rows_f<32, KH>(t, lds); break;
    default: inv_rows_f<64, KH>(t, lds); break;
  }
}

template <class KV, bool INV>
TA_DEV void cols_fh(const BatchTile& t, float* lds) {
  switch (t.lh) {
    case 2: cols_f<4, KV, INV>(t, lds); break;
    case 3: cols_f<8, KV, INV>(t, lds); break;
    case 4: cols_f<16, KV, INV>(t, lds); break;
    case 5: cols_f<32, KV, INV>(t, lds); break;
    default: cols_f<64, KV, INV>(t, lds); break;
  }
}

template <bool INV>
TA_DEV void cols_f_kind(const BatchTile& t, float* lds) {
  switch (t.kind_v) {
    case 0: cols_fh<KC2, INV>(t, lds); break;
    case 1: cols_fh<KS3, INV>(t, lds); break;
    default: cols_fh<KC3, INV>(t, lds); break;
  }
}

// Coalesced float4 stores of the tile from the row-major layout.
TA_DEV void store_tile_f(const BatchArgs& a, const BatchTile& t, const float* lds, const BDesc* desc) {
  const int lq = t.lw - 2;                       // log2 float4 chunks per row
  const int nch = t.count << (t.lh + lq), w1 = (1 << t.lw) + 1, bs = BatchGeoF32::bs(t.lw, t.lh);
  float* out = reinterpret_cast<float*>(a.out);
  for (int ch = threadIdx.x; ch < nch; ch += 256) {
    const int b = ch >> (t.lh + lq), r = (ch >> lq) & ((1 << t.lh) - 1), c0 = (ch & ((1 << lq) - 1)) << 2;
    const BDesc d = desc[b];
    const float* s = lds + b * bs + r * w1 + c0;
    *reinterpret_cast<float4*>(out + d.out_off + (int64_t)r * d.out_stride + c0) = make_float4(s[0], s[1], s[2], s[3]);
  }
}

// One fp32 tile of the forward.  Ends with a barrier.
TA_DEV void fwd_tile_f(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, float* lds, BDesc* desc) {
  switch (t.kind_h) {
    case 0: fwd_rows_fw<KC2>(a, t, blocks, lds, desc); break;
    case 1: fwd_rows_fw<KS3>(a, t, blocks, lds, desc); break;
    default: fwd_rows_fw<KC3>(a, t, blocks, lds, desc); break;
  }
  __syncthreads();
  cols_f_kind<false>(t, lds);
  __syncthreads();
  store_tile_f(a, t, lds, desc);
  __syncthreads();
}

// One fp32 tile of the inverse: coalesced loads -> column-major LDS ->
// columns -> row-major LDS -> rows in place -> coalesced stores.  Ends with
// a barrier.
TA_DEV void inv_tile_f(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, float* lds, BDesc* desc) {
  if ((int)threadIdx.x < t.count) {
    const ta_block d = tile_block_f(a, blocks, t, (int)threadIdx.x);
    desc[threadIdx.x] = BDesc{d.in_off, d.out_off, d.in_stride, d.out_stride};
  }
  __syncthreads();
  {
    // at most 2048 float4 chunks per tile: two rounds of (at most) 4 loads
    // per thread, each round's loads issued together before any is written
    // to LDS
    const int lq = t.lw - 2;
    const int nch = t.count << (t.lh + lq), h1 = (1 << t.lh) + 1, bs = BatchGeoF32::bs(t.lw, t.lh);
    const float* in = reinterpret_cast<const float*>(a.in);
#pragma unroll
    for (int k0 = 0; k0 < 8; k0 += 4) {
      float4 v[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int ch = threadIdx.x + 256 * (k0 + g);
        if (ch < nch) {
          const int b = ch >> (t.lh + lq), r = (ch >> lq) & ((1 << t.lh) - 1), c0 = (ch & ((1 << lq) - 1)) << 2;
          const BDesc d = desc[b];
          v[g] = *reinterpret_cast<const float4*>(in + d.in_off + (int64_t)r * d.in_stride + c0);
        }
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int ch = threadIdx.x + 256 * (k0 + g);
        if (ch < nch) {
          const int b = ch >> (t.lh + lq), r = (ch >> lq) & ((1 << t.lh) - 1), c0 = (ch & ((1 << lq) - 1)) << 2;
          float* dst = lds + b * bs + c0 * h1 + r;
          dst[0] = v[g].x; dst[h1] = v[g].y; dst[2 * h1] = v[g].z; dst[3 * h1] = v[g].w;
        }
      }
    }
  }
  __syncthreads();
  cols_f_kind<true>(t, lds);
  __syncthreads();
  switch (t.kind_h) {
    case 0: inv_rows_fw<KC2>(t, lds); break;
    case 1: inv_rows_fw<KS3>(t, lds); break;
    default: inv_rows_fw<KC3>(t, lds); break;
  }
  __syncthreads();
  store_tile_f(a, t, lds, desc);
  __syncthreads();
}

template <bool INV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_f32(BatchArgs a) {
  __shared__ __align__(16) float lds[kBatchLdsF32];
  __shared__ BDesc desc[kMaxTileBlocks];
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = (gridDim.x + kXcds - 1 - xcd) / kXcds;
  const int64_t end = a.xcount ? a.xstart[xcd] + a.xcount[xcd] : a.xstart[xcd + 1];
  for (int64_t ti = a.xstart[xcd] + blockIdx.x / kXcds; ti < end; ti += per_xcd) {
    const BatchTile t = a.tiles[ti];
    if (INV)
      inv_tile_f(a, t, a.blocks, lds, desc);
    else
      fwd_tile_f(a, t, a.blocks, lds, desc);
  }
}

// ---------------------------------------------------------------- block lists
// Unplanned: the descriptor list is cut into sort windows of kSortWin
// consecutive descriptors, each handled by kSortWin / kDescWindow workgroups
// ("quarters").  Every quarter sorts the whole window in LDS by
// (configuration, position) with a bitonic network, which groups the
// window's descriptors of equal size and axis ids in list order, and then
// runs its own kDescWindow sorted entries as tiles of up to BatchGeo::nb_for
// blocks.  The quarters of all windows are split into kXcds contiguous
// ranges, one per XCD (workgroup b runs on XCD b mod kXcds), so that
// neighbouring blocks of a list in frame order share their L2.  A descriptor
// that the planner would reject (size outside 4..64, negative offset, stride
// below the width, offsets or strides not multiples of the vector width, an
// axis id outside the table or with no batched kind at its size) sorts last
// and is skipped: its output is left untouched.
constexpr int kSortWin = 1024;
constexpr int kQuarters = kSortQuarters;
static_assert(kSortWin == kDescWindow * kSortQuarters, "sort window");
static_assert(kDescWindow == 256 && kSortWin % kDescWindow == 0, "one sorted entry per thread of a quarter");
static_assert(kAxisIds <= 256, "axis ids take 8 key bits");

// 22-bit configuration key of a descriptor, or -1 when it breaks a rule
TA_DEV int config_key(const AxisDev* axes, const ta_block& d) {
  const int ch = d.log2w >= 3 ? 8 : 4;                  // elements per vector access
  if (d.log2w < 2 || d.log2w > 6 || d.log2h < 2 || d.log2h > 6 || d.in_off < 0 || d.out_off < 0 ||
      d.in_stride < (1 << d.log2w) || d.out_stride < (1 << d.log2w) || d.axis_h >= kAxisIds ||
      d.axis_v >= kAxisIds || ((d.in_off | d.out_off | (int64_t)d.in_stride | (int64_t)d.out_stride) & (ch - 1)))
    return -1;
  if (axes[d.axis_h * kAxisSizes + d.log2w].kind < 0 || axes[d.axis_v * kAxisSizes + d.log2h].kind < 0) return -1;
  return d.log2w | (d.log2h << 3) | (d.axis_h << 6) | (d.axis_v << 14);
}

// (fp32: the larger tile buffer leaves room for three workgroups per CU)
template <bool INV, bool F32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(F32 ? 3 : 4))) void batch_desc(BatchArgs a) {
  __shared__ __align__(16) uint32_t lds[F32 ? kBatchLdsF32 : kBatchLds];
  __shared__ BDesc desc[kMaxTileBlocks];
  __shared__ uint32_t skey[kSortWin];            // (configuration << 10 | position), sorted
  __shared__ ta_block qdesc[kDescWindow];        // this quarter's descriptors, in sorted order
  constexpr uint32_t kInvalid = ~0u;             // above every valid key (lw <= 6)
  const int tid = threadIdx.x;
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = (gridDim.x + kXcds - 1 - xcd) / kXcds;   // >= 1: the grid has >= kXcds groups
  const int64_t nunits = (a.nblocks + kSortWin - 1) / kSortWin * kQuarters;
  const int64_t uend = nunits * (xcd + 1) / kXcds;
  for (int64_t u = nunits * xcd / kXcds + blockIdx.x / kXcds; u < uend; u += per_xcd) {
    const int64_t w0 = u / kQuarters * kSortWin;
    const int q0 = (int)(u % kQuarters) * kDescWindow;
    const int cnt = (int)min<int64_t>(kSortWin, a.nblocks - w0);
#pragma unroll
    for (int r = 0; r < kQuarters; ++r) {
      const int i = tid + r * 256;
      uint32_t sk = kInvalid;
      if (i < cnt) {
        const int k = config_key(a.axes, a.blocks[w0 + i]);
        if (k >= 0) sk = ((uint32_t)k << 10) | (uint32_t)i;
      }
      skey[i] = sk;
    }
    // ascending sort; the position in the low bits makes every key
    // distinct, so equal configurations keep list order
    bitonic_sort_window<kSortWin>(skey, tid);
    __syncthreads();
    const int qcnt = min(kDescWindow, cnt - q0);
    if (tid < qcnt && skey[q0 + tid] != kInvalid) qdesc[tid] = a.blocks[w0 + (skey[q0 + tid] & (kSortWin - 1))];
    __syncthreads();
    int j = 0;
    while (j < qcnt) {                 // every thread walks the same runs
      const uint32_t s0 = skey[q0 + j];
      if (s0 == kInvalid) break;       // the rest are invalid too
      const uint32_t k = s0 >> 10;
      const int lw = (int)(k & 7), lh = (int)((k >> 3) & 7);
      const int ah = (int)((k >> 6) & 0xff), av = (int)((k >> 14) & 0xff);
      const int cap = F32 ? BatchGeoF32::nb_for(lw, lh) : BatchGeo::nb_for(lw, lh);
      int len = 1;
      while (j + len < qcnt && len < cap && (skey[q0 + j + len] >> 10) == k) ++len;
      const AxisDev& h = a.axes[ah * kAxisSizes + lw];
      const AxisDev& v = a.axes[av * kAxisSizes + lh];
      BatchTile t;
      t.lw = lw;
      t.lh = lh;
      t.kind_h = h.kind;
      t.kind_v = v.kind;
      t.first = j;
      t.count = len;
      t.pad = 0;
      if (F32) {
        t.ph_f = reinterpret_cast<const uint32_t*>(h.ff);
        t.ph_i = reinterpret_cast<const uint32_t*>(h.fi);
        t.pv_f = reinterpret_cast<const uint32_t*>(v.ff);
        t.pv_i = reinterpret_cast<const uint32_t*>(v.fi);
        float* fl = reinterpret_cast<float*>(lds);
        if (INV)
          inv_tile_f(a, t, qdesc, fl, desc);
        else
          fwd_tile_f(a, t, qdesc, fl, desc);
      } else {
        t.ph_f = h.pf;
        t.ph_i = h.pi;
        t.pv_f = v.pf;
        t.pv_i = v.pi;
        if (INV)
          inv_tile(a, t, qdesc, lds, desc);
        else
          fwd_tile(a, t, qdesc, lds, desc);
      }
      j += len;
    }
    __syncthreads();                   // the window buffers are rewritten next
  }
}


// ---------------------------------------------------------------- device planning
// Block lists planned on the device (ta_transform_fwd_ws / _inv_ws).  One
// workgroup per window of kPlanWin consecutive descriptors:
//  1. the valid descriptors (the block-list rules, an axis kind of the fast
//     kernels, and rows that span at most 2^30 input and 2^31 output
//     elements) enter their configuration (size and axis ids) in a hash
//     table in LDS and take a rank in its slot; the others are skipped;
//  2. a scan over the slots' counts groups the window by configuration;
//  3. tile cuts where the configuration or the row strides change and after
//     every nb_planned(size) blocks of a run (two scans: the start of each
//     entry's run, then the tile index of each entry);
//  4. the tiles go to the list of XCD (window mod kXcds), at slots taken
//     from that list's counter; each block's deltas are its offsets minus
//     the window's smallest input and output offsets.  A window whose blocks
//     span more than 2^30 input or 2^31 output elements makes every block a
//     tile of its own, based at its own offsets.
constexpr int kPlanPer = kPlanWin / kPlanThreads;     // grouped entries per thread (consecutive)
constexpr int64_t kSpanIn = int64_t(1) << 30, kSpanOut = int64_t(1) << 31;

// Scan of the threads' values (sum, or maximum with MAX) across the
// workgroup: within each wave by shuffles, then over the wave totals in
// wsum.  Returns the exclusive result (0, or -1 with MAX, for thread 0) and
// the total in *total.  Two barriers.
template <bool MAX>
TA_DEV int scan_excl(int v, int* wsum, int tid, int* total) {
  constexpr int kWaves = kPlanThreads / 64, kId = MAX ? -1 : 0;
  const int lane = tid & 63, wave = tid >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc = MAX ? max(inc, y) : inc + y;
  }
  int exc = __shfl_up(inc, 1);
  if (lane == 0) exc = kId;
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  int pre = kId, tot = kId;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const int x = wsum[w];
    if (w < wave) pre = MAX ? max(pre, x) : pre + x;
    tot = MAX ? max(tot, x) : tot + x;
  }
  __syncthreads();                     // wsum is free for the next scan
  *total = tot;
  return MAX ? max(pre, exc) : pre + exc;
}

// the rules of the fast kernels, plus (int16) the row spans the deltas can hold
template <bool F32>
TA_DEV int plan_key(const AxisDev* axes, const ta_block& d) {
  const int k = config_key(axes, d);
  if (k < 0 || F32) return k;
  const int64_t w = int64_t(1) << d.log2w, hm1 = (int64_t(1) << d.log2h) - 1;
  if (hm1 * d.in_stride + w > kSpanIn || hm1 * d.out_stride + w > kSpanOut) return -1;
  return k;
}

// (fp32: the tiles are those of batch_f32, which reads each block's
// descriptor; the list indices of the window's blocks are written in grouped
// order instead of deltas, and the span fallback does not apply)
template <bool F32>
__global__ __launch_bounds__(kPlanThreads) void desc_plan(PlanArgs a) {
  constexpr int kWaves = kPlanThreads / 64;
  constexpr uint32_t kEmpty = ~0u;     // above every configuration key (22 bits)
  __shared__ uint32_t hkey[kPlanWin + 1];   // hash table of configurations; later the tile starts
  __shared__ int hcnt[kPlanWin];            // blocks per table slot, then the slot's first position
  __shared__ int order[kPlanWin];           // grouped position -> window entry
  __shared__ int wsum[kWaves];
  __shared__ int64_t red[kWaves][4];   // per wave: min in, max in end, min out, max out end
  __shared__ int base_slot;
  int* sc = reinterpret_cast<int*>(hkey);
  const int tid = threadIdx.x;
  const int64_t w0 = (int64_t)blockIdx.x * kPlanWin;
  const int cnt = (int)min<int64_t>(kPlanWin, a.nblocks - w0);
  const int xcd = (int)(blockIdx.x % kXcds);
#pragma unroll
  for (int r = 0; r < kPlanPer; ++r) {
    hkey[tid + kPlanThreads * r] = kEmpty;
    hcnt[tid + kPlanThreads * r] = 0;
  }
  __syncthreads();
  // 1. each valid descriptor finds its configuration's slot in the table
  //    (open addressing: at most kPlanWin keys in kPlanWin slots, so a free
  //    slot always exists) and takes a rank in it; the window's offset range
  //    over its valid blocks.  The loads of a thread's descriptors are
  //    issued together.
  int64_t mn_i = INT64_MAX, mx_i = INT64_MIN, mn_o = INT64_MAX, mx_o = INT64_MIN;
  uint32_t slot_rank[kPlanPer];        // slot << 12 | rank, or kEmpty
  {
    ta_block d[kPlanPer];
#pragma unroll
    for (int r = 0; r < kPlanPer; ++r) {
      const int i = tid + kPlanThreads * r;
      if (i < cnt) d[r] = a.blocks[w0 + i];
    }
#pragma unroll
    for (int r = 0; r < kPlanPer; ++r) {
      const int i = tid + kPlanThreads * r;
      slot_rank[r] = kEmpty;
      if (i < cnt) {
        const int c = plan_key<F32>(a.axes, d[r]);
        if (c >= 0) {
          uint32_t sl = ((uint32_t)c * 0x9E3779B1u) >> (32 - 12);
          for (;;) {
            const uint32_t old = atomicCAS(&hkey[sl], kEmpty, (uint32_t)c);
            if (old == kEmpty || old == (uint32_t)c) break;
            sl = (sl + 1) & (kPlanWin - 1);
          }
          slot_rank[r] = (sl << 12) | (uint32_t)atomicAdd(&hcnt[sl], 1);
          const int64_t hm1 = (int64_t(1) << d[r].log2h) - 1, w = int64_t(1) << d[r].log2w;
          mn_i = min(mn_i, d[r].in_off);
          mx_i = max(mx_i, d[r].in_off + hm1 * d[r].in_stride + w);
          mn_o = min(mn_o, d[r].out_off);
          mx_o = max(mx_o, d[r].out_off + hm1 * d[r].out_stride + w);
        }
      }
    }
  }
  static_assert(kPlanWin == 1 << 12, "12-bit slots and ranks");
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn_i = min(mn_i, (int64_t)__shfl_xor((long long)mn_i, o));
    mx_i = max(mx_i, (int64_t)__shfl_xor((long long)mx_i, o));
    mn_o = min(mn_o, (int64_t)__shfl_xor((long long)mn_o, o));
    mx_o = max(mx_o, (int64_t)__shfl_xor((long long)mx_o, o));
  }
  if ((tid & 63) == 0) {
    red[tid >> 6][0] = mn_i;
    red[tid >> 6][1] = mx_i;
    red[tid >> 6][2] = mn_o;
    red[tid >> 6][3] = mx_o;
  }
  __syncthreads();
  // 2. group the entries by slot: the slots' first positions (a scan over the
  //    table, this thread's slots 4 tid .. 4 tid + 3), then each entry's
  //    grouped position
  int nvalid;
  {
    int c4[kPlanPer], sum = 0;
#pragma unroll
    for (int e = 0; e < kPlanPer; ++e) {
      c4[e] = hcnt[tid * kPlanPer + e];
      sum += c4[e];
    }
    int pre = scan_excl<false>(sum, wsum, tid, &nvalid);
#pragma unroll
    for (int e = 0; e < kPlanPer; ++e) {
      hcnt[tid * kPlanPer + e] = pre;
      pre += c4[e];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPlanPer; ++r)
    if (slot_rank[r] != kEmpty)
      order[hcnt[slot_rank[r] >> 12] + (int)(slot_rank[r] & (kPlanWin - 1))] = tid + kPlanThreads * r;
  __syncthreads();
  int64_t wmin_i = INT64_MAX, wmax_i = INT64_MIN, wmin_o = INT64_MAX, wmax_o = INT64_MIN;
#pragma unroll
  for (int v = 0; v < kWaves; ++v) {
    wmin_i = min(wmin_i, red[v][0]);
    wmax_i = max(wmax_i, red[v][1]);
    wmin_o = min(wmin_o, red[v][2]);
    wmax_o = max(wmax_o, red[v][3]);
  }
  const bool own = !F32 && nvalid > 0 && (wmax_i - wmin_i > kSpanIn || wmax_o - wmin_o > kSpanOut);
  // 3. this thread's consecutive grouped entries [e0, e0 + kPlanPer): their
  //    descriptors (and the one before the first), run starts
  const int e0 = tid * kPlanPer;
  ta_block d[kPlanPer + 1];            // d[0]: entry e0 - 1
#pragma unroll
  for (int e = 0; e <= kPlanPer; ++e) {
    const int i = e0 + e - 1;
    if (i >= 0 && i < nvalid) d[e] = a.blocks[w0 + order[i]];
  }
  int last_start = -1;                 // the last run start among this thread's entries
  uint32_t starts = 0;                 // bit e: entry e0 + e starts a run
#pragma unroll
  for (int e = 0; e < kPlanPer; ++e) {
    const int i = e0 + e;
    if (i < nvalid) {
      const ta_block &p = d[e], &q = d[e + 1];
      const bool st = i == 0 || own || q.log2w != p.log2w || q.log2h != p.log2h || q.axis_h != p.axis_h ||
                      q.axis_v != p.axis_v || q.in_stride != p.in_stride || q.out_stride != p.out_stride;
      if (st) {
        starts |= 1u << e;
        last_start = i;
      }
    }
  }
  int last_any;
  int run0 = scan_excl<true>(last_start, wsum, tid, &last_any);   // the run start before this thread's entries
  // tile cuts: a run start, or every nb_planned blocks into a run
  uint32_t cuts = 0;
  int ncut = 0;
#pragma unroll
  for (int e = 0; e < kPlanPer; ++e) {
    const int i = e0 + e;
    if (i < nvalid) {
      if (starts & (1u << e)) run0 = i;
      const int cap = F32 ? BatchGeoF32::nb_for(d[e + 1].log2w, d[e + 1].log2h)
                          : BatchGeo::nb_planned(d[e + 1].log2w, d[e + 1].log2h);
      if ((i - run0) % cap == 0) {
        cuts |= 1u << e;
        ++ncut;
      }
    }
  }
  int ntiles;
  const int tile0 = scan_excl<false>(ncut, wsum, tid, &ntiles) - 1;   // tile index before this thread's entries
  // 4. slots in this XCD's list; tile start positions
  if (tid == 0)
    base_slot = ntiles > 0 ? __hip_atomic_fetch_add(a.count + xcd, ntiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : 0;
  {
    int tile = tile0;
#pragma unroll
    for (int e = 0; e < kPlanPer; ++e)
      if (cuts & (1u << e)) sc[++tile] = e0 + e;
  }
  if (tid == 0) sc[ntiles] = nvalid;
  __syncthreads();
  const int64_t slot0 = (int64_t)xcd * a.cap + base_slot;
  if (base_slot + ntiles > a.cap) return;   // (cannot happen: the lists hold every window's blocks)
  int tile = tile0;
#pragma unroll
  for (int e = 0; e < kPlanPer; ++e) {
    const int i = e0 + e;
    if (i >= nvalid) continue;
    const ta_block& b = d[e + 1];
    const int64_t ib = own ? b.in_off : wmin_i, ob = own ? b.out_off : wmin_o;
    if (F32) {
      a.index[w0 + i] = (int32_t)(w0 + order[i]);
    } else {
      a.deltas[2 * (w0 + i)] = (int32_t)(b.in_off - ib);
      a.deltas[2 * (w0 + i) + 1] = (int32_t)(b.out_off - ob);
    }
    if (cuts & (1u << e)) {
      ++tile;
      const int lw = b.log2w, lh = b.log2h;
      const AxisDev& h = a.axes[b.axis_h * kAxisSizes + lw];
      const AxisDev& v = a.axes[b.axis_v * kAxisSizes + lh];
      BatchTile t;
      t.lw = lw;
      t.lh = lh;
      t.kind_h = h.kind;
      t.kind_v = v.kind;
      t.first = w0 + i;
      t.count = sc[tile + 1] - i;
      t.in_stride = b.in_stride;
      if (F32) {
        t.ph_f = reinterpret_cast<const uint32_t*>(h.ff);
        t.ph_i = reinterpret_cast<const uint32_t*>(h.fi);
        t.pv_f = reinterpret_cast<const uint32_t*>(v.ff);
        t.pv_i = reinterpret_cast<const uint32_t*>(v.fi);
      } else {
        t.ph_f = h.pf;
        t.ph_i = h.pi;
        t.pv_f = v.pf;
        t.pv_i = v.pi;
      }
      t.in_base = ib;
      t.out_base = ob;
      t.out_stride = b.out_stride;
      t.pad = 0;
      a.tiles[slot0 + tile] = t;
    }
  }
}

__global__ __launch_bounds__(256) void zero_words(int32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += 256) p[i] = 0;
}
}  // namespace

const void* batch_kernel(int inv, int desc, int f32) {
  if (desc && f32)
    return inv ? reinterpret_cast<const void*>(&batch_desc<true, true>)
               : reinterpret_cast<const void*>(&batch_desc<false, true>);
  if (desc)
    return inv ? reinterpret_cast<const void*>(&batch_desc<true, false>)
               : reinterpret_cast<const void*>(&batch_desc<false, false>);
  if (f32) return inv ? reinterpret_cast<const void*>(&batch_f32<true>) : reinterpret_cast<const void*>(&batch_f32<false>);
  return inv ? reinterpret_cast<const void*>(&batch_inv) : reinterpret_cast<const void*>(&batch_fwd);
}

const void* desc_plan_kernel(int f32) {
  return f32 ? reinterpret_cast<const void*>(&desc_plan<true>) : reinterpret_cast<const void*>(&desc_plan<false>);
}
const void* zero_words_kernel() { return reinterpret_cast<const void*>(&zero_words); }

}  // namespace ta
