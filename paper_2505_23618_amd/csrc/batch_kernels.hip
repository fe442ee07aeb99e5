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
// The planned kernels overlap a tile's global loads with the work on the
// tile before.  Loads go straight to LDS (global_load_lds, the LDS DMA path)
// and complete on their own: while tile k runs its column phase and stores,
// the data of tile k+1 streams into the staging buffer and the descriptors
// of tile k+2 into the descriptor staging slot; the tile records of k+2 are
// read (plain loads) right after tile k's stores.  One vmcnt(0) wait and
// barrier at the head of each tile publishes all of it.
//
// Staging layout: the tile's rows in order (row = b * H + r), in 16-byte
// units (4-byte units for 4-wide blocks), so one wave's loads cover whole
// rows; the units of a row are XOR-permuted by swz(row) so that the wide
// LDS reads of the forward row phase (thread = row) fall in distinct banks
// for 8- and 16-unit bank periods alike.
using lds_void = __attribute__((address_space(3))) void;
constexpr int kStageDwords = 4096;             // the largest tile: 8192 halfwords

constexpr bool tile_stage_fits() {
  for (int lw = 2; lw <= 6; ++lw)
    for (int lh = 2; lh <= 6; ++lh) {
      const int elems = BatchGeo::nb_for(lw, lh) << (lw + lh);
      if (elems > 2 * kStageDwords) return false;
      if (lw == 2 && elems / 2 > 512) return false;      // two rounds of 4-byte units
      if (lw >= 3 && elems / 8 > 1024) return false;     // four rounds of 16-byte units
      if ((BatchGeo::nb_for(lw, lh) << lh) > 256) return false;   // one thread per row
    }
  return true;
}
static_assert(tile_stage_fits(), "a tile does not fit the staging buffer");
static_assert(kMaxTileBlocks * sizeof(ta_block) <= 256 * 16, "descriptor staging: one 16-byte unit per thread");

TA_DEV int swz(int row, int lcpr) { return ((row >> (4 - lcpr)) ^ (row >> (3 - lcpr))) & ((1 << lcpr) - 1); }

TA_DEV void dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

// The thread index, opaque to the compiler: addresses derived from it are
// computed where they are used instead of being hoisted out of the tile
// loop and spilled (a spill reload waits on vmcnt, that is, on the loads
// in flight into LDS).
TA_DEV int tid_here() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// What the loads of a tile need: its size, block count and first block.
// Tile records are read through the constant address space (the kernel
// never writes them): scalar loads, counted apart from the vector loads and
// stores, so fetching the next record waits on neither.
struct TileHead {
  int lw, lh, count;
  int64_t first;
};

typedef const __attribute__((address_space(4))) uint32_t* ConstWords;

TA_DEV TileHead tile_head(const BatchTile* p) {
  const ConstWords w = (ConstWords)p;
  static_assert(offsetof(BatchTile, lw) == 0 && offsetof(BatchTile, lh) == 4 && offsetof(BatchTile, first) == 16 &&
                    offsetof(BatchTile, count) == 24, "tile record layout");
  const uint32_t lo = __builtin_amdgcn_readfirstlane(w[4]), hi = __builtin_amdgcn_readfirstlane(w[5]);
  return TileHead{__builtin_amdgcn_readfirstlane((int)w[0]), __builtin_amdgcn_readfirstlane((int)w[1]),
                  __builtin_amdgcn_readfirstlane((int)w[6]), (int64_t)(((uint64_t)hi << 32) | lo)};
}
TA_DEV TileHead tile_head(const BatchTile& t) { return TileHead{t.lw, t.lh, t.count, t.first}; }
TA_DEV BatchTile uniform_tile(const BatchTile* p) {
  const ConstWords w = (ConstWords)p;
  BatchTile t;
  uint32_t* d = reinterpret_cast<uint32_t*>(&t);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(BatchTile) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(w[i]);
  return t;
}

// descriptors of tile t -> dst (2 units of 16 bytes per block)
TA_DEV void stage_descs(const BatchArgs& a, const TileHead& t, ta_block* dst) {
  const int s = tid_here(), base = s & ~63;
  if (s < 2 * t.count)
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint4*>(a.blocks + t.first) + s,
                                     (lds_void*)(reinterpret_cast<uint4*>(dst) + base), 16, 0, 0);
}

// data of tile t -> stage, through its descriptors dl (in LDS)
TA_DEV void stage_data(const BatchArgs& a, const TileHead& t, const ta_block* dl, uint32_t* stage) {
  const int tx = tid_here(), wb = tx & ~63, lane = tx & 63;
  const int hm = (1 << t.lh) - 1;
  if (t.lw >= 3) {
    const int lcpr = t.lw - 3, nu = t.count << (t.lh + lcpr);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int base = g * 256 + wb, s = base + lane;
      if (s < nu) {
        const int row = s >> lcpr;
        const int c = (s & ((1 << lcpr) - 1)) ^ swz(row, lcpr);
        const ta_block& d = dl[row >> t.lh];
        const int16_t* src = a.in + d.in_off + (int64_t)(row & hm) * d.in_stride + c * 8;
        __builtin_amdgcn_global_load_lds(src, (lds_void*)(stage + base * 4), 16, 0, 0);
      }
    }
  } else {
    const int nu = t.count << (t.lh + 1);
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int base = g * 256 + wb, s = base + lane;
      if (s < nu) {
        const int row = s >> 1;
        const ta_block& d = dl[row >> t.lh];
        const int16_t* src = a.in + d.in_off + (int64_t)(row & hm) * d.in_stride + (s & 1) * 2;
        __builtin_amdgcn_global_load_lds(src, (lds_void*)(stage + base), 4, 0, 0);
      }
    }
  }
}

TA_DEV void copy_descs(const TileHead& t, const ta_block* src, ta_block* dst) {
  const int tx = tid_here();
  if (tx < 2 * t.count) reinterpret_cast<uint4*>(dst)[tx] = reinterpret_cast<const uint4*>(src)[tx];
}

// forward row phase from the staged rows
template <int W, class KH>
TA_DEV void fwd_rows_st(const BatchArgs& a, const BatchTile& t, const uint32_t* stage, uint16_t* pch, int s_row) {
  const int tid = tid_here();
  if (tid >= (t.count << t.lh)) return;
  const int b = tid >> t.lh, r = tid & ((1 << t.lh) - 1);
  fx::Packed<W> x;
  if constexpr (W >= 8) {
    constexpr int LC = W == 8 ? 0 : W == 16 ? 1 : W == 32 ? 2 : 3;
    const uint4* row = reinterpret_cast<const uint4*>(stage) + (tid << LC);
    const int f = swz(tid, LC);
#pragma unroll
    for (int q = 0; q < W / 8; ++q) {
      const uint4 v = row[q ^ f];
      x.p[4 * q] = v.x; x.p[4 * q + 1] = v.y; x.p[4 * q + 2] = v.z; x.p[4 * q + 3] = v.w;
    }
  } else {
    const uint2 v = reinterpret_cast<const uint2*>(stage)[tid];
    x.p[0] = v.x; x.p[1] = v.y;
  }
  const auto y = fx::run_pass<W, KH, false>(x, as_cparam(t.ph_f), as_cparam(t.ph_i), s_row, a.a);
  const int base = ((r >> 1) * BatchGeo::pc_pitch(t.lh) + b * W) * 2 + (r & 1);
#pragma unroll
  for (int j = 0; j < W / 2; ++j) {
    const uint32_t v = y.pair(2 * j, 2 * j + 1);
    pch[base + (2 * j) * 2] = (uint16_t)v;
    pch[base + (2 * j + 1) * 2] = (uint16_t)(v >> 16);
  }
}

template <class KH>
TA_DEV void fwd_rows_st_w(const BatchArgs& a, const BatchTile& t, const uint32_t* stage, uint16_t* pch, int s) {
  switch (t.lw) {
    case 2: fwd_rows_st<4, KH>(a, t, stage, pch, s); break;
    case 3: fwd_rows_st<8, KH>(a, t, stage, pch, s); break;
    case 4: fwd_rows_st<16, KH>(a, t, stage, pch, s); break;
    case 5: fwd_rows_st<32, KH>(a, t, stage, pch, s); break;
    default: fwd_rows_st<64, KH>(a, t, stage, pch, s); break;
  }
}

// inverse: the staged rows -> pair-row layout
TA_DEV void inv_scatter(const BatchTile& t, const uint32_t* stage, uint16_t* pch) {
  const int p = BatchGeo::pc_pitch(t.lh), hm = (1 << t.lh) - 1, tx = tid_here();
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
        const int base = ((r >> 1) * p + ((row >> t.lh) << t.lw) + c0) * 2 + (r & 1);
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
    for (int g = 0; g < 2; ++g) {
      const int s = tx + 256 * g;
      if (s < nu) {
        const uint32_t v = stage[s];
        const int row = s >> 1, r = row & hm;
        const int base = ((r >> 1) * p + ((row >> t.lh) << 2) + (s & 1) * 2) * 2 + (r & 1);
        pch[base] = (uint16_t)v;
        pch[base + 2] = (uint16_t)(v >> 16);
      }
    }
  }
}

// coalesced store of the row-major layout through the descriptors dl (LDS);
// a tile has at most 1024 chunks: four rounds, the LDS reads issued first
TA_DEV void store_tile(const BatchArgs& a, const BatchTile& t, const uint16_t* rm, const ta_block* dl) {
  const int lch = t.lw >= 3 ? 3 : 2, tx = tid_here();
  const int q = BatchGeo::rm_pitch(t.lh);
  const int nch = t.count << (t.lw + t.lh - lch);
  uint4 v[4];
  int64_t off[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int ch = tx + 256 * g;
    if (ch < nch) {
      const Chunk k(ch, t.lw, t.lh, lch);
      const ta_block& d = dl[k.b];
      off[g] = d.out_off + (int64_t)k.r * d.out_stride + k.c0;
      const uint16_t* src = rm + k.r * q + (k.b << t.lw) + k.c0;
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
    const int ch = tx + 256 * g;
    if (ch < nch) {
      if (lch == 3)
        *reinterpret_cast<uint4*>(a.out + off[g]) = v[g];
      else
        *reinterpret_cast<uint2*>(a.out + off[g]) = make_uint2(v[g].x, v[g].y);
    }
  }
}

// The walk of one workgroup over its XCD's tile list (grid stride P):
// tile k is processed while the data of k+1 and the descriptors of k+2 load.
template <bool INV>
TA_DEV void planned_tiles(const BatchArgs& a, uint32_t* lds, uint32_t* stage, ta_block (*ring)[kMaxTileBlocks],
                          ta_block* dnext) {
  const int xcd = blockIdx.x % kXcds;
  const int64_t P = (gridDim.x + kXcds - 1 - xcd) / kXcds;
  const int64_t end = a.xstart[xcd + 1];
  int64_t ti = a.xstart[xcd] + blockIdx.x / kXcds;
  if (ti >= end) return;
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  BatchTile t = uniform_tile(a.tiles + ti);
  bool has_n = ti + P < end, has_nn = ti + 2 * P < end;
  TileHead n = has_n ? tile_head(a.tiles + ti + P) : tile_head(t);
  stage_descs(a, tile_head(t), ring[0]);
  dma_wait();
  tile_sync();
  stage_data(a, tile_head(t), ring[0], stage);
  if (has_n) stage_descs(a, n, dnext);
  TileHead nn = has_nn ? tile_head(a.tiles + ti + 2 * P) : n;
  int cur = 0;
  for (;;) {
    dma_wait();                          // this tile's data, the next descriptors, the last stores
    tile_sync();
    if (has_n) copy_descs(n, dnext, ring[cur ^ 1]);
    if (INV) {
      inv_scatter(t, stage, pch);
    } else {
      const int s_row = t.lw + a.bd + a.m - 15;
      switch (t.kind_h) {
        case 0: fwd_rows_st_w<KC2>(a, t, stage, pch, s_row); break;
        case 1: fwd_rows_st_w<KS3>(a, t, stage, pch, s_row); break;
        default: fwd_rows_st_w<KC3>(a, t, stage, pch, s_row); break;
      }
    }
    tile_sync();                         // stage and dnext are free
    if (has_n) stage_data(a, n, ring[cur ^ 1], stage);
    if (has_nn) stage_descs(a, nn, dnext);
    if (INV) {
      const int s_col = a.m + 1, s_row = a.m + 14 - a.bd;
      switch (t.kind_v) {
        case 0: inv_cols_h<KC2>(a, t, lds, s_col); break;
        case 1: inv_cols_h<KS3>(a, t, lds, s_col); break;
        default: inv_cols_h<KC3>(a, t, lds, s_col); break;
      }
      tile_sync();
      switch (t.kind_h) {
        case 0: inv_rows_w<KC2>(a, t, pch, s_row); break;
        case 1: inv_rows_w<KS3>(a, t, pch, s_row); break;
        default: inv_rows_w<KC3>(a, t, pch, s_row); break;
      }
    } else {
      const int s_col = t.lh + a.m;
      switch (t.kind_v) {
        case 0: fwd_cols_h<KC2>(a, t, lds, s_col); break;
        case 1: fwd_cols_h<KS3>(a, t, lds, s_col); break;
        default: fwd_cols_h<KC3>(a, t, lds, s_col); break;
      }
    }
    tile_sync();
    store_tile(a, t, pch, ring[cur]);
    if (!has_n) break;
    ti += P;
    t = uniform_tile(a.tiles + ti);
    n = nn;
    has_n = has_nn;
    has_nn = ti + 2 * P < end;
    if (has_nn) nn = tile_head(a.tiles + ti + 2 * P);
    cur ^= 1;
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_fwd(BatchArgs a) {
  __shared__ __align__(16) uint32_t lds[kBatchLds];
  __shared__ __align__(16) uint32_t stage[kStageDwords];
  __shared__ __align__(16) ta_block ring[2][kMaxTileBlocks];
  __shared__ __align__(16) ta_block dnext[kMaxTileBlocks];
  planned_tiles<false>(a, lds, stage, ring, dnext);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_inv(BatchArgs a) {
  __shared__ __align__(16) uint32_t lds[kBatchLds];
  __shared__ __align__(16) uint32_t stage[kStageDwords];
  __shared__ __align__(16) ta_block ring[2][kMaxTileBlocks];
  __shared__ __align__(16) ta_block dnext[kMaxTileBlocks];
  planned_tiles<true>(a, lds, stage, ring, dnext);
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

// forward row phase: global row -> transform -> column-major LDS
template <int W, class KH>
TA_DEV void fwd_rows_f(const BatchArgs& a, const BatchTile& t, const ta_block* blocks, float* lds, BDesc* desc) {
  const int tid = threadIdx.x;
  if (tid >= (t.count << t.lh)) return;
  const int b = tid >> t.lh, r = tid & ((1 << t.lh) - 1), h1 = (1 << t.lh) + 1;
  const ta_block d = blocks[t.first + b];
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
    const ta_block d = blocks[t.first + threadIdx.x];
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
  const int64_t end = a.xstart[xcd + 1];
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
TA_DEV int config_key(const BatchArgs& a, const ta_block& d) {
  const int ch = d.log2w >= 3 ? 8 : 4;                  // elements per vector access
  if (d.log2w < 2 || d.log2w > 6 || d.log2h < 2 || d.log2h > 6 || d.in_off < 0 || d.out_off < 0 ||
      d.in_stride < (1 << d.log2w) || d.out_stride < (1 << d.log2w) || d.axis_h >= kAxisIds ||
      d.axis_v >= kAxisIds || ((d.in_off | d.out_off | (int64_t)d.in_stride | (int64_t)d.out_stride) & (ch - 1)))
    return -1;
  if (a.axes[d.axis_h * kAxisSizes + d.log2w].kind < 0 || a.axes[d.axis_v * kAxisSizes + d.log2h].kind < 0) return -1;
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
        const int k = config_key(a, a.blocks[w0 + i]);
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

}  // namespace ta
