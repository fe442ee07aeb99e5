// Batched uneven blocks: one persistent launch over a planned list of tiles.
//
// The host planner groups blocks by (W, H, horizontal kind, vertical kind)
// and cuts the groups into tiles of NB = 256 / max(W, H) blocks.  Each
// workgroup walks the tile list with a grid stride.  Within a tile the
// forward runs the same phases as the packed kernels (rows -> pair-column
// LDS -> columns -> row-major LDS -> coalesced stores), but block addresses
// come from the block descriptors (offsets and row strides into frame
// buffers) and the block size and kinds are wave-uniform runtime values:
// the row phase dispatches on (W, row kind), the column phase on (H, column
// kind), so the kernel holds 15 row bodies and 15 column bodies per
// direction rather than one body per (W, H, kind, kind).
//
// Kinds: 0 = DCT-2, 1 = DST-3 + 4-tap band (adjusted DST-7),
//        2 = DCT-3 + 4-tap band with flipped taps (adjusted DCT-8, eq. 3).
#include "fx.hpp"
#include "kernels.hpp"

namespace ta {

// One tile of the plan (device memory, written by the host planner).


namespace {

using fx::Axis;
using KC2 = Axis<C_DCT2, ADJ_NONE, 0>;
using KS3 = Axis<C_DST3, ADJ_BAND, 4>;
using KC3 = Axis<C_DCT3, ADJ_BAND, 4>;

// LDS of the largest tile (dwords); every tile fits 20 KiB
constexpr int max_tile_lds() {
  int m = 0;
  for (int lw = 2; lw <= 6; ++lw)
    for (int lh = 2; lh <= 6; ++lh) {
      const int nb = BatchGeo::nb_for(lw, lh);
      const int v = BatchGeo::lds_bytes(1 << lw, 1 << lh, nb, BatchGeo::pad_for(lw, lh));
      m = v > m ? v : m;
    }
  return (m + 3) / 4;
}
constexpr int kBatchLds = max_tile_lds();
static_assert(kBatchLds * 4 <= BatchGeo::kLdsBytes, "tile LDS above 20 KiB");
using Geo = BatchGeo;

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
// row phase of one tile for kind KH at width W
template <int W, class KH>
TA_DEV void fwd_rows(const BatchArgs& a, const BatchTile& t, const Geo& g, uint16_t* pch, int s_row) {
  const int tid = threadIdx.x;
  if (tid >= t.count * g.H) return;
  const int b = tid / g.H, r = tid % g.H;
  const ta_block d = a.blocks[t.first + b];
  fx::Packed<W> x;
  load_strided_row<W>(a.in + d.in_off + (int64_t)r * d.in_stride, x);
  const auto y = fx::run_pass<W, KH, false>(x, as_cparam(t.ph_f), as_cparam(t.ph_i), s_row, a.a);
  const int base = (b * g.PCB + (r >> 1) * g.PP) * 2 + (r & 1);
#pragma unroll
  for (int j = 0; j < W / 2; ++j) {
    const uint32_t v = y.pair(2 * j, 2 * j + 1);
    pch[base + (2 * j) * 2] = (uint16_t)v;
    pch[base + (2 * j + 1) * 2] = (uint16_t)(v >> 16);
  }
}

// column phase: read PC, transform, barrier (PC dead), write RM (pitch W)
template <int H, class KV>
TA_DEV void fwd_cols(const BatchArgs& a, const BatchTile& t, const Geo& g, uint32_t* lds, int s_col) {
  const int tid = threadIdx.x;
  const bool act = tid < t.count * g.W;
  const int b = act ? tid / g.W : 0, c = act ? tid % g.W : 0;
  uint32_t o[H / 2];
  if (act) {
    fx::Packed<H> z;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) z.p[i] = lds[b * g.PCB + i * g.PP + c];
    const auto y = fx::run_pass<H, KV, false>(z, as_cparam(t.pv_f), as_cparam(t.pv_i), s_col, a.a);
#pragma unroll
    for (int i = 0; i < H / 2; ++i) o[i] = y.pair(2 * i, 2 * i + 1);
  }
  __syncthreads();
  if (act) {
    uint16_t* rm = reinterpret_cast<uint16_t*>(lds);
    const int base = b * g.RMBF + c;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) {
      rm[base + (2 * i) * g.W] = (uint16_t)o[i];
      rm[base + (2 * i + 1) * g.W] = (uint16_t)(o[i] >> 16);
    }
  }
}

template <class KH>
TA_DEV void fwd_rows_w(const BatchArgs& a, const BatchTile& t, const Geo& g, uint16_t* pch, int s) {
  switch (t.lw) {
    case 2: fwd_rows<4, KH>(a, t, g, pch, s); break;
    case 3: fwd_rows<8, KH>(a, t, g, pch, s); break;
    case 4: fwd_rows<16, KH>(a, t, g, pch, s); break;
    case 5: fwd_rows<32, KH>(a, t, g, pch, s); break;
    default: fwd_rows<64, KH>(a, t, g, pch, s); break;
  }
}

template <class KV>
TA_DEV void fwd_cols_h(const BatchArgs& a, const BatchTile& t, const Geo& g, uint32_t* lds, int s) {
  switch (t.lh) {
    case 2: fwd_cols<4, KV>(a, t, g, lds, s); break;
    case 3: fwd_cols<8, KV>(a, t, g, lds, s); break;
    case 4: fwd_cols<16, KV>(a, t, g, lds, s); break;
    case 5: fwd_cols<32, KV>(a, t, g, lds, s); break;
    default: fwd_cols<64, KV>(a, t, g, lds, s); break;
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_fwd(BatchArgs a) {
  __shared__ __align__(16) uint32_t lds[kBatchLds];
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  // this workgroup's XCD list and its stride within that list
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = (gridDim.x + kXcds - 1 - xcd) / kXcds;
  const int64_t end = a.xstart[xcd + 1];
  for (int64_t ti = a.xstart[xcd] + blockIdx.x / kXcds; ti < end; ti += per_xcd) {
    const BatchTile t = a.tiles[ti];
    const Geo g(t.lw, t.lh);
    const int s_row = t.lw + a.bd + a.m - 15, s_col = t.lh + a.m;
    switch (t.kind_h) {
      case 0: fwd_rows_w<KC2>(a, t, g, pch, s_row); break;
      case 1: fwd_rows_w<KS3>(a, t, g, pch, s_row); break;
      default: fwd_rows_w<KC3>(a, t, g, pch, s_row); break;
    }
    __syncthreads();
    switch (t.kind_v) {
      case 0: fwd_cols_h<KC2>(a, t, g, lds, s_col); break;
      case 1: fwd_cols_h<KS3>(a, t, g, lds, s_col); break;
      default: fwd_cols_h<KC3>(a, t, g, lds, s_col); break;
    }
    __syncthreads();
    // coalesced store of the tile (RM pitch W, chunks of CH halfwords)
    const int rmb = g.RMBF;
    const int cpr = g.W / g.CH, cpb = g.H * cpr;
    const int nch = t.count * cpb;
    for (int c = threadIdx.x; c < nch; c += 256) {
      const int b = c / cpb, q = c % cpb, r = q / cpr, c0 = (q % cpr) * g.CH;
      const ta_block d = a.blocks[t.first + b];
      int16_t* dst = a.out + d.out_off + (int64_t)r * d.out_stride + c0;
      const uint16_t* src = pch + b * rmb + r * g.W + c0;
      if (g.CH == 8)
        *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(src);
      else
        *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(src);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- inverse
template <int H, class KV>
TA_DEV void inv_cols(const BatchArgs& a, const BatchTile& t, const Geo& g, uint32_t* lds, int s_col) {
  const int tid = threadIdx.x;
  const bool act = tid < t.count * g.W;
  const int b = act ? tid / g.W : 0, c = act ? tid % g.W : 0;
  uint32_t o[H / 2];
  if (act) {
    fx::Packed<H> z;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) z.p[i] = lds[b * g.PCB + i * g.PP + c];
    const auto y = fx::run_pass<H, KV, true>(z, as_cparam(t.pv_f), as_cparam(t.pv_i), s_col, a.a);
#pragma unroll
    for (int i = 0; i < H / 2; ++i) o[i] = y.pair(2 * i, 2 * i + 1);
  }
  __syncthreads();
  if (act) {
    uint16_t* rm = reinterpret_cast<uint16_t*>(lds);
    const int base = b * g.RMB + c;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) {
      rm[base + (2 * i) * g.RP] = (uint16_t)o[i];
      rm[base + (2 * i + 1) * g.RP] = (uint16_t)(o[i] >> 16);
    }
  }
}

template <int W, class KH>
TA_DEV void inv_rows(const BatchArgs& a, const BatchTile& t, const Geo& g, const uint16_t* rm, int s_row) {
  const int tid = threadIdx.x;
  if (tid >= t.count * g.H) return;
  const int b = tid / g.H, r = tid % g.H;
  fx::Packed<W> x;
  const uint16_t* s = rm + b * g.RMB + r * g.RP;
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
  const ta_block d = a.blocks[t.first + b];
  int16_t* dst = a.out + d.out_off + (int64_t)r * d.out_stride;
  uint32_t o[W / 2];
#pragma unroll
  for (int j = 0; j < W / 2; ++j) o[j] = y.pair(2 * j, 2 * j + 1);
  if constexpr (W >= 8) {
#pragma unroll
    for (int q = 0; q < W / 8; ++q)
      reinterpret_cast<uint4*>(dst)[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
  } else {
    *reinterpret_cast<uint2*>(dst) = make_uint2(o[0], o[1]);
  }
}

template <class KV>
TA_DEV void inv_cols_h(const BatchArgs& a, const BatchTile& t, const Geo& g, uint32_t* lds, int s) {
  switch (t.lh) {
    case 2: inv_cols<4, KV>(a, t, g, lds, s); break;
    case 3: inv_cols<8, KV>(a, t, g, lds, s); break;
    case 4: inv_cols<16, KV>(a, t, g, lds, s); break;
    case 5: inv_cols<32, KV>(a, t, g, lds, s); break;
    default: inv_cols<64, KV>(a, t, g, lds, s); break;
  }
}

template <class KH>
TA_DEV void inv_rows_w(const BatchArgs& a, const BatchTile& t, const Geo& g, const uint16_t* rm, int s) {
  switch (t.lw) {
    case 2: inv_rows<4, KH>(a, t, g, rm, s); break;
    case 3: inv_rows<8, KH>(a, t, g, rm, s); break;
    case 4: inv_rows<16, KH>(a, t, g, rm, s); break;
    case 5: inv_rows<32, KH>(a, t, g, rm, s); break;
    default: inv_rows<64, KH>(a, t, g, rm, s); break;
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_inv(BatchArgs a) {
  __shared__ __align__(16) uint32_t lds[kBatchLds];
  uint16_t* pch = reinterpret_cast<uint16_t*>(lds);
  // this workgroup's XCD list and its stride within that list
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = (gridDim.x + kXcds - 1 - xcd) / kXcds;
  const int64_t end = a.xstart[xcd + 1];
  for (int64_t ti = a.xstart[xcd] + blockIdx.x / kXcds; ti < end; ti += per_xcd) {
    const BatchTile t = a.tiles[ti];
    const Geo g(t.lw, t.lh);
    const int s_col = a.m + 1, s_row = a.m + 14 - a.bd;
    // coalesced load of the tile into the pair-column layout
    const int cpr = g.W / g.CH, cpb = g.H * cpr;
    const int nch = t.count * cpb;
    for (int c = threadIdx.x; c < nch; c += 256) {
      const int b = c / cpb, q = c % cpb, r = q / cpr, c0 = (q % cpr) * g.CH;
      const ta_block d = a.blocks[t.first + b];
      const int16_t* src = a.in + d.in_off + (int64_t)r * d.in_stride + c0;
      uint32_t w[4];
      if (g.CH == 8) {
        const uint4 v = *reinterpret_cast<const uint4*>(src);
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
      } else {
        const uint2 v = *reinterpret_cast<const uint2*>(src);
        w[0] = v.x; w[1] = v.y; w[2] = 0; w[3] = 0;
      }
      const int base = (b * g.PCB + (r >> 1) * g.PP + c0) * 2 + (r & 1);
      for (int k = 0; k < g.CH / 2; ++k) {
        pch[base + (2 * k) * 2] = (uint16_t)w[k];
        pch[base + (2 * k + 1) * 2] = (uint16_t)(w[k] >> 16);
      }
    }
    __syncthreads();
    switch (t.kind_v) {
      case 0: inv_cols_h<KC2>(a, t, g, lds, s_col); break;
      case 1: inv_cols_h<KS3>(a, t, g, lds, s_col); break;
      default: inv_cols_h<KC3>(a, t, g, lds, s_col); break;
    }
    __syncthreads();
    switch (t.kind_h) {
      case 0: inv_rows_w<KC2>(a, t, g, pch, s_row); break;
      case 1: inv_rows_w<KS3>(a, t, g, pch, s_row); break;
      default: inv_rows_w<KC3>(a, t, g, pch, s_row); break;
    }
    __syncthreads();
  }
}

}  // namespace

const void* batch_kernel(int inv) {
  return inv ? reinterpret_cast<const void*>(&batch_inv) : reinterpret_cast<const void*>(&batch_fwd);
}

}  // namespace ta
