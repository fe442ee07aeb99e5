// General block transforms: every axis kind of the library, in block lists
// (planned or unplanned) and in packed batches without a specialised kernel.
//
// An axis is a program of at most two 1-D stages (GenProg, built by the host
// from the registered axis: the core kind after the DCT-8 flip, the band or
// sub-block tables in the orientation of the direction).  A tile holds NB
// blocks of one size W x H; one kernel serves both directions:
//   load   coalesced 16-byte (int16) or float4 (fp32) chunks of every block
//          into LDS, row-major, row pitch RP (GenGeo)
//   pass 1 forward: every row by the horizontal program; inverse: every
//          column by the vertical program (one vector per thread, updated in
//          place)
//   pass 2 the other axis
//   store  coalesced chunks back out.
// Stages are wave-uniform runtime choices (the tile's program); each is a
// compile-time body per vector length, and the two passes share one call
// site per length.  The stages are those of the specialised kernels
// (fx.hpp, fp.hpp): the butterfly cores, the K-tap band and the B x B
// sub-block, plus a dense N x N product for the direct DST-7 / DCT-8 and for
// sub-blocks of a side without a compiled stage.  Fixed point is exact (the
// same integers as every other kernel); fp32 has no rounding.
#include "gen.hpp"
#include "window_sort.hpp"

namespace ta {
namespace {

using gen::vec_f;
using gen::vec_fx;

// Offsets and strides of the blocks of the current tile (in LDS).
struct GDesc {
  int64_t in_off, out_off;
  int32_t in_stride, out_stride;
};
constexpr int kGenMaxBlocks = 64;

// ---------------------------------------------------------------- one tile
// Where the blocks of a tile are: descriptors (first + b), or a packed batch
// (block first + b at (first + b) * W * H, row stride W).
TA_DEV GDesc tile_desc(const ta_block* blocks, int64_t idx, int lw, int lh) {
  if (blocks) {
    const ta_block d = blocks[idx];
    return GDesc{d.in_off, d.out_off, d.in_stride, d.out_stride};
  }
  const int64_t off = idx << (lw + lh);
  return GDesc{off, off, 1 << lw, 1 << lw};
}

// One tile: NB blocks of 2^lw x 2^lh at descriptors first..first+count-1,
// programs ph (rows) and pv (columns) of the launch direction.  Ends with a
// barrier (LDS free for the next tile).
template <bool F32>
TA_DEV void gen_tile(const GenArgs& a, const ta_block* blocks, int64_t first, int lw, int lh, int count,
                     const GenProg* ph, const GenProg* pv, void* lds_raw, GDesc* desc) {
  const int tid = threadIdx.x;
  const int w = 1 << lw;
  const int rp = GenGeo::rp(lw, F32), bs = GenGeo::bs(lw, lh, F32);
  if (tid < count) desc[tid] = tile_desc(blocks, first + tid, lw, lh);
  __syncthreads();
  // coalesced load: chunks of 8 halfwords / 4 floats (4 halfwords for 4-wide int16 rows)
  const int lch = F32 ? 2 : (lw >= 3 ? 3 : 2);
  const int lq = lw - lch;                             // log2 chunks per row
  const int nch = count << (lh + lq);
  // groups of 4 chunks per thread: the group's loads are issued together
  // before any is written to LDS
  for (int ch0 = tid; ch0 < nch; ch0 += 1024) {
    uint4 v[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int ch = ch0 + 256 * g;
      if (ch < nch) {
        const int b = ch >> (lh + lq), r = (ch >> lq) & ((1 << lh) - 1), c0 = (ch & ((1 << lq) - 1)) << lch;
        const GDesc d = desc[b];
        if constexpr (F32) {
          const float4 f = *reinterpret_cast<const float4*>(static_cast<const float*>(a.in) + d.in_off +
                                                            (int64_t)r * d.in_stride + c0);
          v[g] = make_uint4(__float_as_uint(f.x), __float_as_uint(f.y), __float_as_uint(f.z), __float_as_uint(f.w));
        } else {
          const int16_t* src = static_cast<const int16_t*>(a.in) + d.in_off + (int64_t)r * d.in_stride + c0;
          if (lch == 3) {
            v[g] = *reinterpret_cast<const uint4*>(src);
          } else {
            const uint2 h = *reinterpret_cast<const uint2*>(src);
            v[g] = make_uint4(h.x, h.y, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int ch = ch0 + 256 * g;
      if (ch < nch) {
        const int b = ch >> (lh + lq), r = (ch >> lq) & ((1 << lh) - 1), c0 = (ch & ((1 << lq) - 1)) << lch;
        if constexpr (F32) {
          float* dst = static_cast<float*>(lds_raw) + b * bs + r * rp + c0;
          dst[0] = __uint_as_float(v[g].x); dst[1] = __uint_as_float(v[g].y);
          dst[2] = __uint_as_float(v[g].z); dst[3] = __uint_as_float(v[g].w);
        } else {
          uint32_t* dst = reinterpret_cast<uint32_t*>(static_cast<uint16_t*>(lds_raw) + b * bs + r * rp + c0);
          dst[0] = v[g].x; dst[1] = v[g].y;
          if (lch == 3) { dst[2] = v[g].z; dst[3] = v[g].w; }
        }
      }
    }
  }
  __syncthreads();
  // two passes: forward rows then columns, inverse columns then rows
  const int s_row = a.inv ? a.m + 14 - a.bd : lw + a.bd + a.m - 15;
  const int s_col = a.inv ? a.m + 1 : lh + a.m;
#pragma unroll 1
  for (int ps = 0; ps < 2; ++ps) {
    const bool rows = (ps == 0) == (a.inv == 0);
    const int nlog = rows ? lw : lh;
    const int nvec = count << (rows ? lh : lw);
    if (tid < nvec) {
      const int b = tid >> (rows ? lh : lw), i = tid & ((1 << (rows ? lh : lw)) - 1);
      const int base = b * bs + (rows ? i * rp : i);
      const int stride = rows ? 1 : rp;
      const GenProg* pr = rows ? ph : pv;
      const int sc = rows ? s_row : s_col;
      if constexpr (F32) {
        float* l = static_cast<float*>(lds_raw);
        switch (nlog) {
          case 2: vec_f<4>(l, base, stride, pr); break;
          case 3: vec_f<8>(l, base, stride, pr); break;
          case 4: vec_f<16>(l, base, stride, pr); break;
          case 5: vec_f<32>(l, base, stride, pr); break;
          default: vec_f<64>(l, base, stride, pr); break;
        }
      } else {
        uint16_t* l = static_cast<uint16_t*>(lds_raw);
        switch (nlog) {
          case 2: vec_fx<4>(l, base, stride, pr, sc, a.a); break;
          case 3: vec_fx<8>(l, base, stride, pr, sc, a.a); break;
          case 4: vec_fx<16>(l, base, stride, pr, sc, a.a); break;
          case 5: vec_fx<32>(l, base, stride, pr, sc, a.a); break;
          default: vec_fx<64>(l, base, stride, pr, sc, a.a); break;
        }
      }
    }
    __syncthreads();
  }
  // coalesced store
  for (int ch = tid; ch < nch; ch += 256) {
    const int b = ch >> (lh + lq), r = (ch >> lq) & ((1 << lh) - 1), c0 = (ch & ((1 << lq) - 1)) << lch;
    const GDesc d = desc[b];
    if constexpr (F32) {
      const float* s = static_cast<const float*>(lds_raw) + b * bs + r * rp + c0;
      *reinterpret_cast<float4*>(static_cast<float*>(a.out) + d.out_off + (int64_t)r * d.out_stride + c0) =
          make_float4(s[0], s[1], s[2], s[3]);
    } else {
      const uint32_t* s = reinterpret_cast<const uint32_t*>(static_cast<const uint16_t*>(lds_raw) + b * bs + r * rp + c0);
      int16_t* dst = static_cast<int16_t*>(a.out) + d.out_off + (int64_t)r * d.out_stride + c0;
      if (lch == 3)
        *reinterpret_cast<uint4*>(dst) = make_uint4(s[0], s[1], s[2], s[3]);
      else
        *reinterpret_cast<uint2*>(dst) = make_uint2(s[0], s[1]);
    }
  }
  __syncthreads();
}

constexpr int lds_dwords(bool f32) { return f32 ? kGenLdsF32 : kGenLdsI16 / 2; }

// Planned tile lists (one per XCD, walked with a grid stride by the
// workgroups of that XCD), or a packed batch (tiles == null): tile t holds
// blocks t * NB .. t * NB + NB - 1, walked with a grid stride.
template <bool F32>
__global__ __launch_bounds__(256) void gen_plan(GenArgs a) {
  __shared__ __align__(16) uint32_t lds[lds_dwords(F32)];
  __shared__ GDesc desc[kGenMaxBlocks];
  if (a.tiles) {
    const int xcd = blockIdx.x % kXcds;
    const int64_t per_xcd = (gridDim.x + kXcds - 1 - xcd) / kXcds;
    const int64_t end = a.xstart[xcd + 1];
    for (int64_t ti = a.xstart[xcd] + blockIdx.x / kXcds; ti < end; ti += per_xcd) {
      const BatchTile t = a.tiles[ti];
      const GenProg* ph = reinterpret_cast<const GenProg*>(a.inv ? t.ph_i : t.ph_f);
      const GenProg* pv = reinterpret_cast<const GenProg*>(a.inv ? t.pv_i : t.pv_f);
      gen_tile<F32>(a, a.blocks, t.first, t.lw, t.lh, t.count, ph, pv, lds, desc);
    }
  } else {
    const int nb = GenGeo::nb_for(a.lw, a.lh, F32);
    const int64_t ntiles = (a.nblocks + nb - 1) / nb;
    for (int64_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
      const int64_t first = ti * nb;
      const int count = (int)min<int64_t>(nb, a.nblocks - first);
      gen_tile<F32>(a, nullptr, first, a.lw, a.lh, count, a.ph, a.pv, lds, desc);
    }
  }
}

// ---------------------------------------------------------------- block lists
// Unplanned descriptors, grouped on the device as in the fast block-list
// kernel (batch_kernels.hip): windows of kSortWin descriptors, each shared by
// kSortQuarters workgroups that sort the whole window by (configuration,
// position) and run their own quarter of it as tiles of equal size and axis
// ids.  A descriptor that breaks a rule the kernel can check (size, offset
// sign and alignment, stride, axis id, no program for the axis at its size)
// sorts last and is skipped, and so is one that the fast block-list kernel
// runs in the same call (both axes of a fast kind, when `fast` is set).
constexpr int kSortWin = kDescWindow * kSortQuarters;

TA_DEV const GenProg* axis_prog(const GenArgs& a, int axis, int lsize, int inv) {
  return a.progs + ((size_t)axis * kAxisSizes + lsize) * 2 + inv;
}

TA_DEV int gen_key(const GenArgs& a, const ta_block& d) {
  const int ch = d.log2w >= 3 ? 8 : 4;
  if (d.log2w < 2 || d.log2w > 6 || d.log2h < 2 || d.log2h > 6 || d.in_off < 0 || d.out_off < 0 ||
      d.in_stride < (1 << d.log2w) || d.out_stride < (1 << d.log2w) || d.axis_h >= kAxisIds ||
      d.axis_v >= kAxisIds || ((d.in_off | d.out_off | (int64_t)d.in_stride | (int64_t)d.out_stride) & (ch - 1)))
    return -1;
  if (axis_prog(a, d.axis_h, d.log2w, a.inv)->nst <= 0 || axis_prog(a, d.axis_v, d.log2h, a.inv)->nst <= 0) return -1;
  if (a.fast && a.fast[d.axis_h * kAxisSizes + d.log2w].kind >= 0 && a.fast[d.axis_v * kAxisSizes + d.log2h].kind >= 0)
    return -1;   // the fast block-list kernel runs this one
  return d.log2w | (d.log2h << 3) | (d.axis_h << 6) | (d.axis_v << 14);
}

template <bool F32>
__global__ __launch_bounds__(256) void gen_desc(GenArgs a) {
  __shared__ __align__(16) uint32_t lds[lds_dwords(F32)];
  __shared__ GDesc desc[kGenMaxBlocks];
  __shared__ uint32_t skey[kSortWin];
  __shared__ ta_block qdesc[kDescWindow];
  constexpr uint32_t kInvalid = ~0u;
  const int tid = threadIdx.x;
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = (gridDim.x + kXcds - 1 - xcd) / kXcds;
  const int64_t nunits = (a.nblocks + kSortWin - 1) / kSortWin * kSortQuarters;
  const int64_t uend = nunits * (xcd + 1) / kXcds;
  for (int64_t u = nunits * xcd / kXcds + blockIdx.x / kXcds; u < uend; u += per_xcd) {
    const int64_t w0 = u / kSortQuarters * kSortWin;
    const int q0 = (int)(u % kSortQuarters) * kDescWindow;
    const int cnt = (int)min<int64_t>(kSortWin, a.nblocks - w0);
#pragma unroll
    for (int r = 0; r < kSortQuarters; ++r) {
      const int i = tid + r * 256;
      uint32_t sk = kInvalid;
      if (i < cnt) {
        const int k = gen_key(a, a.blocks[w0 + i]);
        if (k >= 0) sk = ((uint32_t)k << 10) | (uint32_t)i;
      }
      skey[i] = sk;
    }
    bitonic_sort_window<kSortWin>(skey, tid);
    __syncthreads();
    const int qcnt = min(kDescWindow, cnt - q0);
    if (tid < qcnt && skey[q0 + tid] != kInvalid) qdesc[tid] = a.blocks[w0 + (skey[q0 + tid] & (kSortWin - 1))];
    __syncthreads();
    int j = 0;
    while (j < qcnt) {
      const uint32_t s0 = skey[q0 + j];
      if (s0 == kInvalid) break;
      const uint32_t k = s0 >> 10;
      const int lw = (int)(k & 7), lh = (int)((k >> 3) & 7);
      const int ah = (int)((k >> 6) & 0xff), av = (int)((k >> 14) & 0xff);
      const int cap = GenGeo::nb_for(lw, lh, F32);
      int len = 1;
      while (j + len < qcnt && len < cap && (skey[q0 + j + len] >> 10) == k) ++len;
      gen_tile<F32>(a, qdesc, j, lw, lh, len, axis_prog(a, ah, lw, a.inv), axis_prog(a, av, lh, a.inv), lds, desc);
      j += len;
    }
    __syncthreads();
  }
}

}  // namespace

const void* gen_kernel(int desc, int f32) {
  if (desc)
    return f32 ? reinterpret_cast<const void*>(&gen_desc<true>) : reinterpret_cast<const void*>(&gen_desc<false>);
  return f32 ? reinterpret_cast<const void*>(&gen_plan<true>) : reinterpret_cast<const void*>(&gen_plan<false>);
}

}  // namespace ta
