// Kernel registry shared by the kernel translation units and the C ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tadj.h"

namespace ta {

// Arguments of the packed-batch kernels (fixed point and fp32).
struct PackedArgs {
  const void* in;
  void* out;
  int64_t nblocks;
  const void* ph_f;  // horizontal axis parameters, forward orientation
  const void* ph_i;  // horizontal axis parameters, transposed (inverse)
  const void* pv_f;  // vertical axis parameters
  const void* pv_i;
  int s_row;         // core shift of the row pass (fixed point)
  int s_col;         // core shift of the column pass
  int a;             // adjustment shift
};

// Identifies one compiled kernel: direction, dtype, block size and both axes.
struct KernelKey {
  int inv, dtype, lw, lh;
  int core_h, adj_h, kb_h;
  int core_v, adj_v, kb_v;
  bool operator==(const KernelKey& o) const {
    return inv == o.inv && dtype == o.dtype && lw == o.lw && lh == o.lh && core_h == o.core_h &&
           adj_h == o.adj_h && kb_h == o.kb_h && core_v == o.core_v && adj_v == o.adj_v && kb_v == o.kb_v;
  }
};

struct KernelEntry {
  KernelKey key;
  const void* fn;     // __global__ function
  int blocks_per_wg;  // blocks of the batch handled by one workgroup (per iteration)
  int threads;        // workgroup size
  int max_wgs;        // grid cap: 0 = one workgroup per tile, > 0 a fixed cap,
                      // -1 = persistent, as many as are resident at once
  bool same_params;   // requires the horizontal and vertical parameters to be the same set
};

// One tile of a batched plan (device memory, written by the host planner):
// up to 256 / max(W, H) blocks of one size and one pair of axis kinds.
struct BatchTile {
  int32_t lw, lh, kind_h, kind_v;
  int64_t first;          // index of the first block descriptor of the tile
  int32_t count;          // blocks in this tile
  int32_t pad;
  const uint32_t* ph_f;   // band taps of the horizontal axis (forward / transposed)
  const uint32_t* ph_i;
  const uint32_t* pv_f;   // band taps of the vertical axis
  const uint32_t* pv_i;
};

// The plan's tiles form one list per XCD (8 lists, concatenated; list x is
// tiles[xstart[x] .. xstart[x+1])), ordered region by region, so that the
// workgroups of one XCD (consecutive workgroup ids go to consecutive XCDs)
// process the blocks of the same frame region together and share its L2.
constexpr int kXcds = 8;

struct BatchArgs {
  const BatchTile* tiles;
  int64_t ntiles;
  int64_t xstart[kXcds + 1];
  const ta_block* blocks;
  const int16_t* in;
  int16_t* out;
  int bd, m, a;
};

// Persistent batched kernels over a planned tile list (batch_kernels.hip).
const void* batch_kernel(int inv);

// Differentiable Givens-band path (givens_kernels.hip).
constexpr int kMaxAng = 96;   // angle slots per workgroup partial (N <= 32, L <= 3)
struct GivensArgs {
  const float* theta;
  const float* x;
  const float* gy;
  float* y;
  float* gx;
  float* partial;   // [grid][kMaxAng] per-workgroup angle-gradient partials
  int64_t nvec;
};
const void* givens_kernel(int bwd, int n, int layers, int base);
const void* givens_reduce_kernel();

// Tables of compiled kernels (defined in the kernel translation units).
const KernelEntry* fx_kernels(int* count);
const KernelEntry* f32_kernels(int* count);
const KernelEntry* mfma_kernels(int* count);

}  // namespace ta
