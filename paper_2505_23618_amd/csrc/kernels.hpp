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
// blocks of one size and one pair of axis kinds.  The blocks of a tile share
// their row strides, and each block's offsets are int32 deltas from the
// tile's bases (the planner cuts tiles so that they fit), kept in the plan's
// delta array (in_delta, out_delta per block, in block order).
struct BatchTile {
  int32_t lw, lh, kind_h, kind_v;
  int64_t first;          // index of the first block (descriptors and deltas) of the tile
  int32_t count;          // blocks in this tile
  int32_t in_stride;      // input row stride of every block of the tile
  const uint32_t* ph_f;   // band taps of the horizontal axis (forward / transposed)
  const uint32_t* ph_i;
  const uint32_t* pv_f;   // band taps of the vertical axis
  const uint32_t* pv_i;
  int64_t in_base;        // block b's input at in_base + in_delta[first + b]
  int64_t out_base;
  int32_t out_stride;
  int32_t pad;
};

// The plan's tiles form one list per XCD (8 lists, concatenated; list x is
// tiles[xstart[x] .. xstart[x+1])), ordered region by region, so that the
// workgroups of one XCD (consecutive workgroup ids go to consecutive XCDs)
// process the blocks of the same frame region together and share its L2.
constexpr int kXcds = 8;

// Tile geometry of the batched kernels, shared by the host planner and the
// device code.  A tile holds NB blocks of one size W x H side by side: in
// LDS, pair-row i of the tile (rows 2i, 2i+1 of every block, packed in
// dwords) has pitch PC_PITCH(H) dwords and row r has pitch RM_PITCH(H)
// halfwords, block b starting at column b * W.  With NB * W <= 256 (<= 128
// for H = 64) the pitches depend on H only, so a column thread (index
// b * W + c) finds its values at compile-time offsets from its own index.
// NB = 256 / max(W, H) (one thread per row and per column), capped by the
// column limit.
struct BatchGeo {
  static constexpr int pc_pitch(int lh) { return lh == 6 ? 129 : 257; }
  static constexpr int rm_pitch(int lh) { return lh == 6 ? 136 : 264; }
  static constexpr int nb_for(int lw, int lh) {
    const int nb = 256 >> (lw > lh ? lw : lh);
    const int cap = (lh == 6 ? 128 : 256) >> lw;
    return nb < cap ? nb : cap;
  }
  // LDS of a tile (dwords): the pair-row and row layouts alias one buffer
  static constexpr int lds_dwords(int lh) {
    const int h = 1 << lh;
    const int pc = (h / 2) * pc_pitch(lh), rm = (h * rm_pitch(lh) + 1) / 2;
    return pc > rm ? pc : rm;
  }
  static constexpr int max_lds_dwords() {
    int m = 0;
    for (int lh = 2; lh <= 6; ++lh) m = lds_dwords(lh) > m ? lds_dwords(lh) : m;
    return m;
  }
  // Planned int16 tiles (batch_fwd / batch_inv) are larger: up to 8192
  // coefficients (4096 for 4-wide blocks, whose loads move 4 bytes a lane),
  // the row and column phases looping over their rows and columns.  The
  // tile's columns (NB * W) never exceed 8192 / H, and the pitches are those
  // of that width whatever the tile holds: pl_pc(H) = 8192 / H + 1 dwords
  // (pair rows) and pl_rm(H) = 8192 / H + 8 halfwords (rows), compile-time
  // per H so that a column thread's accesses are immediate offsets.
  static constexpr int kPlannedBlocks = 256;
  static constexpr int nb_planned(int lw, int lh) {
    const int nb = (lw == 2 ? 4096 : 8192) >> (lw + lh);
    return nb < kPlannedBlocks ? nb : kPlannedBlocks;
  }
  static constexpr int pl_pc(int lh) { return (8192 >> lh) + 1; }
  static constexpr int pl_rm(int lh) { return (8192 >> lh) + 8; }
  static constexpr int planned_lds_dwords(int lh) {
    const int h = 1 << lh;
    const int pc = (h / 2) * pl_pc(lh), rm = (h * pl_rm(lh) + 1) / 2;
    return pc > rm ? pc : rm;
  }
};

// FP32 tiles: block b of the tile holds BS(W, H) floats at b * BS, laid
// out column-major (pitch H + 1) for the column phase and row-major (pitch
// W + 1) for the row phase and the coalesced stores; odd pitches keep the
// per-element accesses of a wave in distinct banks.  NB = 256 / max(W, H),
// capped so that the tile fits kLds floats (34 KiB: four workgroups per CU).
struct BatchGeoF32 {
  static constexpr int kLds = 8704;
  static constexpr int bs(int lw, int lh) {
    const int w = 1 << lw, h = 1 << lh, cm = w * (h + 1), rm = h * (w + 1);
    return cm > rm ? cm : rm;
  }
  static constexpr int nb_for(int lw, int lh) {
    const int nb = 256 >> (lw > lh ? lw : lh);
    const int cap = kLds / bs(lw, lh);
    return nb < cap ? nb : cap;
  }
};

// What one axis id means at one block size, for kernels that read block
// descriptors directly: the batched kind (0 DCT-2, 1 adjusted DST-7,
// 2 adjusted DCT-8; -1 not usable at this size) and its band taps, as
// packed int16 pairs (pf, pi) and as fp32 (ff, fi).
struct AxisDev {
  int32_t kind;
  int32_t pad;
  const uint32_t* pf;
  const uint32_t* pi;
  const float* ff;
  const float* fi;
};
constexpr int kAxisIds = 256;
constexpr int kAxisSizes = 7;   // indexed by log2 of the size (2..6 used)
// descriptors per workgroup of the block-list kernels (one per thread), and
// descriptors sorted together by kSortQuarters such workgroups
constexpr int kDescWindow = 256;
constexpr int kSortQuarters = 4;

constexpr int kSchedPitch = 32;     // dwords between schedule counters (128 B)
constexpr int kSchedDwords = (kXcds + 1) * kSchedPitch;

struct BatchArgs {
  const BatchTile* tiles;
  int64_t ntiles;
  int64_t xstart[kXcds + 1];
  const ta_block* blocks;
  const int32_t* deltas;  // planned int16: (in_delta, out_delta) per block
  // planned int16: tiles per XCD list in device memory (list x is
  // tiles[xstart[x] .. xstart[x] + xcount[x])), or null for xstart[x + 1]
  const int32_t* xcount;
  // planned fp32: block b of a tile is blocks[order[first + b]], or null for
  // blocks[first + b]
  const int32_t* order;
  // planned int16: the tile counters of the dynamic schedule (one per XCD
  // list, then the count of finished workgroups, kSchedPitch dwords apart;
  // zero between launches), or null for a static grid stride
  int32_t* sched;
  const int16_t* in;      // int16 data; the fp32 kernels read these as float*
  int16_t* out;
  int bd, m, a;
  // unplanned block lists (ta_transform_fwd / _inv): descriptors are read as
  // they are, grouped into tiles on the device
  const AxisDev* axes;    // kAxisIds x kAxisSizes
  int64_t nblocks;
};

// Persistent batched kernels (batch_kernels.hip): over a planned tile list
// (desc = 0) or directly over a device array of block descriptors (desc = 1);
// int16 fixed point, or fp32 with f32 = 1.
const void* batch_kernel(int inv, int desc = 0, int f32 = 0);

// Block lists planned on the device (ta_transform_fwd_ws / _inv_ws): one
// workgroup per window of kPlanWin consecutive descriptors writes the
// window's tiles and block deltas for the planned int16 kernels.
constexpr int kPlanWin = 4096;
constexpr int kPlanThreads = 1024;   // threads of a planning workgroup
struct PlanArgs {
  const ta_block* blocks;
  int64_t nblocks;
  const AxisDev* axes;    // kAxisIds x kAxisSizes
  BatchTile* tiles;       // kXcds lists of `cap` tiles (list x from x * cap)
  int32_t* deltas;        // int16: (in_delta, out_delta) by window and grouped position
  int32_t* index;         // fp32: list index of each block, by window and grouped position
  int32_t* count;         // tiles written to each list (zero before the launch)
  int64_t cap;
};
const void* desc_plan_kernel(int f32);
// zeroes n dwords (one workgroup; the counters of a device-planned call)
const void* zero_words_kernel();

// Encoder evaluation of the five separable transforms (multi_kernels.hip):
// out holds 5 consecutive packed batches of nblocks N x N int16 blocks.
struct MultiArgs {
  const int16_t* in;
  int16_t* out;
  int64_t nblocks;
  const void* q_eo;   // sub-block Q of the DST-7 design, even/odd column pairs
  int s_row, s_col, a;
};
const void* multi_kernel(int log2n, int b, int* threads, int* blocks);

// Quantised-coefficient statistics (stats_kernels.hip).
struct StatsArgs {
  const int16_t* in;
  int64_t nblocks;
  int64_t total;          // coefficients: nblocks * positions
  int64_t wave_steps;     // wave steps over the batch (64 positions each)
  int64_t full_steps;     // workgroup steps wholly inside the batch
  int64_t steps;          // workgroup steps (4 wave steps each)
  int64_t steps_per_wg;   // workgroup steps per block range
  int64_t ranges;         // block ranges (workgroups per 64 positions)
  int64_t wstride;        // elements between wave steps: max(positions, 64)
  int positions, log2h, log2w;
  int slabs;              // workgroups side by side: max(positions / 64, 1)
  int step, offset;
  uint32_t magic;         // ceil(2^k / step), k = magic_shift
  int magic_shift;        // 16 + ceil(log2 step)
  uint32_t* hist;         // positions x 65 symbol counts
  uint64_t* esc_bits;
  uint64_t* energy;
  uint64_t* dist;
  double* rate;
  double* summary;
  uint32_t* part;         // workspace: ranges x positions x 33 packed counters
  uint64_t* part_e;       // workspace: ranges x positions each
  uint64_t* part_d;
  uint64_t* part_b;
  double* log_energy;     // workspace: log2(E_p / n) per position
};
constexpr int kStatsSymbols = 65;       // levels -31..31 and the two escapes
constexpr int kStatsPartDwords = 33;    // packed counter dwords per partial
// 0 fill, 1 accumulate, 2 rate per position, 3 summary, 4 reduce partials
const void* stats_kernel(int which);

// Batched adjustment design search (design_kernels.hip).
struct DesignArgs {
  const double* mats;   // nmat x N x N
  int nmat;
  const int* cands;     // ncand x {base index, target index, mode (0 pre, 1 post), sigma (+-1)}
  double* theta;        // ncand x N(N-1)/2, in: start, out: final angles
  int steps;
  double lr, lam, beta1, beta2, eps;
  double* grad;         // ncand x N(N-1)/2 or null: gradient at the final angles
  double* obj;          // ncand x 3: objective, sparsity term, error term at the final angles
  double* adj;          // ncand x N x N or null: the final adjustment M
};
const void* design_kernel(int n, int* threads);

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
// Static scratch of the allocation-free backward (givens_kernels.hip): room
// for the partial rows of kNoAllocGroups workgroups of 256 vectors.
constexpr int64_t kNoAllocGroups = 4096;
// Device address of the scratch on `device` (looked up once per device):
// 0, or -1 for a device index out of range, -2 for a HIP failure.
int givens_scratch(int device, float** ptr);

// ---- General block transforms (gen_kernels.hip) ---------------------------
// Every axis kind runs as a program of at most two 1-D stages (eq. 1: the
// adjustment A before the base or C after it, never both; the DCT-8 flip is
// folded into the core kind and the parameter tables by the host):
//   forward  none [core], band [A, core], sub-block [core, C]
//   inverse  the transposed stages in reverse order.
// Each stage ends with clip16(RS(sum, shift)) in fixed point, the core stage
// shifting by the pass's core shift and the adjustment by a.
enum GenOp : int32_t {
  GS_C2 = 0,     // DCT-2 butterfly
  GS_S2 = 1,     // DST-2 = R DCT-2 S
  GS_C3 = 2,     // DCT-3 butterfly
  GS_S3 = 3,     // DST-3 = S DCT-3 R
  GS_DENSE = 4,  // N x N matrix from p (direct DST-7 / DCT-8 and their transposes,
                 // sub-blocks of a side without a compiled stage, as blkdiag(C, 2^a I))
  GS_BAND = 5,   // K-tap band from p, K = arg, transposed window when tr
  GS_POST = 6    // B x B sub-block from p on the first B entries, B = arg in {4, 8, 16}
};
struct GenStage {
  int32_t op, arg, tr;
  int32_t adj;        // 1: shift by the adjustment precision a; 0: by the core shift
  const void* p;      // int16 pairs (fixed point) or floats (fp32), by the launch dtype
};
struct GenProg {
  int32_t nst, pad;   // stages in use (1 or 2)
  GenStage st[2];
};
constexpr int kGenLdsI16 = 16896;   // halfwords of a general int16 tile (64 x 64: 4 blocks of 64 rows of 66; 33 KiB)
constexpr int kGenLdsF32 = 8704;    // floats of a general fp32 tile (34 KiB)
// Tile geometry of the general kernels: NB blocks of W x H side by side,
// block b at b * BS elements, row r of a block at r * RP (int16: RP = W + 2
// halfwords, an odd number of dwords; fp32: RP = W + 1 floats).
struct GenGeo {
  static constexpr int rp(int lw, bool f32) { return (1 << lw) + (f32 ? 1 : 2); }
  static constexpr int bs(int lw, int lh, bool f32) { return (1 << lh) * rp(lw, f32); }
  static constexpr int nb_for(int lw, int lh, bool f32) {
    const int nb = 256 >> (lw > lh ? lw : lh);
    const int cap = (f32 ? kGenLdsF32 : kGenLdsI16) / bs(lw, lh, f32);
    return nb < cap ? nb : cap;
  }
};
struct GenArgs {
  // planned tiles (ph_f / ph_i / pv_f / pv_i hold GenProg pointers of the
  // forward and inverse programs) in per-XCD lists, or null for a packed batch
  const BatchTile* tiles;
  int64_t xstart[kXcds + 1];
  const ta_block* blocks;   // descriptors (planned order, or the caller's list)
  const void* in;
  void* out;
  int inv, bd, m, a;
  // packed batch (tiles == null, blocks == null): nblocks blocks of
  // 2^lw x 2^lh with the programs ph, pv of the launch direction;
  // unplanned list (tiles == null, blocks != null): nblocks descriptors
  int lw, lh;
  int64_t nblocks;
  const GenProg* ph;
  const GenProg* pv;
  // unplanned: programs per (axis id, log2 size, direction) for this dtype
  // (kAxisIds x kAxisSizes x 2; nst = 0 where the axis has none)
  const GenProg* progs;
  // unplanned, beside the fast block-list kernel: the fast kinds' table; a
  // descriptor whose two axes both have a fast kind is left to that kernel
  const AxisDev* fast;
};
// 0 = planned or packed, 1 = unplanned descriptors; fp32 with f32 = 1
const void* gen_kernel(int desc, int f32);

// ---- Backward of the fp32 block-list transform (bwd_kernels.hip) ----------
constexpr int kBwdMaxEntries = 512;   // matrix-gradient entries: 64 x 8 band support, 16 x 16 sub-block
constexpr int kBwdMaxAngles = 128;    // 126 for a 64-point 8-tap band, 120 for a 16 x 16 sub-block
struct BwdArgs {
  const ta_block* blocks;
  int64_t nblocks;
  const float* x;             // forward inputs (at in_off, in_stride)
  const float* gy;            // dL/dY (at out_off, out_stride)
  float* gx;                  // dL/dX (at in_off, in_stride)
  const GenProg* progs;       // fp32 stage programs [axis id][log2 size][direction]
  const int32_t* axis_use;    // per axis id: param id | flip << 8 | adjustment << 9, or -1
  int pid, kind, n, k_or_b;   // the angle set: id, TA_ADJ_BAND / TA_ADJ_POST, size, K or B
  int ne;                     // matrix-gradient entries: n * K (band support) or B * B
  float* part;                // [grid][ne] per-workgroup partial sums
};
struct BwdChainArgs {
  const float* part;
  int64_t groups;             // partial rows to sum
  int ne, kind, n, k_or_b, nang;
  const double* angles;       // the set's angles (band theta, sub-block phi)
  const double* q0;           // sub-block Q0 (B x B), null for the identity
  float* gtheta;
};
// 0 = per-block gradients (persistent over the list), 1 = chain rule (one workgroup)
const void* bwd_kernel(int which);

// Tables of compiled kernels (defined in the kernel translation units).
const KernelEntry* fx_kernels(int* count);
const KernelEntry* f32_kernels(int* count);
const KernelEntry* mfma_kernels(int* count);

}  // namespace ta
