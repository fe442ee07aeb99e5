/*
 * tadj.h -- C ABI of libtadj: batched separable 2-D adjusted DCT/DST
 * transforms of residual blocks on AMD Instinct MI355X (gfx950).
 *
 * What is computed (Said, Egilmez, Chao, "Low-complexity transform
 * adjustments for video coding"):
 *   eq. 1        H = C B A approximates a desired transform D (DST-7/DCT-8),
 *                B in {DCT-2, DCT-3, DST-2, DST-3} (section 2.1), A a sparse
 *                band ("K-tap") orthogonal pre-adjustment, C a top-left
 *                B x B sub-block orthogonal post-adjustment; only one of A, C
 *                per axis (section 2.2).
 *   eq. 3/4/5    DCT-8 from a DST-7 design: H -> S H R; for the sub-block
 *                after the DCT-2 the adjustment becomes S C S.
 *   section 2.2  separable application: every row of a W x H block by the
 *                horizontal H_h, every column by the vertical H_v, i.e.
 *                Y = H_v X H_h^T; the inverse is X = H_v^T Y H_h.
 *
 * Arithmetic.
 *   TA_I16 (fixed point): int16 in, int32 accumulation, int16 out.  Integer
 *   tables T_int = round_half_away(2^m sqrt(N) T) (m = 8); adjustments at
 *   scale 2^a.  Each stage computes clip16((sum + 2^(s-1)) >> s).  Core
 *   shifts: forward rows first with s = log2 W + bd + m - 15, then columns
 *   with s = log2 H + m; inverse columns first with s = m + 1, then rows with
 *   s = m + 14 - bd; adjustment stages shift by a.  The library returns the
 *   exact integers of that definition (any int16 input).
 *   TA_F32: the same stages in fp32 on orthonormal tables, no rounding.
 *
 * Layout.  Blocks are row-major (index r*W + c), int16 or fp32.  A "packed
 * batch" is nblocks contiguous W x H blocks.  A "block list" is an array of
 * ta_block descriptors in device memory, each naming its own offsets,
 * strides, size and per-axis transform.
 *
 * Ownership.  The caller owns every input/output buffer (device memory, for
 * example from torch).  The context owns its parameter tables (device memory
 * allocated by ta_create / ta_set_*).  in and out must not alias.
 *
 * Streams.  Transform calls are asynchronous on the given hipStream_t (0 =
 * null stream), allocate nothing, never synchronise, and may be captured in
 * a HIP graph.  Configuration calls (ta_set_*) are synchronous.
 *
 * Errors.  Every call returns 0 on success or a negative TA_E* code; nothing
 * is launched when a call fails.  ta_last_error() returns a thread-local
 * message describing the last failure.
 */
#ifndef TADJ_H
#define TADJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ta_ctx ta_ctx;
typedef struct ihipStream_t* ta_stream_t;   /* hipStream_t */

enum {
  TA_OK = 0,
  TA_EINVAL = -1,        /* null pointer, negative count, bad enum value, aliasing */
  TA_EUNSUPPORTED = -2,  /* size not a power of two in 4..64, K/B out of range,
                            combination without a kernel */
  TA_ENOPARAMS = -3,     /* axis or parameter id not registered */
  TA_EHIP = -4           /* HIP runtime error (message in ta_last_error) */
};

/* Data types of transform inputs/outputs. */
enum { TA_I16 = 0, TA_F32 = 1 };

/* Base transforms (section 2.1; DST-7/DCT-8 as full matrices, eq. 3). */
enum { TA_DCT2 = 0, TA_DCT3 = 1, TA_DST2 = 2, TA_DST3 = 3, TA_DST7 = 4, TA_DCT8 = 5 };

/* Adjustment kinds (eq. 1, Fig. 2): none, band A before B, sub-block C after B. */
enum { TA_ADJ_NONE = 0, TA_ADJ_BAND = 1, TA_ADJ_POST = 2 };

/* One axis of a separable transform. */
typedef struct {
  int32_t base;      /* TA_DCT2 .. TA_DCT8 */
  int32_t adj;       /* TA_ADJ_* ; TA_DST7/TA_DCT8 require TA_ADJ_NONE */
  int32_t flip;      /* 1: use S H R (the DCT-8 version of a DST-7 design, eq. 3, eq. 5) */
  int32_t param_id;  /* parameter set for adj != NONE (ta_set_band / ta_set_post) */
} ta_axis;

/* Block descriptor for block lists (32 bytes, device memory). */
typedef struct {
  int64_t in_off;      /* element offset of the block's (0,0) in the input buffer */
  int64_t out_off;     /* element offset of the block's (0,0) in the output buffer */
  int32_t in_stride;   /* elements between rows in the input (>= W) */
  int32_t out_stride;  /* elements between rows in the output (>= W) */
  uint8_t log2w;       /* 2..6 */
  uint8_t log2h;       /* 2..6 */
  uint16_t axis_h;     /* axis id (ta_set_axis) of the horizontal (row) transform */
  uint16_t axis_v;     /* axis id of the vertical (column) transform */
  uint16_t reserved;
} ta_block;

/* Create a context on HIP device `device`.  bit_depth (bd) in 6..16 sets the
 * fixed-point shifts; m (integer-matrix precision) in 6..9 sets the integer
 * base tables round_half_away(2^m sqrt(N) T) (m = 6 is the scaling of the
 * video-codec integer transforms the paper integrates into; m above 9 could
 * overflow the int32 sums of 64-point stages), with bd + m >= 14 so that
 * every core shift is at least 1; a (adjustment precision) in 6..14 is the
 * scale 2^a of integer adjustment parameters.  The specialised and
 * matrix-core fixed-point kernels hold the m = 8 tables: at another m every
 * fixed-point transform runs on the general kernel (the same definition),
 * ta_set_impl(1) finds no kernel and ta_fwd_multi is unsupported. */
int ta_create(ta_ctx** out, int device, int bit_depth, int m, int a);

/* The n x n integer base table of kind TA_DCT2 .. TA_DCT8 at precision m
 * (6..9), row-major (rows = basis vectors), as every kernel of a context
 * with that m uses it (section 2.1: DCT-3 = DCT-2^T, DST-2 = R DCT-2 S,
 * DST-3 = S DCT-3 R, each exact in integers).  Host memory; needs no
 * device.  Errors: TA_EINVAL (kind, null), TA_EUNSUPPORTED (n, m). */
int ta_int_table(int kind, int n, int m, int16_t* out);
int ta_destroy(ta_ctx* ctx);

/* Register a K-tap band pre-adjustment A (section 2.2 item 1, Fig. 2a) for
 * size n (4..64), K in {2,4,6,8}, as dense row-major n x n host arrays:
 * a_int at scale 2^a (int16) and a_f32 (orthonormal, fp32).  Row i may have
 * non-zeros only in columns [s_i, s_i + K) with
 * s_i = i - K/2 + ((i + K/2) mod 2), the support of K/2 layers of parallel
 * Givens rotations on adjacent pairs (even pairs first); otherwise
 * TA_EUNSUPPORTED.  Copied synchronously; param_id in 0..255.
 * Registering a param_id again stores new device tables; the previous ones
 * stay allocated until ta_destroy, so a plan built earlier keeps the values
 * it was built with.  Must not run concurrently with transform calls on the
 * same context. */
int ta_set_band(ta_ctx* ctx, int param_id, int n, int taps,
                const int16_t* a_int, const float* a_f32);

/* Register a B x B sub-block post-adjustment Q (section 2.2 item 2, Fig. 2b):
 * C = blkdiag(Q, I_{n-B}), 2 <= B <= n, B even; q_int at scale 2^a.  Same
 * copy and re-registration rules as ta_set_band. */
int ta_set_post(ta_ctx* ctx, int param_id, int n, int b,
                const int16_t* q_int, const float* q_f32);

/* Register axis configuration `axis_id` (0..255).  The size of the axis is
 * taken from the block; parameter sets must match that size. */
int ta_set_axis(ta_ctx* ctx, int axis_id, const ta_axis* axis);

/* The same registration with the size and K/B stated (eq. 1: one adjustment
 * per axis, band A or sub-block C, never both).  log2n = 0 leaves the size to
 * the block; otherwise, with an adjustment, it must be the parameter set's
 * size.  k_or_b = 0 takes K (band taps) or B (sub-block side) from the
 * parameter set; otherwise it must equal it.  An axis without adjustment
 * takes k_or_b = 0.  Errors: TA_EINVAL (mismatch, null), TA_ENOPARAMS,
 * TA_EUNSUPPORTED as for ta_set_axis. */
typedef struct {
  int32_t base, adj, flip;   /* as in ta_axis */
  int32_t log2n;             /* 0 or 2..6 */
  int32_t k_or_b;            /* 0, or K taps (band) / B (sub-block) */
  int32_t param_id;
} ta_axis_cfg;
int ta_set_axis_cfg(ta_ctx* ctx, int axis_id, const ta_axis_cfg* cfg);

/* Register parameter set `param_id` from a layout triple
 * layout = {adj, size, k_or_b}: TA_ADJ_BAND takes n = size * size dense
 * entries (ta_set_band with K = k_or_b), TA_ADJ_POST takes n = k_or_b^2
 * entries of Q (ta_set_post with B = k_or_b).  int_taps at scale 2^a and
 * f32_params in host memory, copied synchronously.  Errors: TA_EINVAL
 * (layout kind, n does not match the layout, null), then those of
 * ta_set_band / ta_set_post. */
int ta_set_params(ta_ctx* ctx, int param_id, const int16_t* int_taps, const float* f32_params,
                  const int32_t* layout, int64_t n);

/* Forward / inverse transform of a packed batch of nblocks W x H blocks
 * (W = 2^log2w, H = 2^log2h), horizontal axis axis_h, vertical axis_v.
 * in/out: device pointers to nblocks*W*H elements of dtype, 16-byte aligned,
 * not overlapping.  Every registered axis kind runs at every size 4..64 (a
 * parameter set serves the size it was registered for): common pairs have
 * specialised kernels (and the matrix-core ones, see ta_set_impl), the
 * others run on the general kernel, which applies each axis as its stages
 * (eq. 1: band A then base, or base then sub-block C; the inverse transposed
 * in reverse order) with the same integer results.  TA_EUNSUPPORTED only
 * when ta_set_impl(1) requires a matrix-core kernel that is not built. */
int ta_fwd_packed(ta_ctx* ctx, int axis_h, int axis_v, int log2w, int log2h,
                  int64_t nblocks, const void* in, void* out, int dtype, ta_stream_t stream);
int ta_inv_packed(ta_ctx* ctx, int axis_h, int axis_v, int log2w, int log2h,
                  int64_t nblocks, const void* in, void* out, int dtype, ta_stream_t stream);

/* ---- Encoder evaluation of the five separable transforms ------------------
 * Section "Simultaneous transform adjustments for the DCT-8 and DST-7" and
 * eq. 5: an encoder compares, per block, DCT-2 x DCT-2 and the four
 * (vertical, horizontal) pairs of DST-7 and DCT-8.  With the sub-block
 * post-adjustment all five share the DCT-2, and the DCT-8 adjustment S Q S
 * is computed together with the DST-7 one Q at the cost of one adjustment.
 * ta_fwd_multi writes, for a packed batch of nblocks N x N int16 blocks
 * (N = 2^log2n), five consecutive packed int16 batches into out:
 *   out[0]: DCT-2 rows and columns,
 *   out[1]: vertical DST-7, horizontal DST-7,
 *   out[2]: vertical DST-7, horizontal DCT-8,
 *   out[3]: vertical DCT-8, horizontal DST-7,
 *   out[4]: vertical DCT-8, horizontal DCT-8,
 * each (out + k * nblocks * N * N) bit-identical to ta_fwd_packed with the
 * corresponding axes (DCT-2; DCT-2 + sub-block param_id; the same flipped).
 * param_id: a set registered with ta_set_post for size N (the DST-7 design).
 * Built for (N, B) = (32, 8) and (64, 16); fixed point only; out holds
 * 5 * nblocks * N * N int16 and must not overlap in.  Errors: TA_ENOPARAMS
 * (not a sub-block set), TA_EINVAL (size mismatch, null, misaligned,
 * overlap), TA_EUNSUPPORTED (other N, B). */
int ta_fwd_multi(ta_ctx* ctx, int param_id, int log2n, int64_t nblocks, const void* in, void* out,
                 ta_stream_t stream);

/* ---- Batched uneven blocks (block lists) ----------------------------------
 * A plan takes a host array of n ta_block descriptors (block sizes 4..64 per
 * side, any mix) whose axes are any registered kind (base DCT-2, DCT-3,
 * DST-2, DST-3, direct DST-7 / DCT-8; band or sub-block adjustment of any
 * registered K / B; flipped or not): an axis with an adjustment names the
 * parameter set of one size, so a workload registers one axis id per
 * (type, size).  A plan whose axes are all DCT-2, DST-3 + 4-tap band or its
 * flip (the adjusted DST-7 / DCT-8) runs on the fast batched kernel; any
 * other kind moves the whole plan to the general kernel (the same results,
 * each axis applied as its stages).  Offsets and row strides are in elements and must be
 * multiples of 8 (4 for 4-wide blocks); the forward reads the residual
 * block at (in_off, in_stride) of `in` and writes its coefficients at
 * (out_off, out_stride) of `out`; the inverse reads coefficients at
 * (in_off, in_stride) and writes residuals at (out_off, out_stride).
 * dtype TA_I16 runs the fixed-point transforms (bit-exact), TA_F32 the
 * orthonormal fp32 ones (the fp32 parameters of each set); in and out then
 * hold int16 or float elements.
 * ta_plan_create copies the descriptors to device memory, grouped by
 * (size, kinds) into tiles (synchronous, allocates).  ta_plan_fwd/_inv run
 * the whole plan as one persistent kernel launch on the stream
 * (asynchronous, no allocation, capturable in a HIP graph).  With an int16
 * plan whose grid is resident at once, the workgroups take tiles from
 * counters the plan holds (one set per direction, reset by each launch at its
 * end): two launches of one plan in the same direction must not run at the
 * same time (serialise them on one stream, or use two plans).
 * ta_plan_autotune times the tile mappings (frame regions of 2^18 .. 2^22
 * input elements per XCD tile list) times the persistent grid sizes (256 ..
 * 8192 workgroups) on the given buffers, then, at the fastest of those, the
 * blocks per tile of each size group (blocks whose larger side is 4, 8, 16,
 * 32 or 64: the kernels' maximum, half of it or a quarter, one group after
 * the other).  Each candidate runs twelve forward launches, then twelve
 * inverse ones (the last six of each timed), on three buffer sets in turn,
 * so that every launch finds the caches holding the other sets' data, as
 * when batches stream through HBM once per call: set 0 is the
 * caller's `in` and `out`, sets 1 and 2 copies of `in` in scratch, and every
 * set's inverse output goes to scratch (the inverse reads its set's forward
 * output, or its set's input when `out` is smaller than the plan's input
 * extent).  The candidates are timed in `reps` interleaved rounds (clocks
 * drift under load) and scored by the sum of their median forward and
 * inverse times; scores within 1 % of the best count as equal, and the
 * smallest grid among them wins.  The tuner checks that every candidate's outputs are
 * bitwise identical and keeps the fastest (synchronous; allocates scratch of
 * twice the plan's input extent plus five times its output extent while it
 * runs; leaves the forward of `in` in `out`).  ta_plan_set_tuning applies
 * a known grid (>= 8) and region (log2 input elements, 12..40) without
 * timing (synchronous).  Both rewrite
 * the plan's device tile list in place: launches captured in a HIP graph
 * before must be captured again.  ta_plan_tuning reports the grid and
 * region in use.  ta_plan_tile_blocks reports how many blocks of size
 * 2^log2w x 2^log2h (log2 sizes 2..6) one tile holds at most, and
 * ta_plan_set_tile_blocks sets it: 1 .. the kernels' maximum for that size
 * and dtype, or 0 for that maximum (synchronous; rebuilds the tile list like
 * ta_plan_set_tuning; TA_EINVAL outside those ranges).  Fewer blocks per tile
 * give more, smaller tiles: better balance across the grid, less overlap of
 * one tile's loads with the previous tile's arithmetic.  Blocks must not
 * overlap in `out`.  A plan runs only with
 * the context that created it (TA_EINVAL otherwise) and must be destroyed
 * before that context: its tiles point into the context's parameter
 * tables. */
typedef struct ta_plan ta_plan;
int ta_plan_create(ta_ctx* ctx, const ta_block* blocks_host, int64_t n, int dtype, ta_plan** out);
int ta_plan_destroy(ta_plan* plan);
int ta_plan_info(const ta_plan* plan, int64_t* nblocks, int64_t* ntiles, int* grid);
/* The plan's dtype and the smallest input / output buffers (in elements)
 * that hold every block it addresses; ta_plan_fwd/_inv cannot check their
 * buffers (they take none of these sizes), so the caller checks them here. */
int ta_plan_extents(const ta_plan* plan, int* dtype, int64_t* in_elems, int64_t* out_elems);
int ta_plan_fwd(ta_ctx* ctx, ta_plan* plan, const void* in, void* out, ta_stream_t stream);
int ta_plan_inv(ta_ctx* ctx, ta_plan* plan, const void* in, void* out, ta_stream_t stream);
int ta_plan_autotune(ta_ctx* ctx, ta_plan* plan, const void* in, void* out, ta_stream_t stream, int reps);
int ta_plan_tuning(const ta_plan* plan, int* grid, int* region_log2);
int ta_plan_set_tuning(ta_plan* plan, int grid, int region_log2);
int ta_plan_tile_blocks(const ta_plan* plan, int log2w, int log2h, int* blocks);
int ta_plan_set_tile_blocks(ta_plan* plan, int log2w, int log2h, int blocks);

/* Unplanned block lists.  ta_transform_fwd / _inv run nblocks descriptors
 * that are already in device memory (blocks_dev, 8-byte aligned, read as
 * they are, e.g. written by an earlier kernel) in one launch: the list is cut
 * into windows of 1024 consecutive descriptors, and the descriptors of equal
 * size and axis ids inside a window are grouped (in list order) into tiles
 * of up to 64 blocks.  Throughput grows with the number of equal
 * configurations per window; a plan (ta_plan_create) groups the whole list
 * on the host once and runs fastest.  The
 * descriptor rules, transforms and dtypes are those of the plans (axes
 * resolve through the context at launch time, so a parameter set registered
 * again is seen by the next call).  The fast batched kernel runs the
 * descriptors whose axes are DCT-2 or the DST-3 + 4-tap band (plain or
 * flipped); once any axis registered with the context has another kind, a
 * second launch on the same stream runs the other descriptors on the
 * general kernel.  A descriptor that breaks a
 * rule the kernel can check (size, offset sign and alignment, stride, axis
 * id, an axis that does not resolve at the block's size) is skipped and its
 * output untouched.
 * Extents are the caller's contract: every block must lie inside in and out
 * and blocks must not overlap in out; ta_validate_blocks checks a list.
 * in and out: 16-byte aligned device memory, not the same buffer.
 * Asynchronous on the stream, allocates nothing, capturable in a HIP graph.
 * Errors: TA_EINVAL (null, negative count, alignment, aliasing, dtype). */
int ta_transform_fwd(ta_ctx* ctx, const ta_block* blocks_dev, int64_t nblocks, const void* in, void* out,
                     int dtype, ta_stream_t stream);
int ta_transform_inv(ta_ctx* ctx, const ta_block* blocks_dev, int64_t nblocks, const void* in, void* out,
                     int dtype, ta_stream_t stream);

/* Unplanned block lists planned on the device.  ta_transform_fwd_ws / _inv_ws
 * take the same arguments and rules as ta_transform_fwd / _inv plus a
 * workspace in device memory (256-byte aligned, at least the size that
 * ta_transform_workspace gives for nblocks; the caller owns it; its contents
 * need no initialisation and are scratch after the call).  At m = 8 a first
 * kernel plans the list: windows of 4096 consecutive descriptors are grouped
 * by configuration (size and axis ids) and cut into tiles of equal
 * configuration and row strides, which the planned kernels (int16 or fp32)
 * then run in one launch.  The tiles are larger than the in-window groups of
 * ta_transform_fwd, so throughput is closer to a plan's.  One more rule
 * applies to int16 lists here: a block whose rows span more than 2^30 input
 * or 2^31 output elements ((h - 1) * stride + w) is skipped.  Contexts with
 * m != 8 run exactly as ta_transform_fwd / _inv (the workspace
 * is not used).  Asynchronous on the stream, allocates nothing, capturable
 * in a HIP graph; two calls that share a workspace must not run at the same
 * time.  Errors: those of ta_transform_fwd, and TA_EINVAL for a missing,
 * misaligned or short workspace.  ta_transform_workspace: bytes of workspace
 * for nblocks descriptors (about 8 + 80 bytes a descriptor; 0 for none);
 * TA_EINVAL for a null pointer or a negative count. */
int ta_transform_workspace(int64_t nblocks, int64_t* bytes);
int ta_transform_fwd_ws(ta_ctx* ctx, const ta_block* blocks_dev, int64_t nblocks, const void* in, void* out,
                        int dtype, void* workspace, int64_t workspace_bytes, ta_stream_t stream);
int ta_transform_inv_ws(ta_ctx* ctx, const ta_block* blocks_dev, int64_t nblocks, const void* in, void* out,
                        int dtype, void* workspace, int64_t workspace_bytes, ta_stream_t stream);

/* Check n device descriptors against the block-list rules and against
 * buffers of in_elems input and out_elems output elements (a debugging aid:
 * copies the list to the host and synchronises).  On the first descriptor
 * that fails, sets *first_bad to its index and returns its error (TA_EINVAL
 * or TA_EUNSUPPORTED, or TA_ENOPARAMS for an unregistered axis) with the
 * reason in ta_last_error(); otherwise *first_bad = -1 and TA_OK.  Overlap
 * of blocks in the output is not checked. */
int ta_validate_blocks(ta_ctx* ctx, const ta_block* blocks_dev, int64_t n, int64_t in_elems, int64_t out_elems,
                       int64_t* first_bad);

/* ---- Quantised-coefficient statistics (coding-gain proxy) -------------------
 * A codec-free stand-in for the coding results of the experiments section
 * (Tables 2 and 3), which compare BD-rates inside a video codec: on the same
 * residual blocks, how the adjusted and the exact transforms compare in
 * energy compaction and in the rate of the quantised coefficients.
 * coef: nblocks packed H x W int16 coefficient blocks (H = 2^log2h,
 * W = 2^log2w, 2 <= log2h, log2w <= 6), e.g. the output of ta_fwd_packed.
 * Quantiser: level q = sign(y) floor((|y| + offset) / step), 1 <= step <=
 * 32768, 0 <= offset < step (offset = step / 2 rounds to nearest, ties away
 * from zero).  Symbols: q itself for |q| <= 31, else an escape +-32, whose
 * suffix is the order-0 Exp-Golomb code of |q| - 32 (2 floor(log2(|q| - 31))
 * + 1 bits).  Positions p = row * W + col, P = H * W.  Outputs (device
 * memory, overwritten, none may overlap another or coef):
 *   hist      P x 65 uint32, hist[p][32 + s] = blocks with symbol s at p
 *   esc_bits  P uint64, suffix bits of the escapes at p
 *   energy    P uint64, sum of y^2 at p
 *   dist      P uint64, sum of (y - q step)^2 at p
 *   rate      P double, entropy of the symbols at p plus esc_bits / nblocks
 *   summary   7 doubles: mean rate per coefficient (bits), distortion and
 *             energy per coefficient, transform coding gain in dB (10 log10
 *             of the arithmetic over the geometric mean of the per-position
 *             mean energies; 0 with no energy, +inf if some position has
 *             none), fraction of the energy in the top-left (H/4) x (W/4)
 *             positions (0 with no energy), fractions of nonzero and of
 *             escaped levels.  All zero for nblocks = 0.
 * workspace: device scratch of at least ta_coef_stats_workspace(ctx, nblocks,
 * log2h, log2w) bytes, 8-byte aligned (partial results per block range;
 * the size depends on the device's occupancy, so query it per context).
 * Counts and sums are exact; rate and summary are reduced in a fixed order
 * (bitwise repeatable).  Asynchronous on the stream, allocates nothing.
 * Errors: TA_EINVAL (null, misaligned, bad step/offset, workspace too small,
 * nblocks * P > 2^34), TA_EUNSUPPORTED (block size). */
int ta_coef_stats_workspace(ta_ctx* ctx, int64_t nblocks, int log2h, int log2w, int64_t* bytes);
int ta_coef_stats(ta_ctx* ctx, const int16_t* coef, int64_t nblocks, int log2h, int log2w, int32_t step,
                  int32_t offset, uint32_t* hist, uint64_t* esc_bits, uint64_t* energy, uint64_t* dist, double* rate,
                  double* summary, void* workspace, int64_t workspace_bytes, ta_stream_t stream);

/* ---- Batched adjustment design search (FP64) -------------------------------
 * The design study of section 2 (Fig. 1): for each candidate, minimise
 *   f(M) = lam sum_ij M_ij^2 / (0.05 + |M_ij|) + sum_ij w_i (H_ij - D_ij)^2,
 *   w_i = exp(-i ln(100) / n), H = B M (pre-adjustment) or M B (post),
 * (lam = 1 is the printed sparsity objective, lam = 0 is eq. 2) over
 * orthogonal M = G(theta) J: G = n layers of parallel Givens rotations on
 * adjacent pairs, layer l on the pairs starting at l mod 2, rotation (p, p+1)
 * by t: v_p = cos t u_p - sin t u_p+1, v_p+1 = sin t u_p + cos t u_p+1,
 * theta (n(n-1)/2 angles) layer by layer; J = diag(sigma, 1, ..., 1).
 * Each candidate takes `steps` Adam updates (betas 0.9, 0.999, eps 1e-8,
 * bias-corrected, step size lr) from its theta, then is evaluated at the
 * final angles.  n in {4, 8, 16, 32}.  All pointers are device memory:
 *   mats   nmat x n x n row-major matrices (bases and targets)
 *   cands  ncand x 4 int32: base index, target index, mode (0 pre, 1 post),
 *          sigma (+1 or -1); a candidate with an index out of range or a bad
 *          mode or sigma gets NaN objective values and is otherwise skipped
 *   theta  ncand x n(n-1)/2, read as the start, overwritten with the result
 *   obj    ncand x 3: f, sparsity term, error term at the final angles
 *   grad   ncand x n(n-1)/2 gradient at the final angles, or null
 *   adj    ncand x n x n final M, or null
 * steps = 0 evaluates f and its gradient at theta.  Asynchronous on the
 * stream, allocates nothing; results are bitwise repeatable.  Errors:
 * TA_EINVAL (null, misaligned, negative counts, lr <= 0, lam < 0),
 * TA_EUNSUPPORTED (n). */
int ta_design_search(ta_ctx* ctx, int n, int nmat, const double* mats, int64_t ncand, const int32_t* cands,
                     double* theta, int steps, double lr, double lam, double* grad, double* obj, double* adj,
                     ta_stream_t stream);

/* ---- Differentiable refit path (fp32) ---------------------------------------
 * y_m = B A(theta) x_m for nvec vectors of n floats (x, y: nvec x n, row per
 * vector), B = TA_DCT2 or TA_DST3, A(theta) = taps/2 layers of parallel
 * Givens rotations on adjacent pairs (section 2: orthogonality through
 * sequential sets of parallel Givens rotations), layer l on the pairs
 * starting at l mod 2, rotation (p, p+1) by t: v_p = cos t u_p - sin t u_p+1,
 * v_p+1 = sin t u_p + cos t u_p+1; theta holds the angles layer by layer
 * (31 for n = 32, taps = 4).  n in {16, 32}, taps in {4, 6}.  All pointers
 * are device memory; calls are asynchronous and allocate nothing.
 * ta_givens_bwd: given dL/dy (gy), writes dL/dx (gx, may not alias x or gy)
 * and dL/dtheta (gtheta, overwritten), using a caller-provided device
 * workspace of ta_givens_workspace(nvec) bytes; the angle gradient is reduced
 * in a fixed order, so repeated calls are bitwise identical. */
int ta_givens_workspace(int64_t nvec, int64_t* bytes);
int ta_givens_fwd(ta_ctx* ctx, int base, int n, int taps, const float* theta, int64_t nvec,
                  const float* x, float* y, ta_stream_t stream);
int ta_givens_bwd(ta_ctx* ctx, int base, int n, int taps, const float* theta, int64_t nvec,
                  const float* x, const float* gy, float* gx, float* gtheta, void* workspace,
                  ta_stream_t stream);

/* ta_givens_bwd for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the same
 * backward, with the per-workgroup partial rows of the angle gradient in a
 * static device array of the library (1.5 MiB per device, held until the
 * process ends) instead of a caller's workspace; allocates nothing.
 * nvec <= 1,048,576 (4,096 workgroups of 256 vectors), else TA_EINVAL.  The
 * array needs no clearing (every row a call reads is written by that call),
 * and every call on one device shares it: calls that overlap on one device
 * (other streams, other contexts or threads) race and must be ordered by the
 * caller.  Results are bitwise identical to ta_givens_bwd's. */
int ta_givens_bwd_noalloc(ta_ctx* ctx, int base, int n, int taps, const float* theta, int64_t nvec,
                          const float* x, const float* gy, float* gx, float* gtheta, ta_stream_t stream);

/* ---- Backward of the block-list transform (fp32) ---------------------------
 * Adjustments parametrised by angles (section 2: orthogonality through
 * sequential sets of parallel Givens rotations; eq. 2 is minimised over
 * them).  ta_set_band_angles registers band set `param_id` as
 * A(theta) = G_{L-1} ... G_0, L = taps / 2 layers, layer l rotating the
 * adjacent pairs that start at l mod 2, rotation (p, p+1) by t:
 * v_p = cos t u_p - sin t u_p+1, v_p+1 = sin t u_p + cos t u_p+1; theta
 * (host, double) holds the angles layer by layer, pairs in order.
 * ta_set_post_angles registers sub-block set `param_id` (B in {4, 8, 16},
 * B <= n) as Q = Q0 R(phi), R(phi) the rotations over the pairs (p, q),
 * p < q in lexicographic order, each applied after the previous ones; q0 is
 * a B x B row-major orthogonal matrix (host, double) or null for the
 * identity.  Both store the integer (round half away of 2^a M) and fp32
 * tables exactly as ta_set_band / ta_set_post do (so the set serves every
 * transform), and keep the angles for ta_transform_bwd.  Synchronous,
 * allocate; errors as ta_set_band / ta_set_post. */
int ta_set_band_angles(ta_ctx* ctx, int param_id, int n, int taps, const double* theta);
int ta_set_post_angles(ta_ctx* ctx, int param_id, int n, int b, const double* q0, const double* phi);

/* Backward of the fp32 forward ta_transform_fwd over a block list (eq. 1,
 * section 2.2: Y = H_v X H_h^T per block): given dL/dY in gy_dev (each
 * block at out_off, out_stride, like the forward's output), writes
 * dL/dX = H_v^T (dL/dY) H_h into gx_dev (at in_off, in_stride, like the
 * forward's input) and dL/dangles of set param_id into gtheta_dev (its
 * angle count, float), summed over every block axis that uses the set,
 * plain or flipped (DCT-8 from the DST-7 design, eq. 3 / eq. 5); x_dev holds
 * the forward's input (at in_off, in_stride).  All pointers are device
 * memory; gx_dev must not alias x_dev or gy_dev; blocks must not overlap in
 * gx_dev.  The set must have been registered by its angles (else
 * TA_ENOPARAMS).  Descriptors the transforms skip are skipped (their gx left
 * untouched).  The angle gradient is reduced in a fixed order (bitwise
 * repeatable) through a workspace the set owns: calls for one set must not
 * overlap (one stream, or ordered by the caller).  Asynchronous on the
 * stream, allocates nothing.  Errors: TA_EINVAL (null, alignment, aliasing,
 * negative count), TA_ENOPARAMS. */
int ta_transform_bwd(ta_ctx* ctx, const ta_block* blocks_dev, int64_t nblocks, const float* x_dev,
                     const float* gy_dev, float* gx_dev, float* gtheta_dev, int param_id, ta_stream_t stream);

/* Select the kernels used for packed batches: 0 = automatic (the matrix-core
 * kernels for int16 transforms without a band adjustment, where one is built;
 * otherwise the VALU butterfly kernels, which are faster with a band), 1 =
 * matrix-core kernels only (TA_EUNSUPPORTED when none is built), 2 = VALU
 * kernels only.  Both give identical results. */
int ta_set_impl(ta_ctx* ctx, int impl);

/* Library version string. */
const char* ta_version(void);

/* Thread-local description of the last error. */
const char* ta_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TADJ_H */
