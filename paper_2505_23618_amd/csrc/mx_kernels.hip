// 32x32 int16 transforms with the dense core on the int8 matrix cores and the
// band adjustment on VALU (forward direction; one wave per block, persistent
// waves so that the per-lane constant operands are built once).
//
// Forward, block X (32x32), horizontal core Mh with band Ah, vertical Mv, Av:
//   pass 1 (rows):    Z[j][k]  = sum_n u[j][n] Mh[k][n],  u = band_h(X row j)
//   pass 2 (columns): Y[kv][c] = sum_i Mv[kv][i] u2[i][c], u2 = band_v(Z column c)
// Pass 1 is D1 = A1 B1 with A1 rows = block rows (lane l loads block row
// sigma(l%32), positions 16h..16h+15, h = l/32) and B1 columns = output
// frequencies; sigma is chosen so that the result registers r = 0..15 of lane
// (q, h) hold Z[16h + r][q]: rows 16h..16h+15 of column q in order.  That is
// exactly the operand pass 2 needs (contraction over rows in registers), so
// the two passes exchange nothing but a two-row halo between lane halves for
// the vertical band.  Pass 2 is computed transposed, D2[c][kv], so that lane
// (q, h) ends with row kv = q of Y at columns 8a + 4h + (0..3): 8-byte stores.
#include "kernels.hpp"
#include "mx.hpp"

namespace ta {
namespace {

constexpr int kMaxWgs = 1024;   // persistent grid: 4 waves per workgroup

// Halo (in int16 pairs, each side) that the windows of a K-tap band over
// positions 16h..16h+15 reach: window starts are r - L + ((r + L) & 1) for
// L = K/2, so the lowest start is -2*(K/4) and the highest end 16 + 2*(K/4).
template <int K>
constexpr int halo_pairs() {
  int lo = 0, hi = 16;
  for (int r = 0; r < 16 && K > 0; ++r) {
    const int s = r - K / 2 + ((r + K / 2) & 1);
    lo = s < lo ? s : lo;
    hi = s + K > hi ? s + K : hi;
  }
  const int below = (-lo + 1) / 2, above = (hi - 16 + 1) / 2;
  return below > above ? below : above;
}
static_assert(halo_pairs<0>() == 0 && halo_pairs<2>() == 0 && halo_pairs<4>() == 1 &&
              halo_pairs<6>() == 1 && halo_pairs<8>() == 2, "band halo");

// K-tap band over 16 consecutive positions 16h..16h+15 of one vector.
// xs[HP + j] holds positions (16h + 2j, 16h + 2j + 1) for j = -HP .. 8 + HP - 1.
template <int K>
TA_DEV void band16(const uint32_t* xs, const uint32_t (&taps)[16][K / 2], int off, int (&u)[16]) {
  constexpr int L = K / 2, HP = halo_pairs<K>();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int s = r - L + ((r + L) & 1);            // window start relative to 16h (even)
    int acc = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const uint32_t pr = xs[HP + (s >> 1) + t];
      if (t == 0) {
        asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(acc) : "v"(pr), "v"(taps[r][0]), "v"(off));
      } else {
        acc = dot2(pr, taps[r][t], acc);
      }
    }
    u[r] = acc;
  }
}

// SAME: both axes use the same band parameters (one set of tap registers);
// the host only selects such a kernel when the two parameter pointers match.
template <int CH, int KH, int CV, int KV, bool SAME>
__global__ __launch_bounds__(256) void mx_fwd(PackedArgs p) {
  constexpr int N = 32;
  constexpr int HP1 = halo_pairs<KH>(), HP2 = halo_pairs<KV>();
  const int lane = threadIdx.x & 63, q = lane & 31, h = lane >> 5;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * 4;

  // constant operands: B columns for this lane (output frequency q), for the
  // 16 contraction positions 16h..16h+15
  mx::Planes m1, m2;
  int sum1 = 0, sum2 = 0;
  {
    int b1[16], b2[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      b1[j] = mx::core_entry<N>(CH, false, q, 16 * h + j);
      b2[j] = mx::core_entry<N>(CV, false, q, 16 * h + j);
    }
    for (int n = 0; n < N; ++n) {
      sum1 += mx::core_entry<N>(CH, false, q, n);
      sum2 += mx::core_entry<N>(CV, false, q, n);
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      m1.h[w] = (int)mx::pack4(mx::hi_byte(b1[4 * w]), mx::hi_byte(b1[4 * w + 1]), mx::hi_byte(b1[4 * w + 2]), mx::hi_byte(b1[4 * w + 3]));
      m1.l[w] = (int)mx::pack4(mx::lo_byte(b1[4 * w]), mx::lo_byte(b1[4 * w + 1]), mx::lo_byte(b1[4 * w + 2]), mx::lo_byte(b1[4 * w + 3]));
      m2.h[w] = (int)mx::pack4(mx::hi_byte(b2[4 * w]), mx::hi_byte(b2[4 * w + 1]), mx::hi_byte(b2[4 * w + 2]), mx::hi_byte(b2[4 * w + 3]));
      m2.l[w] = (int)mx::pack4(mx::lo_byte(b2[4 * w]), mx::lo_byte(b2[4 * w + 1]), mx::lo_byte(b2[4 * w + 2]), mx::lo_byte(b2[4 * w + 3]));
    }
  }
  const int kc1 = 128 * sum1 + (1 << (p.s_row - 1));
  const int kc2 = 128 * sum2 + (1 << (p.s_col - 1));
  const int offa = 1 << (p.a - 1);

  // band taps of the 16 output positions 16h + r (packed pairs, even-aligned windows)
  uint32_t t1[16][KH > 0 ? KH / 2 : 1], t2[16][(KV > 0 && !SAME) ? KV / 2 : 1];
  if constexpr (KH > 0) {
    const uint32_t* ph = static_cast<const uint32_t*>(p.ph_f);
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int t = 0; t < KH / 2; ++t) t1[r][t] = ph[(16 * h + r) * (KH / 2) + t];
  }
  if constexpr (KV > 0 && !SAME) {
    const uint32_t* pv = static_cast<const uint32_t*>(p.pv_f);
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int t = 0; t < KV / 2; ++t) t2[r][t] = pv[(16 * h + r) * (KV / 2) + t];
  }

  const int16_t* __restrict__ in = static_cast<const int16_t*>(p.in);
  int16_t* __restrict__ out = static_cast<int16_t*>(p.out);
  // block row loaded by this lane: result register r of pass 1 is row 16h + r
  const int row = 16 * ((q >> 2) & 1) + 4 * (q >> 3) + (q & 3);

  // Global traffic is coalesced through a per-wave LDS tile (one 32x32 int16
  // block, rows padded to 80 bytes so that the per-lane row reads below are
  // conflict-free): lane t moves 16-byte chunks t and t + 64 of the block.
  constexpr int RP = 40;                            // halfwords per LDS row
  __shared__ __align__(16) uint16_t tile_all[4][N * RP];
  uint16_t* tile = tile_all[threadIdx.x >> 6];
  auto chunk_addr = [&](int c) { return (c >> 2) * RP + (c & 3) * 8; };

  if (wave >= p.nblocks) return;
  uint4 g0 = reinterpret_cast<const uint4*>(in + wave * (N * N))[lane];
  uint4 g1 = reinterpret_cast<const uint4*>(in + wave * (N * N))[lane + 64];
  for (int64_t blk = wave; blk < p.nblocks; blk += nwaves) {
    // stage this block, then prefetch the next one of this wave
    *reinterpret_cast<uint4*>(tile + chunk_addr(lane)) = g0;
    *reinterpret_cast<uint4*>(tile + chunk_addr(lane + 64)) = g1;
    const int64_t nxt = blk + nwaves < p.nblocks ? blk + nwaves : blk;
    g0 = reinterpret_cast<const uint4*>(in + nxt * (N * N))[lane];
    g1 = reinterpret_cast<const uint4*>(in + nxt * (N * N))[lane + 64];
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_wave_barrier();
    // positions 16h-2HP1 .. 16h+15+2HP1 of block row `row`
    uint32_t xs[8 + 2 * HP1];
    {
      const uint16_t* xr = tile + row * RP;
      const uint4 a = *reinterpret_cast<const uint4*>(xr + 16 * h);
      const uint4 b = *reinterpret_cast<const uint4*>(xr + 16 * h + 8);
      xs[HP1 + 0] = a.x; xs[HP1 + 1] = a.y; xs[HP1 + 2] = a.z; xs[HP1 + 3] = a.w;
      xs[HP1 + 4] = b.x; xs[HP1 + 5] = b.y; xs[HP1 + 6] = b.z; xs[HP1 + 7] = b.w;
#pragma unroll
      for (int k = 0; k < HP1; ++k) {
        const uint32_t lo = reinterpret_cast<const uint32_t*>(xr + 16 - 2 * (HP1 - k))[0];
        const uint32_t hi = reinterpret_cast<const uint32_t*>(xr + 16 + 2 * k)[0];
        xs[k] = h ? lo : 0u;
        xs[HP1 + 8 + k] = h ? 0u : hi;
      }
    }
    uint32_t up[8];
    if constexpr (KH > 0) {
      int u[16];
      band16<KH>(xs, t1, offa, u);
#pragma unroll
      for (int j = 0; j < 8; ++j) up[j] = satpk(u[2 * j] >> p.a, u[2 * j + 1] >> p.a);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) up[j] = xs[j];
    }
    mx::Planes x1;
    mx::split_planes(up, x1.h, x1.l);
    int z[16];
    mx::product(x1, m1, kc1, z);
    // Z[16h + r][q] -> packed pairs of consecutive rows
    uint32_t zs[8 + 2 * HP2];
#pragma unroll
    for (int j = 0; j < 8; ++j) zs[HP2 + j] = satpk(z[2 * j] >> p.s_row, z[2 * j + 1] >> p.s_row);

    // ---- pass 2: vertical band with a halo of HP2 pairs from the other half
    uint32_t vp[8];
    if constexpr (KV > 0) {
#pragma unroll
      for (int k = 0; k < HP2; ++k) {
        const uint32_t send = h ? zs[HP2 + k] : zs[HP2 + 8 - HP2 + k];
        const uint32_t recv = (uint32_t)__shfl_xor((int)send, 32);
        zs[k] = h ? recv : 0u;                // rows 16h - 2(HP2-k) .. (from the lower half)
        zs[HP2 + 8 + k] = h ? 0u : recv;      // rows 16h + 16 + 2k .. (from the upper half)
      }
      int u2[16];
      if constexpr (SAME)
        band16<KV>(zs, t1, offa, u2);
      else
        band16<KV>(zs, t2, offa, u2);
#pragma unroll
      for (int j = 0; j < 8; ++j) vp[j] = satpk(u2[2 * j] >> p.a, u2[2 * j + 1] >> p.a);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) vp[j] = zs[j];
    }
    mx::Planes x2;
    mx::split_planes(vp, x2.h, x2.l);
    int y[16];
    mx::product(x2, m2, kc2, y);
    // lane (q, h), register r = 4a + t: Y[q][8a + 4h + t]; the tile is free
    // once every lane has read its row (wave barrier), then it holds Y
    __builtin_amdgcn_wave_barrier();
    uint16_t* yr = tile + q * RP + 4 * h;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const uint32_t lo = satpk(y[4 * a] >> p.s_col, y[4 * a + 1] >> p.s_col);
      const uint32_t hi = satpk(y[4 * a + 2] >> p.s_col, y[4 * a + 3] >> p.s_col);
      *reinterpret_cast<uint2*>(yr + 8 * a) = make_uint2(lo, hi);
    }
    __builtin_amdgcn_wave_barrier();
    uint4* yo = reinterpret_cast<uint4*>(out + blk * (N * N));
    yo[lane] = *reinterpret_cast<const uint4*>(tile + chunk_addr(lane));
    yo[lane + 64] = *reinterpret_cast<const uint4*>(tile + chunk_addr(lane + 64));
    __builtin_amdgcn_wave_barrier();
  }
}


// Inverse of a plain core on the matrix cores (no adjustment), columns first:
//   pass 1 (columns): U[i][c] = sum_m Mv[m][i] Y[m][c]
//   pass 2 (rows):    X[i][n] = sum_c Mh[c][n] U[i][c]
// Pass 1 is computed as D1[c][i] (A = columns of Y, read from a column-major
// LDS tile, B = Mv^T), so lane (q, h) ends with row i = q of U at columns
// m_r = 8(r/4) + 4h + r%4; pass 2 contracts over those registers, computed as
// D2[n][i] (A = Mh^T rows, B = U rows), leaving row q of X at columns m_r.
template <int CH, int CV>
__global__ __launch_bounds__(256) void mx_inv(PackedArgs p) {
  constexpr int N = 32;
  const int lane = threadIdx.x & 63, q = lane & 31, h = lane >> 5;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * 4;

  // pass 1 B operand: column i = q of Mv^T, i.e. Mv[m][q], rows m = 16h + j
  // pass 2 A operand: row n = q of Mh^T, i.e. Mh[c][q], columns c = m_j
  mx::Planes m1, m2;
  int sum1 = 0, sum2 = 0;
  {
    int b1[16], b2[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      b1[j] = mx::core_entry<N>(CV, true, q, 16 * h + j);
      b2[j] = mx::core_entry<N>(CH, true, q, 8 * (j >> 2) + 4 * h + (j & 3));
    }
    for (int n = 0; n < N; ++n) {
      sum1 += mx::core_entry<N>(CV, true, q, n);
      sum2 += mx::core_entry<N>(CH, true, q, n);
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      m1.h[w] = (int)mx::pack4(mx::hi_byte(b1[4 * w]), mx::hi_byte(b1[4 * w + 1]), mx::hi_byte(b1[4 * w + 2]), mx::hi_byte(b1[4 * w + 3]));
      m1.l[w] = (int)mx::pack4(mx::lo_byte(b1[4 * w]), mx::lo_byte(b1[4 * w + 1]), mx::lo_byte(b1[4 * w + 2]), mx::lo_byte(b1[4 * w + 3]));
      m2.h[w] = (int)mx::pack4(mx::hi_byte(b2[4 * w]), mx::hi_byte(b2[4 * w + 1]), mx::hi_byte(b2[4 * w + 2]), mx::hi_byte(b2[4 * w + 3]));
      m2.l[w] = (int)mx::pack4(mx::lo_byte(b2[4 * w]), mx::lo_byte(b2[4 * w + 1]), mx::lo_byte(b2[4 * w + 2]), mx::lo_byte(b2[4 * w + 3]));
    }
  }
  // pass 1: every result of lane (q, h) is U[q][.] with sum over Mv^T row q;
  // pass 2 computes the transposed product, whose results are X[q][n] for
  // several n, so its constant is per register and is added after the product
  const int kc1 = 128 * sum1 + (1 << (p.s_col - 1));
  const int off2 = 1 << (p.s_row - 1);
  int kc2r[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int n = 8 * (r >> 2) + 4 * h + (r & 3);
    int sm = 0;
    for (int c = 0; c < N; ++c) sm += mx::core_entry<N>(CH, true, n, c);
    kc2r[r] = 128 * sm + off2;
  }

  const int16_t* __restrict__ in = static_cast<const int16_t*>(p.in);
  int16_t* __restrict__ out = static_cast<int16_t*>(p.out);
  constexpr int RP = 40;   // row-major output tile pitch (halfwords)
  constexpr int CP = 34;   // column-major input tile pitch (halfwords)
  __shared__ __align__(16) uint16_t tile_all[4][N * RP];
  uint16_t* tile = tile_all[threadIdx.x >> 6];

  if (wave >= p.nblocks) return;
  uint4 g0 = reinterpret_cast<const uint4*>(in + wave * (N * N))[lane];
  uint4 g1 = reinterpret_cast<const uint4*>(in + wave * (N * N))[lane + 64];
  for (int64_t blk = wave; blk < p.nblocks; blk += nwaves) {
    // scatter this block column-major: chunk c is row c/4, columns 8(c%4)..+7
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int c = lane + 64 * half;
      const uint4 v = half ? g1 : g0;
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      const int r0 = c >> 2, c0 = (c & 3) * 8;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        tile[(c0 + 2 * k) * CP + r0] = (uint16_t)w[k];
        tile[(c0 + 2 * k + 1) * CP + r0] = (uint16_t)(w[k] >> 16);
      }
    }
    const int64_t nxt = blk + nwaves < p.nblocks ? blk + nwaves : blk;
    g0 = reinterpret_cast<const uint4*>(in + nxt * (N * N))[lane];
    g1 = reinterpret_cast<const uint4*>(in + nxt * (N * N))[lane + 64];
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_wave_barrier();
    // column q of Y, rows 16h..16h+15
    uint32_t ys[8];
    const uint32_t* col = reinterpret_cast<const uint32_t*>(tile + q * CP + 16 * h);
#pragma unroll
    for (int j = 0; j < 8; ++j) ys[j] = col[j];
    mx::Planes x1;
    mx::split_planes(ys, x1.h, x1.l);
    int z[16];
    mx::product(x1, m1, kc1, z);
    uint32_t us[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) us[j] = satpk(z[2 * j] >> p.s_col, z[2 * j + 1] >> p.s_col);
    mx::Planes x2;
    mx::split_planes(us, x2.h, x2.l);
    // D2[n][i] = sum_c Mh^T[n][c] U[i][c]: A = table rows, B = U rows
    int y[16];
    {
      const mx::i16v zero = {};
      const mx::i16v p1 = mx::mfma(m2.h, x2.h, zero);
      mx::i16v p2 = mx::mfma(m2.l, x2.h, zero);
      p2 = mx::mfma(m2.h, x2.l, p2);
      const mx::i16v p3 = mx::mfma(m2.l, x2.l, zero);
#pragma unroll
      for (int r = 0; r < 16; ++r) y[r] = (((p1[r] << 8) + p2[r]) << 8) + p3[r] + kc2r[r];
    }
    // lane (q, h), register r: X[q][m_r]; rows of D2 are n = m_r, columns i = q
    __builtin_amdgcn_wave_barrier();
    uint16_t* xr = tile + q * RP + 4 * h;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const uint32_t lo = satpk(y[4 * a] >> p.s_row, y[4 * a + 1] >> p.s_row);
      const uint32_t hi = satpk(y[4 * a + 2] >> p.s_row, y[4 * a + 3] >> p.s_row);
      *reinterpret_cast<uint2*>(xr + 8 * a) = make_uint2(lo, hi);
    }
    __builtin_amdgcn_wave_barrier();
    uint4* xo = reinterpret_cast<uint4*>(out + blk * (N * N));
    auto chunk_addr = [&](int c) { return (c >> 2) * RP + (c & 3) * 8; };
    xo[lane] = *reinterpret_cast<const uint4*>(tile + chunk_addr(lane));
    xo[lane + 64] = *reinterpret_cast<const uint4*>(tile + chunk_addr(lane + 64));
    __builtin_amdgcn_wave_barrier();
  }
}

#define TA_MX_INV(CH, CV)                                                                          \
  {{1, 0, 5, 5, CH, ADJ_NONE, 0, CV, ADJ_NONE, 0},                                                \
   reinterpret_cast<const void*>(&mx_inv<CH, CV>), 4, 256, kMaxWgs, false}

#define TA_MX_FWD(CH, KH, CV, KV, SAME)                                                            \
  {{0, 0, 5, 5, CH, KH ? ADJ_BAND : ADJ_NONE, KH, CV, KV ? ADJ_BAND : ADJ_NONE, KV},              \
   reinterpret_cast<const void*>(&mx_fwd<CH, KH, CV, KV, SAME>), 4, 256, kMaxWgs, SAME}

const KernelEntry kTable[] = {
    TA_MX_FWD(C_DST3, 4, C_DST3, 4, true),    // 32x32 adjusted DST-7, one band set
    TA_MX_FWD(C_DST3, 4, C_DST3, 4, false),   // 32x32 adjusted DST-7
    TA_MX_FWD(C_DCT3, 4, C_DCT3, 4, true),    // 32x32 adjusted DCT-8, one band set
    TA_MX_FWD(C_DCT3, 4, C_DCT3, 4, false),
    TA_MX_FWD(C_DST3, 6, C_DST3, 6, true),    // 32x32 DST-3 + 6-tap band
    TA_MX_FWD(C_DST3, 6, C_DST3, 6, false),
    TA_MX_FWD(C_DST7, 0, C_DST7, 0, false),   // 32x32 direct DST-7
    TA_MX_FWD(C_DCT8, 0, C_DCT8, 0, false),   // 32x32 direct DCT-8
    TA_MX_FWD(C_DCT2, 0, C_DCT2, 0, false),   // 32x32 DCT-2
    TA_MX_INV(C_DST7, C_DST7),                // inverse direct DST-7
    TA_MX_INV(C_DCT8, C_DCT8),                // inverse direct DCT-8
    TA_MX_INV(C_DCT2, C_DCT2),                // inverse DCT-2
};

}  // namespace

const KernelEntry* mfma_kernels(int* count) {
  *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

}  // namespace ta
