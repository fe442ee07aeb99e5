// Statistics of quantised transform coefficients: the codec-free proxy for
// the coding results of the paper's experiments (Tables 2 and 3).  For a
// batch of H x W int16 coefficient blocks and a uniform quantiser
//   q = sign(y) floor((|y| + o) / step)
// the kernels produce, per coefficient position p = row * W + col, the count
// of every symbol (levels -31..31, and +-32 for the escapes |q| > 31), the
// Exp-Golomb suffix bits of the escapes, the energy sum y^2 and the
// distortion sum (y - q step)^2; then the rate of each position (entropy of
// its symbols plus its mean suffix length) and a summary (mean rate,
// distortion and energy per coefficient, transform coding gain, low-band
// energy fraction, fractions of nonzero and escaped levels).
//
// The accumulation kernel streams the coefficients once and uses no global
// atomics.  A workgroup (4 waves) owns 64 consecutive positions (for blocks
// under 64 coefficients: 64 / P blocks side by side), so every wave load is
// one contiguous 128-byte line, and a contiguous range of blocks, dealt to
// its waves in turn.  Each lane owns one position and keeps, in its own LDS
// row, 16-bit counters for the 65 symbols (two per dword, incremented by LDS
// atomic adds that never carry: the host bounds every count below 2^16) and
// its sums in registers.  At the end the workgroup folds its rows per
// position and writes them, with the sums, as one partial result per (block
// range, position); a second kernel adds the partials of all ranges in a
// fixed order.
#include "kernels.hpp"

namespace ta {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = 4;
constexpr int kNear = 31;                 // |levels| counted as their own symbol
constexpr int kRow = kNear + 2;           // dwords per lane row: 32 level pairs + the escapes (odd pitch)
constexpr int kSym = 2 * kNear + 3;       // histogram columns: -32 (escape) .. +32 (escape)

__global__ __launch_bounds__(256) void stats_zero(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

struct Sample {
  uint32_t a;   // |y|
  uint32_t q;   // |level|
  int d;        // |y| - |level| step
};

// q = floor((|y| + o) / step) with 24-bit multiplies only: n = |y| + o < 2^16
// and magic = ceil(2^k / step) with 2^k >= 2^16 step make
// floor(n magic / 2^k) exact (the error n (magic - 2^k / step) / 2^k stays
// below 1 / step); magic < 2^18 and k <= 31, so the 48-bit product and one
// funnel shift of its two halves suffice.  Step 1 is magic 2^16, k = 16.
__device__ inline Sample quantise(int y, const StatsArgs& s) {
  Sample r;
  r.a = (uint32_t)(y < 0 ? -y : y);
  const uint32_t n = r.a + (uint32_t)s.offset;
  const uint64_t prod = (uint64_t)(n & 0xffffffu) * (uint64_t)(s.magic & 0xffffffu);
  r.q = __builtin_amdgcn_alignbit((uint32_t)(prod >> 32), (uint32_t)prod, (uint32_t)s.magic_shift);
  r.d = (int)r.a - (int)((uint32_t)(uint16_t)r.q * (uint32_t)(uint16_t)s.step);   // q < 2^16, step <= 2^15
  return r;
}

__global__ __launch_bounds__(256) void stats_accum(StatsArgs s) {
  __shared__ uint32_t cnt[kThreads * kRow];
  __shared__ unsigned long long sums[3 * kThreads];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);   // wave index, uniform by construction
  const int slab = blockIdx.x % s.slabs;
  const int64_t range = blockIdx.x / s.slabs;
  uint32_t* row = cnt + t * kRow;
#pragma unroll
  for (int j = 0; j < kRow; ++j) row[j] = 0;
  // a lane's row is its own until the fold below: no barrier before it

  const int64_t it0 = range * s.steps_per_wg;
  const int64_t it1 = min(it0 + s.steps_per_wg, s.steps);
  const int64_t wstride = s.wstride;
  uint64_t e_acc = 0, d_acc = 0;
  // suffix bits of an escape |q| >= 32: 2 floor(log2(|q| - 31)) + 1 = 2 f - 1
  // with f = floor(log2(|q| - 31)) + 1, the binary exponent of |q| - 31, and
  // f = 0 for every non-escape; so the lane sums f and subtracts its escape
  // count at the end (at most 2^16 samples of f <= 15)
  uint32_t f_acc = 0;

  // lane row: dword j < 32 counts level +j in its low half and -j in its high
  // half (both halves of dword 0 are level 0); dword 32 counts the escapes,
  // positive low, negative high
  auto count = [&](int y, const Sample& v) {
    const uint32_t inc = 1u + ((uint32_t)(y >> 31) & 0xffffu);   // 1 or 2^16
    atomicAdd(row + min(v.q, (uint32_t)(kNear + 1)), inc);
    const uint32_t x = __builtin_elementwise_sub_sat(v.q, (uint32_t)kNear);   // exact in fp32 (< 2^16)
    f_acc += (uint32_t)__builtin_amdgcn_frexp_expf((float)x);       // 0 for x = 0
  };
  auto add_sums = [&](const Sample& v0, const Sample& v1) {
    // two squares of at most 2^30 each fit 32 bits; |y|, |d| <= 2^15
    e_acc += (uint64_t)((uint32_t)__umul24(v0.a, v0.a) + (uint32_t)__umul24(v1.a, v1.a));
    d_acc += (uint64_t)((uint32_t)__mul24(v0.d, v0.d) + (uint32_t)__mul24(v1.d, v1.d));
  };

  // workgroup step `it` gives wave w the wave step k = 4 it + w: elements
  // k * wstride + slab * 64 + lane.  Steps below full_steps lie wholly inside
  // the batch for every wave; the rest are checked element by element.
  constexpr int U = 16;
  int64_t it = it0;
  const int64_t full_end = min(it1, s.full_steps);
  const int ustride = 2 * kWaves * (int)wstride;   // bytes between unrolled steps
  for (; it + U <= full_end; it += U) {
    // wave-uniform buffer at this wave's first element: the per-lane byte
    // offset is fixed and each unrolled step adds a scalar offset
    const int16_t* base = s.in + (kWaves * it + w) * wstride + slab * 64;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, U * ustride, 0x00020000);
    int y[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      y[u] = __builtin_bit_cast(int16_t, __builtin_amdgcn_raw_buffer_load_b16(rs, 2 * lane, u * ustride, 0));
#pragma unroll
    for (int u = 0; u < U; u += 2) {
      const Sample v0 = quantise(y[u], s), v1 = quantise(y[u + 1], s);
      add_sums(v0, v1);
      count(y[u], v0);
      count(y[u + 1], v1);
    }
  }
  const Sample none{0, 0, 0};
  for (; it < it1; ++it) {
    const int64_t k = kWaves * it + w;
    const int64_t e = k * wstride + slab * 64 + lane;
    if (k < s.wave_steps && e < s.total) {
      const int y = s.in[e];
      const Sample v = quantise(y, s);
      add_sums(v, none);
      count(y, v);
    }
  }

  // fold the rows of the lanes that share a position (4 waves, and 64 / P
  // lanes per wave for blocks under 64 coefficients) into one partial
  sums[t] = e_acc;
  sums[kThreads + t] = d_acc;
  const uint32_t esc = (row[kNear + 1] & 0xffffu) + (row[kNear + 1] >> 16);
  sums[2 * kThreads + t] = 2ull * f_acc - esc;
  __syncthreads();
  const int np = min(s.positions, 64);      // positions of this workgroup
  const int reps = kThreads / np;           // rows per position
  const int64_t pbase = range * s.positions + slab * 64;
  uint32_t* __restrict__ part = s.part + pbase * kRow;
  for (int i = t; i < np * kRow; i += kThreads) {
    const int pl = i / kRow, j = i - pl * kRow;
    uint32_t v = 0;
    for (int r = 0; r < reps; ++r) v += cnt[(pl + r * np) * kRow + j];
    part[i] = v;
  }
  if (t < np) {
    unsigned long long e = 0, d = 0, b = 0;
    for (int r = 0; r < reps; ++r) {
      e += sums[t + r * np];
      d += sums[kThreads + t + r * np];
      b += sums[2 * kThreads + t + r * np];
    }
    s.part_e[pbase + t] = e;
    s.part_d[pbase + t] = d;
    s.part_b[pbase + t] = b;
  }
}

// Adds the partials of all block ranges in range order: thread (p, j) writes
// the counts of levels +j and -j at position p (j = 32: the two escapes);
// 3 P more threads add the energy, distortion and suffix-bit sums.
__global__ __launch_bounds__(256) void stats_reduce(StatsArgs s) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)s.positions * kRow) {
    // the three sums: one thread per (position, sum)
    const int64_t k = i - (int64_t)s.positions * kRow;
    if (k >= 3 * (int64_t)s.positions) return;
    const int which = (int)(k / s.positions), p = (int)(k - (int64_t)which * s.positions);
    const uint64_t* src = which == 0 ? s.part_e : which == 1 ? s.part_d : s.part_b;
    uint64_t acc = 0;
    int64_t r = 0;
    for (; r + 8 <= s.ranges; r += 8) {
      uint64_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[(r + u) * s.positions + p];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; r < s.ranges; ++r) acc += src[r * s.positions + p];
    (which == 0 ? s.energy : which == 1 ? s.dist : s.esc_bits)[p] = acc;
    return;
  }
  const int p = (int)(i / kRow), j = (int)(i - (int64_t)p * kRow);
  const int64_t pstride = (int64_t)s.positions * kRow;
  uint32_t lo = 0, hi = 0;
  int64_t r = 0;
  for (; r + 8 <= s.ranges; r += 8) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = s.part[(r + u) * pstride + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      lo += v[u] & 0xffffu;
      hi += v[u] >> 16;
    }
  }
  for (; r < s.ranges; ++r) {
    const uint32_t v = s.part[r * pstride + i];
    lo += v & 0xffffu;
    hi += v >> 16;
  }
  uint32_t* h = s.hist + (int64_t)p * kSym + (kNear + 1);   // column of level 0
  if (j == 0) {
    h[0] = lo + hi;
  } else {
    h[j] = lo;
    h[-j] = hi;
  }
}

// Block-wide sum in a fixed order (deterministic for a given block size).
template <typename T>
__device__ inline T block_sum(T v, T* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const T r = red[0];
  __syncthreads();
  return r;
}

// One wave per position: R_p = log2 n - (1/n) sum_s c_s log2 c_s + bits_p / n,
// the 65 terms summed in a fixed butterfly order; also log2(E_p / n) for the
// coding gain.
__global__ __launch_bounds__(256) void stats_rate(StatsArgs s) {
  const int p = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= s.positions) return;
  const uint32_t* h = s.hist + (int64_t)p * kSym;
  const uint32_t c0 = h[lane];
  const uint32_t c1 = lane == 0 ? h[64] : 0u;
  double acc = (c0 ? (double)c0 * log2((double)c0) : 0.0) + (c1 ? (double)c1 * log2((double)c1) : 0.0);
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
  if (lane == 0) {
    const double n = (double)s.nblocks;
    s.rate[p] = s.nblocks > 0 ? log2(n) - acc / n + (double)s.esc_bits[p] / n : 0.0;
    s.log_energy[p] = log2((double)s.energy[p] / n);
  }
}

// One workgroup: the summary over all positions.
__global__ __launch_bounds__(256) void stats_summary(StatsArgs s) {
  __shared__ double red[kThreads];
  __shared__ unsigned long long redu[kThreads];
  const int t = threadIdx.x;
  const int qw = 1 << (s.log2w - 2), qh = 1 << (s.log2h - 2);   // low band: (H/4) x (W/4)
  double rsum = 0.0, lsum = 0.0;
  unsigned long long esum = 0, dsum = 0, elow = 0, zeros = 0, escapes = 0;
  for (int p = t; p < s.positions; p += kThreads) {
    const uint64_t e = s.energy[p];
    const uint32_t* h = s.hist + (int64_t)p * kSym;
    rsum += s.rate[p];
    esum += e;
    dsum += s.dist[p];
    if ((p >> s.log2w) < qh && (p & ((1 << s.log2w) - 1)) < qw) elow += e;
    zeros += h[kNear + 1];
    escapes += h[0] + h[kSym - 1];
    lsum += s.log_energy[p];
  }
  rsum = block_sum(rsum, red);
  lsum = block_sum(lsum, red);
  esum = block_sum(esum, redu);
  dsum = block_sum(dsum, redu);
  elow = block_sum(elow, redu);
  zeros = block_sum(zeros, redu);
  escapes = block_sum(escapes, redu);
  if (t == 0) {
    double* o = s.summary;
    if (s.nblocks == 0) {
      for (int i = 0; i < 7; ++i) o[i] = 0.0;
      return;
    }
    const double ncoef = (double)s.nblocks * (double)s.positions;
    const double etot = (double)esum;
    o[0] = rsum / s.positions;
    o[1] = (double)dsum / ncoef;
    o[2] = etot / ncoef;
    o[3] = esum ? 10.0 * log10((etot / ncoef) / exp2(lsum / s.positions)) : 0.0;
    o[4] = esum ? (double)elow / etot : 0.0;
    o[5] = (ncoef - (double)zeros) / ncoef;
    o[6] = (double)escapes / ncoef;
  }
}

}  // namespace

const void* stats_kernel(int which) {
  switch (which) {
    case 0: return reinterpret_cast<const void*>(&stats_zero);
    case 1: return reinterpret_cast<const void*>(&stats_accum);
    case 2: return reinterpret_cast<const void*>(&stats_rate);
    case 3: return reinterpret_cast<const void*>(&stats_summary);
    case 4: return reinterpret_cast<const void*>(&stats_reduce);
    default: return nullptr;
  }
}

}  // namespace ta
