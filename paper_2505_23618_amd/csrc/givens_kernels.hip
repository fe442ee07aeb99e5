// Differentiable FP32 path: y = B A(theta) x over a batch of 1-D vectors,
// A(theta) = G_{L-1} ... G_0 a band of L layers of parallel Givens rotations
// on adjacent pairs (layer l rotates (l mod 2 + 2j, l mod 2 + 2j + 1);
// rotation (p, p+1) by t: v_p = c u_p - s u_{p+1}, v_{p+1} = s u_p + c u_{p+1}),
// B = DCT-2 or DST-3.  Angles are numbered layer by layer, pairs in order.
//
// Backward (for dL/dy = gy): the layer outputs are recomputed from x (no
// stored activations), g = B^T gy, then for l = L-1 .. 0:
//   dL/dt (pair p) += -g_p v_{p+1} + g_{p+1} v_p   (v = output of layer l)
//   g <- G_l^T g;
// finally dL/dx = g.  Angle gradients are summed per vector in registers,
// reduced across the workgroup with wave shuffles and LDS in a fixed order
// into one partial row per workgroup, and the partial rows are summed in a
// fixed order by a second kernel: the result is bitwise reproducible.
#include <mutex>
#include <type_traits>

#include "fp.hpp"
#include "kernels.hpp"

namespace ta {
namespace {


template <int N, int L>
constexpr int n_angles() {
  int c = 0;
  for (int l = 0; l < L; ++l) c += (N - 2 - (l & 1)) / 2 + 1;
  return c;
}

static_assert(n_angles<32, 2>() == 31 && n_angles<32, 3>() == 47 && n_angles<16, 2>() == 15, "angles");

template <int N>
TA_DEV void load_vec(const float* __restrict__ src, float (&v)[N]) {
#pragma unroll
  for (int q = 0; q < N / 4; ++q) {
    const float4 t = reinterpret_cast<const float4*>(src)[q];
    v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
  }
}

template <int N>
TA_DEV void store_vec(float* __restrict__ dst, const float (&v)[N]) {
#pragma unroll
  for (int q = 0; q < N / 4; ++q)
    reinterpret_cast<float4*>(dst)[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// cos/sin of every angle into LDS (one transcendental pair per angle per workgroup)
template <int NA>
TA_DEV void angle_table(const float* __restrict__ theta, float (&cs)[2][kMaxAng]) {
  if (threadIdx.x < NA) {
    float s, c;
    sincosf(theta[threadIdx.x], &s, &c);
    cs[0][threadIdx.x] = c;
    cs[1][threadIdx.x] = s;
  }
  __syncthreads();
}

template <int N, int LAYER>
TA_DEV void rotate(float (&v)[N], const float (&cs)[2][kMaxAng], int r0) {
  int r = r0;
#pragma unroll
  for (int p = (LAYER & 1); p + 1 < N; p += 2, ++r) {
    const float c = cs[0][r], s = cs[1][r];
    const float a = v[p], b = v[p + 1];
    v[p] = c * a - s * b;
    v[p + 1] = s * a + c * b;
  }
}

template <int N, int LAYER>
TA_DEV void rotate_t(float (&g)[N], const float (&cs)[2][kMaxAng], int r0) {
  int r = r0;
#pragma unroll
  for (int p = (LAYER & 1); p + 1 < N; p += 2, ++r) {
    const float c = cs[0][r], s = cs[1][r];
    const float a = g[p], b = g[p + 1];
    g[p] = c * a + s * b;
    g[p + 1] = -s * a + c * b;
  }
}

template <int N, int LAYER>
constexpr int first_angle() {
  int c = 0;
  for (int l = 0; l < LAYER; ++l) c += (N - 2 - (l & 1)) / 2 + 1;
  return c;
}

template <int N, int L, int I = 0>
TA_DEV void apply_layers(float (&v)[N], const float (&cs)[2][kMaxAng]) {
  if constexpr (I < L) {
    rotate<N, I>(v, cs, first_angle<N, I>());
    apply_layers<N, L, I + 1>(v, cs);
  }
}

template <int N, int L, int BASE>
__global__ __launch_bounds__(256) void givens_fwd(GivensArgs a) {
  constexpr int NA = n_angles<N, L>();
  __shared__ float cs[2][kMaxAng];
  angle_table<NA>(a.theta, cs);
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= a.nvec) return;
  float v[N];
  load_vec<N>(a.x + m * N, v);
  apply_layers<N, L>(v, cs);
  fp::Vec<N> u;
#pragma unroll
  for (int i = 0; i < N; ++i) u.v[i] = v[i];
  const fp::Vec<N> y = fp::core<N, BASE, false>(u);
  store_vec<N>(a.y + m * N, y.v);
}

template <int N, int L, int BASE>
__global__ __launch_bounds__(256) void givens_bwd(GivensArgs a) {
  constexpr int NA = n_angles<N, L>();
  __shared__ float cs[2][kMaxAng];
  __shared__ float red[4][kMaxAng];
  angle_table<NA>(a.theta, cs);
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool act = m < a.nvec;
  float gt[NA];
#pragma unroll
  for (int r = 0; r < NA; ++r) gt[r] = 0.0f;
  if (act) {
    // forward recompute: out[l] = output of layer l
    float out[L][N];
    float v[N];
    load_vec<N>(a.x + m * N, v);
    rotate<N, 0>(v, cs, 0);
#pragma unroll
    for (int i = 0; i < N; ++i) out[0][i] = v[i];
    if constexpr (L > 1) {
      rotate<N, 1>(v, cs, first_angle<N, 1>());
#pragma unroll
      for (int i = 0; i < N; ++i) out[1][i] = v[i];
    }
    if constexpr (L > 2) {
      rotate<N, 2>(v, cs, first_angle<N, 2>());
#pragma unroll
      for (int i = 0; i < N; ++i) out[2][i] = v[i];
    }
    // g = B^T gy
    fp::Vec<N> gyv;
    load_vec<N>(a.gy + m * N, gyv.v);
    const fp::Vec<N> g0 = fp::core<N, BASE, true>(gyv);
    float g[N];
#pragma unroll
    for (int i = 0; i < N; ++i) g[i] = g0.v[i];
    // layers in reverse
    auto layer_back = [&](auto layer_tag) {
      constexpr int LY = decltype(layer_tag)::value;
      int r = first_angle<N, LY>();
#pragma unroll
      for (int p = (LY & 1); p + 1 < N; p += 2, ++r)
        gt[r] = -g[p] * out[LY][p + 1] + g[p + 1] * out[LY][p];
      rotate_t<N, LY>(g, cs, first_angle<N, LY>());
    };
    if constexpr (L > 2) layer_back(std::integral_constant<int, 2>{});
    if constexpr (L > 1) layer_back(std::integral_constant<int, 1>{});
    layer_back(std::integral_constant<int, 0>{});
    store_vec<N>(a.gx + m * N, g);
  }
  // workgroup reduction of the angle gradients, fixed order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    float s = gt[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wv][r] = s;
  }
  __syncthreads();
  if (threadIdx.x < NA) {
    const int r = threadIdx.x;
    a.partial[(int64_t)blockIdx.x * kMaxAng + r] = ((red[0][r] + red[1][r]) + red[2][r]) + red[3][r];
  }
}

// Sum of the per-workgroup partial rows, one workgroup per angle: thread t
// adds rows t, t + 256, ... in order, then a fixed-shape tree over the 256
// thread sums; the order never depends on timing, so the result is bitwise
// reproducible.
__global__ __launch_bounds__(256) void givens_reduce(const float* __restrict__ partial, int64_t groups, int na,
                                                     float* __restrict__ gtheta) {
  __shared__ float sum[256];
  const int r = blockIdx.x, t = threadIdx.x;
  if (r >= na) return;
  float s = 0.0f;
  for (int64_t g = t; g < groups; g += 256) s += partial[g * kMaxAng + r];
  sum[t] = s;
  __syncthreads();
#pragma unroll
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sum[t] += sum[t + w];
    __syncthreads();
  }
  if (t == 0) gtheta[r] = sum[0];
}

}  // namespace

// kernel lookup: n in {16, 32}, layers in {2, 3}, base DCT-2 (0) or DST-3 (3)
const void* givens_kernel(int bwd, int n, int layers, int base) {
#define TA_GV(NN, LL, BB)                                                                         \
  if (n == NN && layers == LL && base == BB)                                                      \
    return bwd ? reinterpret_cast<const void*>(&givens_bwd<NN, LL, BB>)                           \
               : reinterpret_cast<const void*>(&givens_fwd<NN, LL, BB>);
  TA_GV(32, 2, C_DCT2) TA_GV(32, 3, C_DCT2) TA_GV(32, 2, C_DST3) TA_GV(32, 3, C_DST3)
  TA_GV(16, 2, C_DCT2) TA_GV(16, 3, C_DCT2) TA_GV(16, 2, C_DST3) TA_GV(16, 3, C_DST3)
#undef TA_GV
  return nullptr;
}

const void* givens_reduce_kernel() { return reinterpret_cast<const void*>(&givens_reduce); }

// Scratch of the allocation-free backward: the per-workgroup partial rows of
// the angle gradient (kMaxAng floats each) for up to kNoAllocGroups
// workgroups.  Every device the library runs on holds its own copy until the
// process ends; every call on a device shares it.
static __device__ __align__(256) float scratch[kNoAllocGroups * kMaxAng];

// Device address of `scratch` on `device`, looked up once per device with
// that device current (the array's name in host code is only a stand-in for
// the symbol, never a device address).
int givens_scratch(int device, float** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static float* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return -2;
    if (prev != device && hipSetDevice(device) != hipSuccess) return -2;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) return -2;
    addr[device] = static_cast<float*>(p);
  }
  *ptr = addr[device];
  return 0;
}

}  // namespace ta
