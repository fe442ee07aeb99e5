// libtadj host side: context, parameter registration, validation, dispatch.
// Implements the C ABI declared in include/tadj.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <utility>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tadj.h"
#include "kernels.hpp"
#include "tables_gen.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// Host allocations sized by the caller (descriptor copies, plan state,
// comparison buffers) must not let an exception cross the C ABI.
template <class F>
int guard(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(TA_EINVAL, "host memory allocation failed (sizes too large?)");
  } catch (...) {
    return fail(TA_EHIP, "unexpected host exception");
  }
}

#define TA_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) return fail(TA_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Makes `dev` the calling thread's current device for the guard's lifetime
// and restores the caller's device afterwards: library calls never change
// which device the caller's thread has current.
class DeviceGuard {
 public:
  DeviceGuard() = default;
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
  hipError_t enter(int dev) {
    hipError_t e = hipGetDevice(&prev_);
    if (e != hipSuccess) return e;
    if (prev_ == dev) return hipSuccess;
    e = hipSetDevice(dev);
    if (e == hipSuccess) switched_ = true;
    return e;
  }
  ~DeviceGuard() {
    if (switched_) (void)hipSetDevice(prev_);
  }

 private:
  int prev_ = -1;
  bool switched_ = false;
};

// Run the rest of the enclosing scope on device `dev` (see DeviceGuard).
#define TA_ON_DEVICE(dev)          \
  DeviceGuard device_guard_;       \
  TA_HIP(device_guard_.enter(dev))

constexpr int kMaxIds = 256;

// Device copies of one parameter set in the four orientations the kernels
// use: forward / transposed, plain / flipped (DCT-8 version).
struct ParamSet {
  int kind = 0;  // TA_ADJ_BAND or TA_ADJ_POST
  int n = 0, kb = 0;
  // fixed point (packed int16 pairs) and fp32; index [flip][transposed]
  void* fx[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  void* f32[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  // sub-block sets: Q (forward, unflipped) as even/odd column pairs, for the
  // simultaneous DST-7 / DCT-8 adjustment
  void* fx_eo = nullptr;
  // sub-block sets of a side without a compiled general stage (B not in
  // {4, 8, 16}): C = blkdiag(Q, 2^a I) (fixed point) and blkdiag(Q, I)
  // (fp32) as dense n x n matrices, [flip][transposed]
  void* dense_fx[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  void* dense_f32[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  // sets registered by their angles (ta_set_band_angles / ta_set_post_angles),
  // for ta_transform_bwd: the angles and Q0 (device, fp64) and the workspace
  // of per-workgroup partial matrix gradients
  int nang = 0;
  double* ang_dev = nullptr;
  double* q0_dev = nullptr;
  float* part_dev = nullptr;
  int part_groups = 0;
};

struct AxisCfg {
  bool set = false;
  ta_axis user{};
};

int core_flip(int base) {
  // S B R for the base kinds (eq. 3, eq. 4): DCT-2 and DST-2 are unchanged,
  // DCT-3 <-> DST-3, DST-7 <-> DCT-8.
  switch (base) {
    case TA_DCT2: return TA_DCT2;
    case TA_DST2: return TA_DST2;
    case TA_DCT3: return TA_DST3;
    case TA_DST3: return TA_DCT3;
    case TA_DST7: return TA_DCT8;
    case TA_DCT8: return TA_DST7;
  }
  return -1;
}

}  // namespace

struct ta_ctx {
  int device = 0;
  int bd = 8, m = 8, a = 10;
  int impl = 0;   // 0 automatic (matrix cores where built), 1 matrix cores only, 2 VALU only
  ParamSet params[kMaxIds];
  AxisCfg axes[kMaxIds];
  // device table of the batched kinds of every (axis id, log2 size), read by
  // the block-list kernels; kind -1 where the axis has no batched kernel
  ta::AxisDev* axes_dev = nullptr;
  // this device's static scratch (ta_givens_bwd_noalloc), looked up at create
  float* scratch = nullptr;
  // general kernels: integer base tables of precision m as dense matrices
  // (packed pairs), [TA_DCT2..TA_DCT8][transposed][log2 n], and the fp32
  // direct DST-7 / DCT-8, [0 DST-7, 1 DCT-8][transposed][log2 n]
  const void* dense_core[6][2][ta::kAxisSizes] = {};
  const void* direct_f32[2][2][ta::kAxisSizes] = {};
  // stage programs of every (axis id, log2 size, direction), one device
  // table per dtype (kAxisIds x kAxisSizes x 2; nst = 0 where the axis does
  // not resolve), and which entries have no fast batched kind
  ta::GenProg* gprogs_dev[2] = {nullptr, nullptr};
  bool general[kMaxIds][ta::kAxisSizes] = {};
  int ngeneral = 0;
  // per axis id: its parameter set, flip and adjustment (param id | flip << 8
  // | adjustment << 9), or -1 without an adjustment (read by the backward)
  int32_t* axis_use_dev = nullptr;
  std::vector<void*> allocations;
  std::mutex mu;
};

namespace {

int upload(ta_ctx* c, const void* host, size_t bytes, void** dev) {
  void* p = nullptr;
  TA_ON_DEVICE(c->device);
  TA_HIP(hipMalloc(&p, bytes));
  c->allocations.push_back(p);
  TA_HIP(hipMemcpy(p, host, bytes, hipMemcpyHostToDevice));
  *dev = p;
  return TA_OK;
}

int log2_exact(int n) {
  for (int l = 0; l < 31; ++l)
    if ((1 << l) == n) return l;
  return -1;
}

// Window start of row i of a K-tap band A = G_{L-1}...G_0 (L = K/2 layers of
// adjacent Givens rotations, layer l on pairs starting at l mod 2) or of its
// transpose.  Row i of a product of layers is {i} expanded by the layers in
// the order they are met from the left: A meets layer L-1 first, A^T meets
// layer 0 (even pairs) first; each expansion widens the window by one on
// both sides after the first, which picks the pair containing i.
int band_start(int i, int k, bool tr) {
  const int l = k / 2;
  return tr ? i - l + 1 - (i & 1) : i - l + ((i + l) & 1);
}

uint32_t pack2(int lo, int hi) {
  return (uint32_t)(uint16_t)(int16_t)lo | ((uint32_t)(uint16_t)(int16_t)hi << 16);
}

struct Resolved {
  int core, adj, kb;
  const void* pf;  // forward-orientation parameters
  const void* pi;  // transposed parameters
  const void* pdf; // sub-block as a dense n x n matrix (sides without a compiled general stage)
  const void* pdi;
  bool operator<(const Resolved& o) const {
    return std::tie(core, adj, kb, pf, pi, pdf, pdi) < std::tie(o.core, o.adj, o.kb, o.pf, o.pi, o.pdf, o.pdi);
  }
};

// Turn a user axis into the kernel's (core, adjustment, K/B, parameters).
int resolve_axis(ta_ctx* c, int id, int n, int dtype, Resolved* r) {
  if (id < 0 || id >= kMaxIds || !c->axes[id].set) return fail(TA_ENOPARAMS, "axis %d not registered", id);
  const ta_axis& u = c->axes[id].user;
  const int core = u.flip ? core_flip(u.base) : u.base;
  r->core = core;
  r->adj = u.adj;
  r->kb = 0;
  r->pf = r->pi = r->pdf = r->pdi = nullptr;
  if (u.adj == TA_ADJ_NONE) return TA_OK;
  const ParamSet& ps = c->params[u.param_id];
  if (ps.kind != u.adj) return fail(TA_ENOPARAMS, "axis %d: parameter set %d missing or of another kind", id, u.param_id);
  if (ps.n != n)
    return fail(TA_EUNSUPPORTED, "axis %d: parameter set %d is for size %d, block needs %d", id, u.param_id, ps.n, n);
  r->kb = ps.kb;
  const int f = u.flip ? 1 : 0;
  r->pf = dtype == TA_I16 ? ps.fx[f][0] : ps.f32[f][0];
  r->pi = dtype == TA_I16 ? ps.fx[f][1] : ps.f32[f][1];
  r->pdf = dtype == TA_I16 ? ps.dense_fx[f][0] : ps.dense_f32[f][0];
  r->pdi = dtype == TA_I16 ? ps.dense_fx[f][1] : ps.dense_f32[f][1];
  return TA_OK;
}

// Sub-block sides with a compiled stage in the general kernels.
bool gen_post_side(int b) { return b == 4 || b == 8 || b == 16; }

// The stage program of a resolved axis at size 2^l (section 2.2, eq. 1):
// forward [A, B] for a band, [B, C] for a sub-block, [B] without adjustment;
// the inverse runs the transposed stages in reverse order.  Butterfly cores
// transpose by kind (DCT-2 <-> DCT-3, DST-2 <-> DST-3); the direct DST-7 /
// DCT-8 run as dense matrices.
ta::GenProg gen_prog(const ta_ctx* c, const Resolved& r, int l, int dtype, int inv) {
  auto butterfly = [](int core) {
    switch (core) {
      case TA_DCT2: return (int)ta::GS_C2;
      case TA_DST2: return (int)ta::GS_S2;
      case TA_DCT3: return (int)ta::GS_C3;
      case TA_DST3: return (int)ta::GS_S3;
    }
    return -1;
  };
  auto transposed = [](int core) {
    switch (core) {
      case TA_DCT2: return (int)TA_DCT3;
      case TA_DCT3: return (int)TA_DCT2;
      case TA_DST2: return (int)TA_DST3;
      case TA_DST3: return (int)TA_DST2;
    }
    return core;
  };
  ta::GenStage core{};
  const int bop = butterfly(inv ? transposed(r.core) : r.core);
  if (bop >= 0 && (dtype == TA_F32 || c->m == 8)) {
    core.op = bop;                 // the butterflies hold the m = 8 tables
  } else {
    core.op = ta::GS_DENSE;
    core.p = dtype == TA_F32 ? c->direct_f32[r.core == TA_DCT8][inv][l] : c->dense_core[r.core][inv][l];
  }
  ta::GenProg pr{};
  if (r.adj == TA_ADJ_NONE) {
    pr.nst = 1;
    pr.st[0] = core;
    return pr;
  }
  ta::GenStage adj{};
  adj.adj = 1;
  if (r.adj == TA_ADJ_BAND) {
    adj.op = ta::GS_BAND;
    adj.arg = r.kb;
    adj.tr = inv;
    adj.p = inv ? r.pi : r.pf;
  } else if (gen_post_side(r.kb)) {
    adj.op = ta::GS_POST;
    adj.arg = r.kb;
    adj.p = inv ? r.pi : r.pf;
  } else {
    adj.op = ta::GS_DENSE;
    adj.p = inv ? r.pdi : r.pdf;
  }
  const bool adj_first = (r.adj == TA_ADJ_BAND) != (inv != 0);
  pr.nst = 2;
  pr.st[0] = adj_first ? adj : core;
  pr.st[1] = adj_first ? core : adj;
  return pr;
}

// kind of a resolved axis in the batched kernel (see batch_kernels.hip),
// whose butterflies hold the m = 8 tables; -1: the general kernel runs it
int batch_kind(const ta_ctx* c, const Resolved& r) {
  if (c->m != 8) return -1;
  if (r.core == TA_DCT2 && r.adj == TA_ADJ_NONE) return 0;
  if (r.core == TA_DST3 && r.adj == TA_ADJ_BAND && r.kb == 4) return 1;
  if (r.core == TA_DCT3 && r.adj == TA_ADJ_BAND && r.kb == 4) return 2;
  return -1;
}

// Rewrite the device axis-table row of axis `id`: for each log2 size the
// batched kind and the band tables, or kind -1.  Sizes the axis does not
// resolve at are expected (a band is registered for one size), so their
// messages are not left in the error slot.  Caller holds c->mu.
int refresh_axis(ta_ctx* c, int id) {
  ta::AxisDev row[ta::kAxisSizes];
  ta::GenProg progs[2][ta::kAxisSizes][2] = {};   // [dtype][log2 size][direction]
  const std::string saved = g_err;
  for (int l = 0; l < ta::kAxisSizes; ++l) {
    row[l] = ta::AxisDev{-1, 0, nullptr, nullptr, nullptr, nullptr};
    Resolved r, rf;
    const bool ok = l >= 2 && l <= 6 && c->axes[id].set && resolve_axis(c, id, 1 << l, TA_I16, &r) == TA_OK &&
                    resolve_axis(c, id, 1 << l, TA_F32, &rf) == TA_OK;
    if (ok && batch_kind(c, r) >= 0) {
      row[l].kind = batch_kind(c, r);
      row[l].pf = static_cast<const uint32_t*>(r.pf);
      row[l].pi = static_cast<const uint32_t*>(r.pi);
      row[l].ff = static_cast<const float*>(rf.pf);
      row[l].fi = static_cast<const float*>(rf.pi);
    }
    if (ok)
      for (int inv = 0; inv < 2; ++inv) {
        progs[0][l][inv] = gen_prog(c, r, l, TA_I16, inv);
        progs[1][l][inv] = gen_prog(c, rf, l, TA_F32, inv);
      }
    const bool gen = ok && batch_kind(c, r) < 0;
    c->ngeneral += (int)gen - (int)c->general[id][l];
    c->general[id][l] = gen;
  }
  g_err = saved;
  TA_ON_DEVICE(c->device);
  TA_HIP(hipMemcpy(c->axes_dev + (size_t)id * ta::kAxisSizes, row, sizeof row, hipMemcpyHostToDevice));
  for (int dt = 0; dt < 2; ++dt)
    TA_HIP(hipMemcpy(c->gprogs_dev[dt] + (size_t)id * ta::kAxisSizes * 2, progs[dt], sizeof progs[dt],
                     hipMemcpyHostToDevice));
  const ta_axis& u = c->axes[id].user;
  const int32_t use = (c->axes[id].set && u.adj != TA_ADJ_NONE) ? (u.param_id | (u.flip << 8) | (u.adj << 9)) : -1;
  TA_HIP(hipMemcpy(c->axis_use_dev + id, &use, sizeof use, hipMemcpyHostToDevice));
  return TA_OK;
}

// After parameter set `pid` changed: refresh every axis that uses it.
int refresh_param_users(ta_ctx* c, int pid) {
  for (int id = 0; id < kMaxIds; ++id) {
    const AxisCfg& ax = c->axes[id];
    if (ax.set && ax.user.adj != TA_ADJ_NONE && ax.user.param_id == pid) {
      int e;
      if ((e = refresh_axis(c, id))) return e;
    }
  }
  return TA_OK;
}

// Round half away from zero (the sign-symmetric rule of the integer tables).
int round_half_away(double v) { return v < 0 ? -(int)std::floor(-v + 0.5) : (int)std::floor(v + 0.5); }

// Orthonormal base matrices (rows = basis vectors, section 2.1): DCT-2 with
// e_0 = 1/sqrt 2, DST-7 and DCT-8 with sqrt(4 / (2N + 1)).
double base_entry(int kind, int n, int k, int j) {
  const double pi = 3.14159265358979323846;
  switch (kind) {
    case TA_DCT2: return std::sqrt(2.0 / n) * (k == 0 ? std::sqrt(0.5) : 1.0) * std::cos(pi * k * (2 * j + 1) / (2.0 * n));
    case TA_DST7: return std::sqrt(4.0 / (2 * n + 1)) * std::sin(pi * (2 * k + 1) * (j + 1) / (2.0 * n + 1));
    default: return std::sqrt(4.0 / (2 * n + 1)) * std::cos(pi * (2 * k + 1) * (2 * j + 1) / (4.0 * n + 2));
  }
}

// Integer base table of precision m (row-major n x n): round_half_away(2^m
// sqrt(n) T) for the DCT-2, DST-7 and DCT-8; DCT-3 = DCT-2^T, DST-2 = R DCT-2 S
// and DST-3 = S DCT-2^T R (section 2.1), exact in integers.
int int_table_entry(int kind, int n, int m, int k, int j) {
  auto c2 = [&](int kk, int jj) { return round_half_away(std::ldexp(std::sqrt((double)n), m) * base_entry(TA_DCT2, n, kk, jj)); };
  switch (kind) {
    case TA_DCT2: return c2(k, j);
    case TA_DCT3: return c2(j, k);
    case TA_DST2: return ((j & 1) ? -1 : 1) * c2(n - 1 - k, j);
    case TA_DST3: return ((k & 1) ? -1 : 1) * c2(n - 1 - j, k);
    default: return round_half_away(std::ldexp(std::sqrt((double)n), m) * base_entry(kind, n, k, j));
  }
}

// The general kernels' context tables: every base kind of every size as a
// dense matrix in both orientations (the direct DST-7 / DCT-8 always run
// dense; the butterfly kinds run dense in fixed point when m != 8, whose
// tables are not compiled into the butterflies), fp32 direct matrices, and
// the (empty) program tables.
int upload_general_tables(ta_ctx* c) {
  int e;
  for (int l = 2; l <= 6; ++l) {
    const int n = 1 << l;
    for (int kind = TA_DCT2; kind <= TA_DCT8; ++kind)
      for (int tr = 0; tr < 2; ++tr) {
        std::vector<uint32_t> fx((size_t)n * n / 2);
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n / 2; ++j) {
            const int r = tr ? 2 * j : k, c0 = tr ? k : 2 * j;
            const int r1 = tr ? 2 * j + 1 : k, c1 = tr ? k : 2 * j + 1;
            fx[(size_t)k * (n / 2) + j] = pack2(int_table_entry(kind, n, c->m, r, c0), int_table_entry(kind, n, c->m, r1, c1));
          }
        void* p = nullptr;
        if ((e = upload(c, fx.data(), fx.size() * 4, &p))) return e;
        c->dense_core[kind][tr][l] = p;
        if (kind >= TA_DST7) {
          std::vector<float> f32((size_t)n * n);
          for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) f32[(size_t)k * n + j] = (float)(tr ? base_entry(kind, n, j, k) : base_entry(kind, n, k, j));
          if ((e = upload(c, f32.data(), f32.size() * 4, &p))) return e;
          c->direct_f32[kind == TA_DCT8][tr][l] = p;
        }
      }
  }
  std::vector<ta::GenProg> empty((size_t)ta::kAxisIds * ta::kAxisSizes * 2, ta::GenProg{});
  for (int dt = 0; dt < 2; ++dt) {
    void* p = nullptr;
    if ((e = upload(c, empty.data(), empty.size() * sizeof(ta::GenProg), &p))) return e;
    c->gprogs_dev[dt] = static_cast<ta::GenProg*>(p);
  }
  std::vector<int32_t> unused(ta::kAxisIds, -1);
  void* p = nullptr;
  if ((e = upload(c, unused.data(), unused.size() * sizeof(int32_t), &p))) return e;
  c->axis_use_dev = static_cast<int32_t*>(p);
  return TA_OK;
}

const ta::KernelEntry* find_kernel(const ta::KernelKey& key, int prefer_mfma, bool mfma_only, bool same) {
  int cnt = 0;
  // Automatic selection uses the matrix-core kernels only where they are the
  // faster ones on gfx950: cores without a band adjustment.  With a band the
  // per-lane tap registers limit occupancy and the VALU butterfly kernels win
  // (both are exact; impl 1 forces the matrix-core kernels).
  const bool band = key.adj_h == TA_ADJ_BAND || key.adj_v == TA_ADJ_BAND;
  if (prefer_mfma && key.dtype == TA_I16 && (mfma_only || !band)) {
    const ta::KernelEntry* t = ta::mfma_kernels(&cnt);
    for (int i = 0; i < cnt; ++i)
      if (t[i].key == key && (!t[i].same_params || same)) return &t[i];
  }
  if (mfma_only) return nullptr;
  const ta::KernelEntry* t = key.dtype == TA_I16 ? ta::fx_kernels(&cnt) : ta::f32_kernels(&cnt);
  for (int i = 0; i < cnt; ++i)
    if (t[i].key == key) return &t[i];
  return nullptr;
}

// Workgroups of kernel k that are resident on device `dev` at once (the grid
// of a persistent kernel): occupancy per CU times the CU count, cached.
int resident_groups(const void* fn, int threads, int dev, int* out) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(fn, dev);
  auto it = cache.find(key);
  if (it == cache.end()) {
    int per_cu = 0, cus = 0;
    TA_ON_DEVICE(dev);
    TA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0));
    TA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (per_cu < 1 || cus < 1) return fail(TA_EHIP, "kernel occupancy query returned %d x %d", per_cu, cus);
    it = cache.emplace(key, per_cu * cus).first;
  }
  *out = it->second;
  return TA_OK;
}

int resident_groups(const ta::KernelEntry* k, int dev, int* out) { return resident_groups(k->fn, k->threads, dev, out); }

// A packed batch without a specialised kernel: the general kernel, with the
// axes' stage programs from the context table, as a persistent grid over
// tiles of GenGeo::nb_for blocks.
int launch_general_packed(ta_ctx* c, int inv, int axis_h, int axis_v, int lw, int lh, int64_t nblocks,
                          const void* in, void* out, int dtype, ta_stream_t stream) {
  const bool f32 = dtype == TA_F32;
  ta::GenArgs g{};
  g.in = in;
  g.out = out;
  g.inv = inv;
  g.bd = c->bd;
  g.m = c->m;
  g.a = c->a;
  g.lw = lw;
  g.lh = lh;
  g.nblocks = nblocks;
  const ta::GenProg* t = c->gprogs_dev[f32];
  g.ph = t + ((size_t)axis_h * ta::kAxisSizes + lw) * 2 + inv;
  g.pv = t + ((size_t)axis_v * ta::kAxisSizes + lh) * 2 + inv;
  g.progs = t;
  const void* fn = ta::gen_kernel(0, f32);
  const int nb = ta::GenGeo::nb_for(lw, lh, f32);
  const int64_t tiles = (nblocks + nb - 1) / nb;
  int cap = 0, e;
  if ((e = resident_groups(fn, 256, c->device, &cap))) return e;
  const int64_t grid = std::min<int64_t>(tiles, cap);
  void* kargs[] = {&g};
  TA_ON_DEVICE(c->device);
  TA_HIP(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(256), kargs, 0, reinterpret_cast<hipStream_t>(stream)));
  return TA_OK;
}

int run_packed(ta_ctx* c, int inv, int axis_h, int axis_v, int log2w, int log2h, int64_t nblocks,
               const void* in, void* out, int dtype, ta_stream_t stream) {
  if (!c) return fail(TA_EINVAL, "null context");
  if (nblocks < 0) return fail(TA_EINVAL, "negative block count");
  if (dtype != TA_I16 && dtype != TA_F32) return fail(TA_EINVAL, "unknown dtype %d", dtype);
  if (log2w < 2 || log2w > 6 || log2h < 2 || log2h > 6)
    return fail(TA_EUNSUPPORTED, "block %dx%d: sizes must be 4..64", 1 << log2w, 1 << log2h);
  if (nblocks == 0) return TA_OK;
  if (!in || !out) return fail(TA_EINVAL, "null buffer");
  const size_t esz = dtype == TA_I16 ? 2 : 4;
  const size_t bytes = (size_t)nblocks << (log2w + log2h);
  const char* ib = static_cast<const char*>(in);
  const char* ob = static_cast<const char*>(out);
  if (ib < ob + bytes * esz && ob < ib + bytes * esz) return fail(TA_EINVAL, "input and output overlap");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(TA_EINVAL, "buffers must be 16-byte aligned");
  Resolved rh, rv;
  int e;
  if ((e = resolve_axis(c, axis_h, 1 << log2w, dtype, &rh))) return e;
  if ((e = resolve_axis(c, axis_v, 1 << log2h, dtype, &rv))) return e;
  const ta::KernelKey key{inv, dtype, log2w, log2h, rh.core, rh.adj, rh.kb, rv.core, rv.adj, rv.kb};
  const int prefer_mfma = c->impl != 2;
  const bool same = rh.pf == rv.pf && rh.pi == rv.pi && rh.kb == rv.kb;
  // the specialised fixed-point kernels hold the m = 8 tables
  const ta::KernelEntry* k = (dtype == TA_I16 && c->m != 8) ? nullptr : find_kernel(key, prefer_mfma, c->impl == 1, same);
  if (!k && c->impl == 1) return fail(TA_EUNSUPPORTED, "no matrix-core kernel for this transform");
  if (!k) return launch_general_packed(c, inv, axis_h, axis_v, log2w, log2h, nblocks, in, out, dtype, stream);
  ta::PackedArgs args;
  args.in = in;
  args.out = out;
  args.nblocks = nblocks;
  args.ph_f = rh.pf;
  args.ph_i = rh.pi;
  args.pv_f = rv.pf;
  args.pv_i = rv.pi;
  if (!inv) {
    args.s_row = log2w + c->bd + c->m - 15;
    args.s_col = log2h + c->m;
  } else {
    args.s_row = c->m + 14 - c->bd;
    args.s_col = c->m + 1;
  }
  args.a = c->a;
  int64_t groups = (nblocks + k->blocks_per_wg - 1) / k->blocks_per_wg;
  int cap = k->max_wgs;
  if (cap < 0 && (e = resident_groups(k, c->device, &cap))) return e;
  if (cap > 0 && groups > cap) groups = cap;
  if (groups > 0x7fffffff) return fail(TA_EUNSUPPORTED, "batch too large for one launch");
  void* kargs[] = {&args};
  TA_ON_DEVICE(c->device);
  TA_HIP(hipLaunchKernel(k->fn, dim3((unsigned)groups), dim3(k->threads), kargs, 0,
                         reinterpret_cast<hipStream_t>(stream)));
  return TA_OK;
}

}  // namespace

extern "C" {

const char* ta_version(void) { return "tadj 0.2 (gfx950)"; }

int ta_int_table(int kind, int n, int m, int16_t* out) {
  if (!out) return fail(TA_EINVAL, "null output");
  if (kind < TA_DCT2 || kind > TA_DCT8) return fail(TA_EINVAL, "kind %d", kind);
  if (log2_exact(n) < 2 || n > 64) return fail(TA_EUNSUPPORTED, "size %d", n);
  if (m < 6 || m > 9) return fail(TA_EUNSUPPORTED, "m=%d outside 6..9", m);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) out[k * n + j] = (int16_t)int_table_entry(kind, n, m, k, j);
  return TA_OK;
}

const char* ta_last_error(void) { return g_err.c_str(); }

int ta_create(ta_ctx** out, int device, int bit_depth, int m, int a) {
  if (!out) return fail(TA_EINVAL, "null output pointer");
  *out = nullptr;
  if (m < 6 || m > 9) return fail(TA_EUNSUPPORTED, "integer-matrix precision m=%d outside 6..9", m);
  if (bit_depth < 6 || bit_depth > 16) return fail(TA_EUNSUPPORTED, "bit depth %d outside 6..16", bit_depth);
  if (bit_depth + m < 14)
    return fail(TA_EUNSUPPORTED, "bit depth %d with m=%d: the 4-point forward row shift log2 4 + bd + m - 15 would be below 1",
                bit_depth, m);
  if (a < 6 || a > 14) return fail(TA_EUNSUPPORTED, "adjustment precision %d outside 6..14", a);
  int ndev = 0;
  TA_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(TA_EINVAL, "device %d not present (%d devices)", device, ndev);
  auto c = std::make_unique<ta_ctx>();
  c->device = device;
  c->bd = bit_depth;
  c->m = m;
  c->a = a;
  static_assert(kMaxIds == ta::kAxisIds, "axis table size");
  std::vector<ta::AxisDev> table((size_t)ta::kAxisIds * ta::kAxisSizes, ta::AxisDev{-1, 0, nullptr, nullptr, nullptr, nullptr});
  int e;
  if ((e = guard([&] { return upload(c.get(), table.data(), table.size() * sizeof(ta::AxisDev),
                                     reinterpret_cast<void**>(&c->axes_dev)); })) ||
      (e = guard([&] { return upload_general_tables(c.get()); }))) {
    for (void* p : c->allocations) (void)hipFree(p);
    return e;
  }
  {
    // the static scratch's address on this device, looked up once per device
    TA_ON_DEVICE(device);
    if (ta::givens_scratch(device, &c->scratch) != 0) {
      for (void* p : c->allocations) (void)hipFree(p);
      return fail(TA_EHIP, "static scratch address lookup failed on device %d", device);
    }
  }
  *out = c.release();
  return TA_OK;
}

int ta_destroy(ta_ctx* c) {
  if (!c) return fail(TA_EINVAL, "null context");
  DeviceGuard device_guard_;
  (void)device_guard_.enter(c->device);
  for (void* p : c->allocations) (void)hipFree(p);
  delete c;
  return TA_OK;
}

int ta_set_impl(ta_ctx* c, int impl) {
  if (!c) return fail(TA_EINVAL, "null context");
  if (impl < 0 || impl > 2) return fail(TA_EINVAL, "impl %d not in 0..2", impl);
  c->impl = impl;
  return TA_OK;
}

int ta_set_band(ta_ctx* c, int id, int n, int k, const int16_t* a_int, const float* a_f32) {
  if (!c || !a_int || !a_f32) return fail(TA_EINVAL, "null argument");
  if (id < 0 || id >= kMaxIds) return fail(TA_EINVAL, "parameter id %d outside 0..255", id);
  if (log2_exact(n) < 2 || n > 64) return fail(TA_EUNSUPPORTED, "band size %d", n);
  if (k != 2 && k != 4 && k != 6 && k != 8) return fail(TA_EUNSUPPORTED, "band taps %d not in {2,4,6,8}", k);
  // check the Givens-band support of A and its transpose
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int s = band_start(i, k, false);
      if ((j < s || j >= s + k) && (a_int[i * n + j] != 0 || a_f32[i * n + j] != 0.0f))
        return fail(TA_EUNSUPPORTED, "band entry (%d,%d) outside the %d-tap Givens band", i, j, k);
    }
  std::lock_guard<std::mutex> lk(c->mu);
  // the new tables are built aside and replace the registered set only once
  // every upload has succeeded (a failure keeps the previous set)
  ParamSet ps;
  ps.kind = TA_ADJ_BAND;
  ps.n = n;
  ps.kb = k;
  for (int flip = 0; flip < 2; ++flip)
    for (int tr = 0; tr < 2; ++tr) {
      // M = A (flip: R A R), transposed when tr.  M[i][j]:
      auto at = [&](int i, int j) -> int {
        int r = i, cc = j;
        if (tr) std::swap(r, cc);
        if (flip) { r = n - 1 - r; cc = n - 1 - cc; }
        return a_int[r * n + cc];
      };
      auto atf = [&](int i, int j) -> float {
        int r = i, cc = j;
        if (tr) std::swap(r, cc);
        if (flip) { r = n - 1 - r; cc = n - 1 - cc; }
        return a_f32[r * n + cc];
      };
      std::vector<uint32_t> packed(n * k / 2);
      std::vector<float> fl(n * k);
      for (int i = 0; i < n; ++i) {
        const int s = band_start(i, k, tr != 0);
        for (int t = 0; t < k / 2; ++t) {
          const int c0 = s + 2 * t, c1 = c0 + 1;
          const int v0 = (c0 >= 0 && c0 < n) ? at(i, c0) : 0;
          const int v1 = (c1 >= 0 && c1 < n) ? at(i, c1) : 0;
          packed[i * (k / 2) + t] = pack2(v0, v1);
        }
        for (int t = 0; t < k; ++t) {
          const int cc = s + t;
          fl[i * k + t] = (cc >= 0 && cc < n) ? atf(i, cc) : 0.0f;
        }
      }
      // every non-zero of M must sit inside its row window (true for Givens bands)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const int s = band_start(i, k, tr != 0);
          if ((j < s || j >= s + k) && (at(i, j) != 0 || atf(i, j) != 0.0f))
            return fail(TA_EUNSUPPORTED, "transposed band entry (%d,%d) outside the window", i, j);
        }
      int e;
      if ((e = upload(c, packed.data(), packed.size() * 4, &ps.fx[flip][tr]))) return e;
      if ((e = upload(c, fl.data(), fl.size() * 4, &ps.f32[flip][tr]))) return e;
    }
  c->params[id] = ps;
  return refresh_param_users(c, id);
}

int ta_set_post(ta_ctx* c, int id, int n, int b, const int16_t* q_int, const float* q_f32) {
  if (!c || !q_int || !q_f32) return fail(TA_EINVAL, "null argument");
  if (id < 0 || id >= kMaxIds) return fail(TA_EINVAL, "parameter id %d outside 0..255", id);
  if (log2_exact(n) < 2 || n > 64) return fail(TA_EUNSUPPORTED, "post size %d", n);
  if (b < 2 || b > n || (b & 1)) return fail(TA_EUNSUPPORTED, "sub-block %d for size %d", b, n);
  std::lock_guard<std::mutex> lk(c->mu);
  ParamSet ps;   // replaces the registered set once every upload succeeded
  ps.kind = TA_ADJ_POST;
  ps.n = n;
  ps.kb = b;
  for (int flip = 0; flip < 2; ++flip)
    for (int tr = 0; tr < 2; ++tr) {
      // M = Q (flip: S Q S, eq. 5), transposed when tr
      auto at = [&](int i, int j) -> int {
        const int r = tr ? j : i, cc = tr ? i : j;
        const int sg = (flip && ((r + cc) & 1)) ? -1 : 1;
        return sg * q_int[r * b + cc];
      };
      auto atf = [&](int i, int j) -> float {
        const int r = tr ? j : i, cc = tr ? i : j;
        const float sg = (flip && ((r + cc) & 1)) ? -1.0f : 1.0f;
        return sg * q_f32[r * b + cc];
      };
      std::vector<uint32_t> packed(b * b / 2);
      std::vector<float> fl(b * b);
      for (int i = 0; i < b; ++i) {
        for (int j = 0; j < b / 2; ++j) packed[i * (b / 2) + j] = pack2(at(i, 2 * j), at(i, 2 * j + 1));
        for (int j = 0; j < b; ++j) fl[i * b + j] = atf(i, j);
      }
      int e;
      if ((e = upload(c, packed.data(), packed.size() * 4, &ps.fx[flip][tr]))) return e;
      if ((e = upload(c, fl.data(), fl.size() * 4, &ps.f32[flip][tr]))) return e;
      if (!gen_post_side(b)) {
        // blkdiag(M, 2^a I) at shift a leaves the entries >= b exactly as
        // they are: RS(2^a y, a) = y
        std::vector<uint32_t> dfx((size_t)n * n / 2);
        std::vector<float> df((size_t)n * n, 0.0f);
        auto dent = [&](int i, int j) { return (i < b && j < b) ? at(i, j) : (i == j ? (1 << c->a) : 0); };
        for (int i = 0; i < n; ++i) {
          for (int j = 0; j < n / 2; ++j) dfx[(size_t)i * (n / 2) + j] = pack2(dent(i, 2 * j), dent(i, 2 * j + 1));
          for (int j = 0; j < n; ++j) df[(size_t)i * n + j] = (i < b && j < b) ? atf(i, j) : (i == j ? 1.0f : 0.0f);
        }
        if ((e = upload(c, dfx.data(), dfx.size() * 4, &ps.dense_fx[flip][tr]))) return e;
        if ((e = upload(c, df.data(), df.size() * 4, &ps.dense_f32[flip][tr]))) return e;
      }
    }
  if (b % 4 == 0) {
    // row i: (Q[i][4t], Q[i][4t+2]) for t < b/4, then (Q[i][4t+1], Q[i][4t+3])
    std::vector<uint32_t> eo(b * b / 2);
    for (int i = 0; i < b; ++i)
      for (int t = 0; t < b / 4; ++t) {
        eo[i * (b / 2) + t] = pack2(q_int[i * b + 4 * t], q_int[i * b + 4 * t + 2]);
        eo[i * (b / 2) + b / 4 + t] = pack2(q_int[i * b + 4 * t + 1], q_int[i * b + 4 * t + 3]);
      }
    int e;
    if ((e = upload(c, eo.data(), eo.size() * 4, &ps.fx_eo))) return e;
  }
  c->params[id] = ps;
  return refresh_param_users(c, id);
}

int ta_set_axis(ta_ctx* c, int id, const ta_axis* ax) {
  if (!c || !ax) return fail(TA_EINVAL, "null argument");
  if (id < 0 || id >= kMaxIds) return fail(TA_EINVAL, "axis id %d outside 0..255", id);
  if (ax->base < TA_DCT2 || ax->base > TA_DCT8) return fail(TA_EINVAL, "base %d", ax->base);
  if (ax->adj < TA_ADJ_NONE || ax->adj > TA_ADJ_POST) return fail(TA_EINVAL, "adjustment %d", ax->adj);
  if (ax->flip != 0 && ax->flip != 1) return fail(TA_EINVAL, "flip %d", ax->flip);
  if (ax->adj != TA_ADJ_NONE) {
    if (ax->base > TA_DST3) return fail(TA_EUNSUPPORTED, "DST-7/DCT-8 matrices take no adjustment");
    if (ax->param_id < 0 || ax->param_id >= kMaxIds || c->params[ax->param_id].kind != ax->adj)
      return fail(TA_ENOPARAMS, "parameter set %d not registered for this adjustment", ax->param_id);
  }
  std::lock_guard<std::mutex> lk(c->mu);
  c->axes[id].set = true;
  c->axes[id].user = *ax;
  return refresh_axis(c, id);
}

int ta_fwd_packed(ta_ctx* c, int axis_h, int axis_v, int log2w, int log2h, int64_t nblocks,
                  const void* in, void* out, int dtype, ta_stream_t stream) {
  return run_packed(c, 0, axis_h, axis_v, log2w, log2h, nblocks, in, out, dtype, stream);
}

int ta_inv_packed(ta_ctx* c, int axis_h, int axis_v, int log2w, int log2h, int64_t nblocks,
                  const void* in, void* out, int dtype, ta_stream_t stream) {
  return run_packed(c, 1, axis_h, axis_v, log2w, log2h, nblocks, in, out, dtype, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched uneven blocks: planning, autotuning, execution
// ---------------------------------------------------------------------------

struct ta_plan {
  const ta_ctx* ctx = nullptr;     // the context whose parameter tables the tiles point into
  int device = 0;
  int dtype = TA_I16;
  int region_log2 = 20;            // frame-region size of the tile lists (autotuned)
  // the validated descriptors and, per block, its class: the axes as resolved
  // when the plan was built (kinds and parameter tables), kept for re-planning
  std::vector<ta_block> host;
  std::vector<uint32_t> cls;
  struct Class { int lw, lh, kh, kv; Resolved rh, rv; };
  std::vector<Class> classes;
  // a plan with an axis kind outside the fast batched kernel's runs on the
  // general kernel: per class the stage programs h forward, h inverse,
  // v forward, v inverse
  bool general = false;
  ta::GenProg* progs_dev = nullptr;
  ta_plan() = default;
  ta_plan(const ta_plan&) = delete;
  ta_plan& operator=(const ta_plan&) = delete;
  ~ta_plan() {
    if (!blocks_dev && !tiles_dev && !progs_dev && !deltas_dev && !sched_dev) return;
    DeviceGuard device_guard_;
    (void)device_guard_.enter(device);
    if (blocks_dev) (void)hipFree(blocks_dev);
    if (tiles_dev) (void)hipFree(tiles_dev);
    if (progs_dev) (void)hipFree(progs_dev);
    if (deltas_dev) (void)hipFree(deltas_dev);
    if (sched_dev) (void)hipFree(sched_dev);
  }
  int64_t nblocks = 0, ntiles = 0;
  int grid = 2048;                 // persistent workgroups (autotuned)
  ta_block* blocks_dev = nullptr;  // block descriptors in plan order
  int32_t* deltas_dev = nullptr;   // (in_off - tile in_base, out_off - tile out_base) per block, plan order
  // tile counters of the int16 kernels' dynamic schedule: forward at 0,
  // inverse at kSchedStride (zero between launches)
  int32_t* sched_dev = nullptr;
  static constexpr int kSchedStride = ta::kSchedDwords;
  ta::BatchTile* tiles_dev = nullptr;
  int64_t max_in_elem = 0, max_out_elem = 0;   // extents touched (for validation)
  int64_t xstart[ta::kXcds + 1] = {};            // per-XCD tile lists
  int tile_blocks[7][7] = {};                    // blocks per tile by (log2 w, log2 h); 0: the kernels' maximum
};

namespace {

// The rules every block-list descriptor meets, shared by the planner and the
// validator (the unplanned kernels apply the same rules and skip a
// descriptor that breaks one): sizes 4..64, non-negative offsets, strides of
// at least the width, offsets and strides multiples of the vector width (8
// elements, 4 for 4-wide blocks), and axes with a batched kind at the size.
int check_block(ta_ctx* c, const ta_block& b, int64_t i, int dtype, Resolved* rh, Resolved* rv, int* kh, int* kv) {
  if (b.log2w < 2 || b.log2w > 6 || b.log2h < 2 || b.log2h > 6)
    return fail(TA_EUNSUPPORTED, "block %lld: size %dx%d outside 4..64", (long long)i, 1 << std::min<int>(b.log2w, 30),
                1 << std::min<int>(b.log2h, 30));
  const int w = 1 << b.log2w, ch = w >= 8 ? 8 : 4;
  if (b.in_off < 0 || b.out_off < 0 || b.in_stride < w || b.out_stride < w)
    return fail(TA_EINVAL, "block %lld: negative offset or stride below the width", (long long)i);
  if (b.in_off % ch || b.out_off % ch || b.in_stride % ch || b.out_stride % ch)
    return fail(TA_EUNSUPPORTED, "block %lld: offsets and strides must be multiples of %d elements", (long long)i, ch);
  int e;
  if ((e = resolve_axis(c, b.axis_h, w, dtype, rh)) || (e = resolve_axis(c, b.axis_v, 1 << b.log2h, dtype, rv))) {
    const std::string m = g_err;
    return fail(e, "block %lld: %s", (long long)i, m.c_str());
  }
  // -1: no fast batched kind, the block runs on the general kernel
  *kh = batch_kind(c, *rh);
  *kv = batch_kind(c, *rv);
  return TA_OK;
}

int launch_plan(ta_ctx* c, ta_plan* p, int inv, const void* in, void* out, ta_stream_t stream, int grid) {
  // at least one workgroup per XCD list
  const int64_t g = std::max<int64_t>(ta::kXcds, std::min<int64_t>(grid, std::max<int64_t>(1, p->ntiles)));
  if (p->general) {
    ta::GenArgs ga{};
    ga.tiles = p->tiles_dev;
    for (int x = 0; x <= ta::kXcds; ++x) ga.xstart[x] = p->xstart[x];
    ga.blocks = p->blocks_dev;
    ga.in = in;
    ga.out = out;
    ga.inv = inv;
    ga.bd = c->bd;
    ga.m = c->m;
    ga.a = c->a;
    void* kargs[] = {&ga};
    TA_ON_DEVICE(c->device);
    TA_HIP(hipLaunchKernel(ta::gen_kernel(0, p->dtype == TA_F32), dim3((unsigned)g), dim3(256), kargs, 0,
                           reinterpret_cast<hipStream_t>(stream)));
    return TA_OK;
  }
  ta::BatchArgs args{};
  args.tiles = p->tiles_dev;
  args.ntiles = p->ntiles;
  for (int x = 0; x <= ta::kXcds; ++x) args.xstart[x] = p->xstart[x];
  args.blocks = p->blocks_dev;
  args.deltas = p->deltas_dev;
  // The int16 kernels hand out tiles dynamically (per-direction counters)
  // when the whole grid is resident at once; a larger grid keeps the static
  // stride (its later workgroups start only as earlier ones finish, which
  // balances the load by itself).
  const void* fn = ta::batch_kernel(inv, 0, p->dtype == TA_F32);
  args.sched = nullptr;
  if (p->dtype == TA_I16 && p->sched_dev) {
    int res = 0, e;
    if ((e = resident_groups(fn, 256, c->device, &res))) return e;
    if (g <= res) args.sched = p->sched_dev + (inv ? ta_plan::kSchedStride : 0);
  }
  args.in = static_cast<const int16_t*>(in);
  args.out = static_cast<int16_t*>(out);
  args.bd = c->bd;
  args.m = c->m;
  args.a = c->a;
  void* kargs[] = {&args};
  TA_ON_DEVICE(c->device);
  TA_HIP(hipLaunchKernel(fn, dim3((unsigned)g), dim3(256), kargs, 0, reinterpret_cast<hipStream_t>(stream)));
  return TA_OK;
}

// The most blocks a tile of size (lw, lh) holds in the plan's kernel.
int max_tile_blocks(const ta_plan* plan, int lw, int lh) {
  const bool f32 = plan->dtype == TA_F32;
  return plan->general ? ta::GenGeo::nb_for(lw, lh, f32)
                       : f32 ? ta::BatchGeoF32::nb_for(lw, lh) : ta::BatchGeo::nb_planned(lw, lh);
}

// Blocks per tile for size (lw, lh): the per-size choice, else the maximum.
int tile_blocks(const ta_plan* plan, int lw, int lh) {
  const int m = max_tile_blocks(plan, lw, lh), c = plan->tile_blocks[lw][lh];
  return c > 0 && c < m ? c : m;
}

// Cut the plan's blocks into tiles: frame regions of 2^region_log2 input
// elements go round-robin to the XCD lists, an XCD's blocks are grouped by
// (size, class, strides) and cut into tiles of consecutive positions, and
// each list is ordered by tile position.  Replaces the plan's device
// descriptor, delta and tile arrays (synchronous, allocates).
int build_tiles(ta_plan* plan, int region_log2) {
  // regions (by input offset) go round-robin to the XCDs; an XCD's blocks are
  // grouped by (size, class, strides) across its regions, so that a group
  // leaves at most one partial tile, and each group is ordered by position
  const int64_t n = plan->nblocks;
  std::map<int64_t, int> region_xcd;
  for (int64_t i = 0; i < n; ++i) region_xcd.emplace(plan->host[(size_t)i].in_off >> region_log2, 0);
  {
    int r = 0;
    for (auto& kv : region_xcd) kv.second = r++ % ta::kXcds;
  }
  typedef std::tuple<int, int, int, uint32_t, int32_t, int32_t> Key;   // xcd, log2w, log2h, class, strides
  std::map<Key, std::vector<int64_t>> groups;
  for (int64_t i = 0; i < n; ++i) {
    const ta_block& b = plan->host[(size_t)i];
    groups[Key{region_xcd[b.in_off >> region_log2], b.log2w, b.log2h, plan->cls[(size_t)i], b.in_stride,
               b.out_stride}]
        .push_back(i);
  }
  std::vector<ta_block> ordered;
  std::vector<int32_t> deltas;
  // each XCD's tiles with the position of their first block
  std::vector<std::pair<int64_t, ta::BatchTile>> lists[ta::kXcds];
  ordered.reserve((size_t)n);
  deltas.reserve(2 * (size_t)n);
  for (auto& kv : groups) {
    const Key& k = kv.first;
    auto& idx = kv.second;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
      return plan->host[(size_t)x].in_off < plan->host[(size_t)y].in_off;
    });
    const int xcd = std::get<0>(k);
    const int lw = std::get<1>(k), lh = std::get<2>(k);
    const int32_t in_stride = std::get<4>(k), out_stride = std::get<5>(k);
    const size_t nb = (size_t)tile_blocks(plan, lw, lh);
    const uint32_t ci = std::get<3>(k);
    const ta_plan::Class& cl = plan->classes[ci];
    // a tile's blocks lie within 2^30 input elements of its base, counting
    // each block's extent, and within 2^31 output elements (int32 deltas)
    const int64_t ext_in = (int64_t)((1 << lh) - 1) * in_stride + (1 << lw);
    size_t s = 0;
    while (s < idx.size()) {
      int64_t in_lo = INT64_MAX, in_hi = INT64_MIN, out_lo = INT64_MAX, out_hi = INT64_MIN;
      size_t e = s;
      while (e < idx.size() && e - s < nb) {
        const ta_block& b = plan->host[(size_t)idx[e]];
        const int64_t il = std::min(in_lo, b.in_off), ih = std::max(in_hi, b.in_off);
        const int64_t ol = std::min(out_lo, b.out_off), oh = std::max(out_hi, b.out_off);
        if (e > s && (ih - il + ext_in > ((int64_t)1 << 30) || oh - ol > INT32_MAX)) break;
        in_lo = il, in_hi = ih, out_lo = ol, out_hi = oh;
        ++e;
      }
      ta::BatchTile t{};
      t.lw = lw;
      t.lh = lh;
      t.kind_h = cl.kh;
      t.kind_v = cl.kv;
      t.first = (int64_t)ordered.size();
      t.count = (int32_t)(e - s);
      t.in_stride = in_stride;
      t.out_stride = out_stride;
      t.in_base = in_lo;
      t.out_base = out_lo;
      if (plan->general) {
        // the class's stage programs (forward / inverse of each axis)
        const ta::GenProg* pr = plan->progs_dev + 4 * (size_t)ci;
        t.ph_f = reinterpret_cast<const uint32_t*>(pr + 0);
        t.ph_i = reinterpret_cast<const uint32_t*>(pr + 1);
        t.pv_f = reinterpret_cast<const uint32_t*>(pr + 2);
        t.pv_i = reinterpret_cast<const uint32_t*>(pr + 3);
      } else {
        t.ph_f = static_cast<const uint32_t*>(cl.rh.pf);
        t.ph_i = static_cast<const uint32_t*>(cl.rh.pi);
        t.pv_f = static_cast<const uint32_t*>(cl.rv.pf);
        t.pv_i = static_cast<const uint32_t*>(cl.rv.pi);
      }
      lists[xcd].push_back({in_lo, t});
      for (size_t j = s; j < e; ++j) {
        const ta_block& b = plan->host[(size_t)idx[j]];
        ordered.push_back(b);
        deltas.push_back((int32_t)(b.in_off - in_lo));
        deltas.push_back((int32_t)(b.out_off - out_lo));
      }
      s = e;
    }
  }
  // an XCD's tiles by position: tiles of different sizes and classes that
  // share cache lines run at about the same time on that XCD
  std::vector<ta::BatchTile> tiles;
  for (int x = 0; x < ta::kXcds; ++x) {
    std::stable_sort(lists[x].begin(), lists[x].end(),
                     [](const std::pair<int64_t, ta::BatchTile>& a, const std::pair<int64_t, ta::BatchTile>& b) {
                       return a.first < b.first;
                     });
    plan->xstart[x] = (int64_t)tiles.size();
    for (const auto& pt : lists[x]) tiles.push_back(pt.second);
  }
  plan->xstart[ta::kXcds] = (int64_t)tiles.size();
  if (tiles.size() > (size_t)INT32_MAX) return fail(TA_EUNSUPPORTED, "more than 2^31 tiles");
  plan->ntiles = (int64_t)tiles.size();
  plan->region_log2 = region_log2;
  TA_ON_DEVICE(plan->device);
  if (n > 0) {
    // allocated once, at their largest (a tile holds at least one block), so
    // that re-planning never moves them
    if (!plan->blocks_dev) TA_HIP(hipMalloc(&plan->blocks_dev, (size_t)n * sizeof(ta_block)));
    if (!plan->tiles_dev) TA_HIP(hipMalloc(&plan->tiles_dev, (size_t)n * sizeof(ta::BatchTile)));
    if (!plan->deltas_dev) TA_HIP(hipMalloc(&plan->deltas_dev, 2 * (size_t)n * sizeof(int32_t)));
    if (!plan->sched_dev) {
      TA_HIP(hipMalloc(&plan->sched_dev, 2 * ta_plan::kSchedStride * sizeof(int32_t)));
      TA_HIP(hipMemset(plan->sched_dev, 0, 2 * ta_plan::kSchedStride * sizeof(int32_t)));
    }
    TA_HIP(hipMemcpy(plan->blocks_dev, ordered.data(), ordered.size() * sizeof(ta_block), hipMemcpyHostToDevice));
    TA_HIP(hipMemcpy(plan->deltas_dev, deltas.data(), deltas.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    TA_HIP(hipMemcpy(plan->tiles_dev, tiles.data(), tiles.size() * sizeof(ta::BatchTile), hipMemcpyHostToDevice));
  }
  return TA_OK;
}

}  // namespace

extern "C" {

int ta_plan_create(ta_ctx* c, const ta_block* blocks, int64_t n, int dtype, ta_plan** out) {
  return guard([&]() -> int {
    if (!c || !out || (n > 0 && !blocks)) return fail(TA_EINVAL, "null argument");
    *out = nullptr;
    if (n < 0) return fail(TA_EINVAL, "negative block count");
    if (dtype != TA_I16 && dtype != TA_F32) return fail(TA_EINVAL, "unknown dtype %d", dtype);
    auto plan = std::make_unique<ta_plan>();
    plan->ctx = c;
    plan->device = c->device;
    plan->dtype = dtype;
    plan->host.assign(blocks, blocks + n);
    plan->cls.resize((size_t)n);
    // a class is one (size, kinds, resolved axes): the general kernel's
    // programs depend on the size also for axes without parameters
    std::map<std::tuple<int, int, int, int, Resolved, Resolved>, uint32_t> class_of;
    for (int64_t i = 0; i < n; ++i) {
      const ta_block& b = blocks[i];
      Resolved rh, rv;
      int kh, kv, e;
      if ((e = check_block(c, b, i, dtype, &rh, &rv, &kh, &kv))) return e;
      const auto key = std::make_tuple((int)b.log2w, (int)b.log2h, kh, kv, rh, rv);
      auto it = class_of.find(key);
      if (it == class_of.end()) {
        it = class_of.emplace(key, (uint32_t)plan->classes.size()).first;
        plan->classes.push_back(ta_plan::Class{b.log2w, b.log2h, kh, kv, rh, rv});
        if (kh < 0 || kv < 0) plan->general = true;
      }
      plan->cls[(size_t)i] = it->second;
      const int w = 1 << b.log2w, h = 1 << b.log2h;
      // the planned int16 kernels address a block's rows with 32-bit byte
      // offsets from their tile's base; rows further apart run on the
      // general kernel
      if (dtype == TA_I16 && (int64_t)(h - 1) * b.in_stride + w > ((int64_t)1 << 30)) plan->general = true;
      plan->max_in_elem = std::max<int64_t>(plan->max_in_elem, b.in_off + (int64_t)(h - 1) * b.in_stride + w);
      plan->max_out_elem = std::max<int64_t>(plan->max_out_elem, b.out_off + (int64_t)(h - 1) * b.out_stride + w);
    }
    plan->nblocks = n;
    int e;
    if (plan->general && !plan->classes.empty()) {
      // stage programs of every class
      std::vector<ta::GenProg> progs(4 * plan->classes.size());
      for (size_t k = 0; k < plan->classes.size(); ++k)
        for (int inv = 0; inv < 2; ++inv) {
          const ta_plan::Class& cl = plan->classes[k];
          progs[4 * k + inv] = gen_prog(c, cl.rh, cl.lw, dtype, inv);
          progs[4 * k + 2 + inv] = gen_prog(c, cl.rv, cl.lh, dtype, inv);
        }
      TA_ON_DEVICE(c->device);
      TA_HIP(hipMalloc(&plan->progs_dev, progs.size() * sizeof(ta::GenProg)));
      TA_HIP(hipMemcpy(plan->progs_dev, progs.data(), progs.size() * sizeof(ta::GenProg), hipMemcpyHostToDevice));
    }
    if ((e = build_tiles(plan.get(), plan->region_log2))) return e;
    *out = plan.release();
    return TA_OK;
  });
}

int ta_plan_destroy(ta_plan* p) {
  if (!p) return fail(TA_EINVAL, "null plan");
  delete p;   // frees the plan's device arrays
  return TA_OK;
}

int ta_plan_info(const ta_plan* p, int64_t* nblocks, int64_t* ntiles, int* grid) {
  if (!p) return fail(TA_EINVAL, "null plan");
  if (nblocks) *nblocks = p->nblocks;
  if (ntiles) *ntiles = p->ntiles;
  if (grid) *grid = p->grid;
  return TA_OK;
}

int ta_plan_extents(const ta_plan* p, int* dtype, int64_t* in_elems, int64_t* out_elems) {
  if (!p) return fail(TA_EINVAL, "null plan");
  if (dtype) *dtype = p->dtype;
  if (in_elems) *in_elems = p->max_in_elem;
  if (out_elems) *out_elems = p->max_out_elem;
  return TA_OK;
}

int ta_plan_tuning(const ta_plan* p, int* grid, int* region_log2) {
  if (!p) return fail(TA_EINVAL, "null plan");
  if (grid) *grid = p->grid;
  if (region_log2) *region_log2 = p->region_log2;
  return TA_OK;
}

int ta_plan_fwd(ta_ctx* c, ta_plan* p, const void* in, void* out, ta_stream_t stream) {
  if (!c || !p) return fail(TA_EINVAL, "null argument");
  if (p->ctx != c) return fail(TA_EINVAL, "plan was created with another context");
  if (p->ntiles == 0) return TA_OK;
  if (!in || !out) return fail(TA_EINVAL, "null buffer");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(TA_EINVAL, "buffers must be 16-byte aligned");
  return launch_plan(c, p, 0, in, out, stream, p->grid);
}

int ta_plan_inv(ta_ctx* c, ta_plan* p, const void* in, void* out, ta_stream_t stream) {
  if (!c || !p) return fail(TA_EINVAL, "null argument");
  if (p->ctx != c) return fail(TA_EINVAL, "plan was created with another context");
  if (p->ntiles == 0) return TA_OK;
  if (!in || !out) return fail(TA_EINVAL, "null buffer");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(TA_EINVAL, "buffers must be 16-byte aligned");
  return launch_plan(c, p, 1, in, out, stream, p->grid);
}

int ta_plan_autotune(ta_ctx* c, ta_plan* p, const void* in, void* out, ta_stream_t stream, int reps) {
  return guard([&]() -> int {
    if (!c || !p) return fail(TA_EINVAL, "null argument");
    if (p->ctx != c) return fail(TA_EINVAL, "plan was created with another context");
    if (p->ntiles == 0) return TA_OK;
    if (!in || !out) return fail(TA_EINVAL, "null buffer");
    if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(TA_EINVAL, "buffers must be 16-byte aligned");
    if (reps < 1) reps = 3;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    TA_ON_DEVICE(c->device);
    // every candidate's outputs are checked bitwise against the first one's
    const size_t esz = p->dtype == TA_F32 ? sizeof(float) : sizeof(int16_t);
    const size_t in_bytes = ((size_t)p->max_in_elem * esz + 255) & ~(size_t)255;
    const size_t bytes = (size_t)p->max_out_elem * esz, out_bytes = (bytes + 255) & ~(size_t)255;
    std::vector<char> ref(bytes), got(bytes), refi(bytes), goti(bytes);
    // A frame batch streams through HBM once per call.  The candidates are
    // timed on kSets buffer sets in turn, so that each launch finds the
    // caches holding the other sets' data, as in a stream of batches: set 0
    // is (in, out, inverse output), the others a copy of `in` with their own
    // forward and inverse outputs, all in one scratch allocation.  The
    // inverse reads its set's forward output when that covers the input
    // extent, else its set's input (the timing barely depends on the values).
    constexpr int kSets = 3;
    char* scratch = nullptr;
    TA_HIP(hipMalloc(&scratch, (kSets - 1) * (in_bytes + out_bytes) + kSets * out_bytes));
    const void* set_in[kSets];
    void* set_out[kSets];
    void* set_inv[kSets];
    set_in[0] = in;
    set_out[0] = out;
    char* sp = scratch;
    for (int k = 1; k < kSets; ++k) {
      set_in[k] = sp;
      set_out[k] = sp + in_bytes;
      sp += in_bytes + out_bytes;
    }
    for (int k = 0; k < kSets; ++k, sp += out_bytes) set_inv[k] = sp;
    const bool inv_from_out = p->max_in_elem <= p->max_out_elem;
    int rc = TA_OK;
    for (int k = 1; k < kSets && rc == TA_OK; ++k)
      if (hipMemcpyAsync(const_cast<void*>(set_in[k]), in, (size_t)p->max_in_elem * esz, hipMemcpyDeviceToDevice, s) !=
          hipSuccess)
        rc = fail(TA_EHIP, "autotune copy failed");
    const int regions[] = {18, 19, 20, 21, 22};     // tile mapping: frame-region size of the XCD lists
    const int grids[] = {256, 512, 1024, 2048, 4096, 8192};
    // events around the timed launches of one direction, recorded back to
    // back (the launches follow each other without a host round trip)
    constexpr int kWarm = 6, kTimed = 6, kEv = kTimed + 1;
    hipEvent_t ev[kEv] = {};
    for (int i = 0; i < kEv && rc == TA_OK; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) rc = fail(TA_EHIP, "event create failed");
    bool have_ref = false;
    // Per candidate, the launch times of each direction (samples[0] forward,
    // samples[1] inverse); a candidate scores the sum of the two medians.
    struct Samples {
      std::vector<float> t[2];
      float score() const {
        float sc = 0.0f;
        for (std::vector<float> v : t) {
          if (v.empty()) return 1e30f;
          std::sort(v.begin(), v.end());
          sc += v.size() % 2 ? v[v.size() / 2] : 0.5f * (v[v.size() / 2 - 1] + v[v.size() / 2]);
        }
        return sc;
      }
    };
    // A run of one direction, as a codec streams batches: kWarm untimed and
    // kTimed timed launches back to back over the sets in turn.  The first
    // launches after a change of kernel run slower while the clocks settle.
    auto run = [&](int g, int inv, Samples* smp) -> int {
      int r0;
      for (int i = 0; i < kWarm + kTimed; ++i) {
        if (i >= kWarm) (void)hipEventRecord(ev[i - kWarm], s);
        const int k = i % kSets;
        const void* src = inv ? (inv_from_out ? set_out[k] : set_in[k]) : set_in[k];
        if ((r0 = launch_plan(c, p, inv, src, inv ? set_inv[k] : set_out[k], stream, g))) return r0;
      }
      (void)hipEventRecord(ev[kTimed], s);
      if (hipEventSynchronize(ev[kTimed]) != hipSuccess) return fail(TA_EHIP, "autotune sync failed");
      for (int i = 0; i < kTimed; ++i) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        smp->t[inv].push_back(ms);
      }
      return TA_OK;
    };
    // After the host rebuilds the tile list the GPU has idled and its clocks
    // have dropped: untimed launches bring them back before the next
    // candidate is timed.
    auto settle = [&](int g) -> int {
      int r0;
      for (int i = 0; i < 64; ++i)
        if ((r0 = launch_plan(c, p, 0, set_in[i % kSets], set_out[i % kSets], stream, g))) return r0;
      return TA_OK;
    };
    // a forward run and an inverse run of the current tiles at grid g (the
    // forward writes every set's output before any inverse reads it); with
    // `check`, the outputs are compared with the first candidate's
    auto time_grid = [&](int g, Samples* smp, bool check) -> int {
      int r0;
      if ((r0 = run(g, 0, smp)) || (r0 = run(g, 1, smp))) return r0;
      if (!check) return TA_OK;
      if (hipMemcpy(have_ref ? got.data() : ref.data(), out, bytes, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(have_ref ? goti.data() : refi.data(), set_inv[0], bytes, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(TA_EHIP, "autotune copy failed");
      if (have_ref && (memcmp(ref.data(), got.data(), bytes) != 0 || memcmp(refi.data(), goti.data(), bytes) != 0))
        return fail(TA_EHIP, "autotune candidate (region 2^%d, grid %d) disagrees", p->region_log2, g);
      have_ref = true;
      return TA_OK;
    };
    // Clocks drift under sustained load, so the candidates are timed in
    // `reps` interleaved rounds (each round visits all of them).
    constexpr int kRegions = sizeof(regions) / sizeof(regions[0]), kGrids = sizeof(grids) / sizeof(grids[0]);
    std::vector<Samples> sums(kRegions * kGrids);
    const int orig_region = p->region_log2;
    int orig_tiles[7][7];
    memcpy(orig_tiles, p->tile_blocks, sizeof orig_tiles);
    int best_grid = p->grid, best_region = orig_region;
    for (int r = 0; r < reps && rc == TA_OK; ++r)
      for (int i = 0; i < kRegions && rc == TA_OK; ++i) {
        if ((rc = build_tiles(p, regions[i])) || (rc = settle(grids[0]))) break;
        for (int j = 0; j < kGrids; ++j)
          if ((rc = time_grid(grids[j], &sums[i * kGrids + j], r == 0))) break;
      }
    // Scores within 1 % of the best are taken as equal (that is about the
    // spread of the measurement); among them the smallest grid wins: the
    // fewest workgroup launches, and tiles handed out by the counters once
    // the grid is resident, which keeps the load balanced when a batch's
    // timing varies.
    if (rc == TA_OK) {
      float best = 1e30f;
      for (const Samples& sm : sums) best = std::min(best, sm.score());
      float pick = 1e30f;
      for (int j = 0; j < kGrids && pick > 1e29f; ++j)
        for (int i = 0; i < kRegions; ++i) {
          const float sc = sums[i * kGrids + j].score();
          if (sc <= best * 1.01f && sc < pick) { pick = sc; best_region = regions[i]; best_grid = grids[j]; }
        }
    }
    // then the blocks per tile of each size group (larger side 4 .. 64), by
    // coordinate descent at the chosen grid and region: the kernels'
    // maximum, half of it or a quarter, timed in interleaved rounds against
    // the current choice
    for (int ls = 2; ls <= 6 && rc == TA_OK; ++ls) {
      bool present = false;
      for (const ta_plan::Class& cl : p->classes) present |= std::max(cl.lw, cl.lh) == ls;
      if (!present) continue;
      int keep[7][7];
      memcpy(keep, p->tile_blocks, sizeof keep);
      const int divs[] = {0, 2, 4};   // 0: the current choice
      Samples sum[3];
      auto apply = [&](int div) {
        memcpy(p->tile_blocks, keep, sizeof keep);
        if (div)
          for (int lw = 2; lw <= 6; ++lw)
            for (int lh = 2; lh <= 6; ++lh)
              if (std::max(lw, lh) == ls) p->tile_blocks[lw][lh] = std::max(1, max_tile_blocks(p, lw, lh) / div);
      };
      for (int r = 0; r < reps && rc == TA_OK; ++r)
        for (int d = 0; d < 3; ++d) {
          apply(divs[d]);
          if ((rc = build_tiles(p, best_region)) || (rc = settle(best_grid)) ||
              (rc = time_grid(best_grid, &sum[d], r == 0)))
            break;
        }
      if (rc != TA_OK) break;
      int bd = 0;
      float bs = sum[0].score();
      for (int d = 1; d < 3; ++d) {
        const float sc = sum[d].score();
        if (sc < bs) { bs = sc; bd = d; }
      }
      apply(divs[bd]);
    }
    for (hipEvent_t x : ev)
      if (x) (void)hipEventDestroy(x);
    (void)hipStreamSynchronize(s);
    (void)hipFree(scratch);
    // keep the fastest mapping (on a failure the plan returns to what it was;
    // either way it is rebuilt so that it stays consistent)
    if (rc != TA_OK) memcpy(p->tile_blocks, orig_tiles, sizeof orig_tiles);
    const int rc2 = build_tiles(p, rc == TA_OK ? best_region : orig_region);
    if (rc == TA_OK && rc2 == TA_OK) p->grid = best_grid;
    return rc != TA_OK ? rc : rc2;
  });
}

int ta_plan_tile_blocks(const ta_plan* p, int log2w, int log2h, int* blocks) {
  if (!p || !blocks) return fail(TA_EINVAL, "null argument");
  if (log2w < 2 || log2w > 6 || log2h < 2 || log2h > 6) return fail(TA_EINVAL, "size outside 4..64");
  *blocks = tile_blocks(p, log2w, log2h);
  return TA_OK;
}

int ta_plan_set_tile_blocks(ta_plan* p, int log2w, int log2h, int blocks) {
  return guard([&]() -> int {
    if (!p) return fail(TA_EINVAL, "null plan");
    if (log2w < 2 || log2w > 6 || log2h < 2 || log2h > 6) return fail(TA_EINVAL, "size outside 4..64");
    const int m = max_tile_blocks(p, log2w, log2h);
    if (blocks < 0 || blocks > m)
      return fail(TA_EINVAL, "%d blocks per tile outside 0..%d for %dx%d", blocks, m, 1 << log2w, 1 << log2h);
    p->tile_blocks[log2w][log2h] = blocks;
    return build_tiles(p, p->region_log2);
  });
}

int ta_plan_set_tuning(ta_plan* p, int grid, int region_log2) {
  return guard([&]() -> int {
    if (!p) return fail(TA_EINVAL, "null plan");
    if (grid < ta::kXcds || grid > (1 << 20)) return fail(TA_EINVAL, "grid %d outside %d..2^20", grid, ta::kXcds);
    if (region_log2 < 12 || region_log2 > 40) return fail(TA_EINVAL, "region 2^%d outside 2^12..2^40", region_log2);
    int e;
    if (region_log2 != p->region_log2 && (e = build_tiles(p, region_log2))) return e;
    p->grid = grid;
    return TA_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Unplanned block lists: descriptors in device memory, read as they are
// ---------------------------------------------------------------------------
namespace {

int run_blocks(ta_ctx* c, int inv, const ta_block* blocks, int64_t n, const void* in, void* out, int dtype,
               ta_stream_t stream) {
  if (!c) return fail(TA_EINVAL, "null context");
  if (n < 0) return fail(TA_EINVAL, "negative block count");
  if (dtype != TA_I16 && dtype != TA_F32) return fail(TA_EINVAL, "unknown dtype %d", dtype);
  if (n == 0) return TA_OK;
  if (!blocks || !in || !out) return fail(TA_EINVAL, "null buffer");
  if (in == out) return fail(TA_EINVAL, "input and output alias");
  if ((uintptr_t)blocks & 7) return fail(TA_EINVAL, "descriptors must be 8-byte aligned");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(TA_EINVAL, "buffers must be 16-byte aligned");
  // one workgroup per quarter of a sort window (the dispatcher balances
  // quarters of uneven cost), and at least one per XCD range
  const int64_t sortwin = (int64_t)ta::kDescWindow * ta::kSortQuarters;
  const int64_t units = (n + sortwin - 1) / sortwin * ta::kSortQuarters;
  const int64_t g = std::max<int64_t>(ta::kXcds, std::min<int64_t>(units, 0x7fffffff));
  const void* fn = ta::batch_kernel(inv, 1, dtype == TA_F32);
  ta::BatchArgs args{};
  args.tiles = nullptr;
  args.ntiles = 0;
  args.blocks = blocks;
  args.in = static_cast<const int16_t*>(in);
  args.out = static_cast<int16_t*>(out);
  args.bd = c->bd;
  args.m = c->m;
  args.a = c->a;
  args.axes = c->axes_dev;
  args.nblocks = n;
  void* kargs[] = {&args};
  TA_ON_DEVICE(c->device);
  // (with m != 8 no axis has a fast kind: the general launch runs them all)
  if (c->m == 8)
    TA_HIP(hipLaunchKernel(fn, dim3((unsigned)g), dim3(256), kargs, 0, reinterpret_cast<hipStream_t>(stream)));
  if (c->ngeneral > 0) {
    // some registered axis has a kind outside the fast kernel's: a second
    // launch runs the descriptors with such an axis through the general
    // kernel (the fast kernel skips them, the general one skips the rest)
    ta::GenArgs ga{};
    ga.blocks = blocks;
    ga.in = in;
    ga.out = out;
    ga.inv = inv;
    ga.bd = c->bd;
    ga.m = c->m;
    ga.a = c->a;
    ga.nblocks = n;
    ga.progs = c->gprogs_dev[dtype == TA_F32];
    ga.fast = c->axes_dev;
    void* gargs[] = {&ga};
    TA_HIP(hipLaunchKernel(ta::gen_kernel(1, dtype == TA_F32), dim3((unsigned)g), dim3(256), gargs, 0,
                           reinterpret_cast<hipStream_t>(stream)));
  }
  return TA_OK;
}

// Workspace of a device-planned block list: tile counters per XCD list, the
// consumer's schedule counters, per-block data (int16: deltas; fp32: list
// indices in grouped order; 8 bytes), then kXcds tile lists of `cap`
// tiles (a window's tiles go to one list; a list holds every tile its
// windows can produce).
struct WsLayout {
  int64_t cap, sched_off, deltas_off, tiles_off, bytes;
};
WsLayout ws_layout(int64_t n) {
  WsLayout L;
  const int64_t nwin = (n + ta::kPlanWin - 1) / ta::kPlanWin;
  L.cap = (nwin + ta::kXcds - 1) / ta::kXcds * ta::kPlanWin;
  auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
  L.sched_off = 256;
  L.deltas_off = up(L.sched_off + 4 * ta::kSchedDwords);
  L.tiles_off = up(L.deltas_off + 8 * n);
  L.bytes = L.tiles_off + (int64_t)sizeof(ta::BatchTile) * ta::kXcds * L.cap;
  return L;
}

int run_blocks_ws(ta_ctx* c, int inv, const ta_block* blocks, int64_t n, const void* in, void* out, int dtype,
                  void* ws, int64_t ws_bytes, ta_stream_t stream) {
  if (!c) return fail(TA_EINVAL, "null context");
  if (n < 0) return fail(TA_EINVAL, "negative block count");
  if (dtype != TA_I16 && dtype != TA_F32) return fail(TA_EINVAL, "unknown dtype %d", dtype);
  if (n == 0) return TA_OK;
  // with m != 8 no axis has a fast kind: as the unplanned lists (all general)
  if (c->m != 8) return run_blocks(c, inv, blocks, n, in, out, dtype, stream);
  const bool f32 = dtype == TA_F32;
  if (!blocks || !in || !out) return fail(TA_EINVAL, "null buffer");
  if (in == out) return fail(TA_EINVAL, "input and output alias");
  if ((uintptr_t)blocks & 7) return fail(TA_EINVAL, "descriptors must be 8-byte aligned");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(TA_EINVAL, "buffers must be 16-byte aligned");
  const WsLayout L = ws_layout(n);
  if (!ws || ((uintptr_t)ws & 255)) return fail(TA_EINVAL, "workspace must be non-null and 256-byte aligned");
  if (ws_bytes < L.bytes)
    return fail(TA_EINVAL, "workspace of %lld bytes, %lld needed", (long long)ws_bytes, (long long)L.bytes);
  if (ta::kXcds * L.cap > INT32_MAX) return fail(TA_EUNSUPPORTED, "block list too long for int32 tile indices");
  char* w = static_cast<char*>(ws);
  int32_t* counts = reinterpret_cast<int32_t*>(w);
  int32_t* sched = reinterpret_cast<int32_t*>(w + L.sched_off);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TA_ON_DEVICE(c->device);
  // counters to zero (a kernel, so that the call stays capturable)
  int32_t* zp = counts;
  int zn = (int)(L.deltas_off / 4);
  void* zargs[] = {&zp, &zn};
  TA_HIP(hipLaunchKernel(ta::zero_words_kernel(), dim3(1), dim3(256), zargs, 0, s));
  ta::PlanArgs pa{};
  pa.blocks = blocks;
  pa.nblocks = n;
  pa.axes = c->axes_dev;
  pa.tiles = reinterpret_cast<ta::BatchTile*>(w + L.tiles_off);
  pa.deltas = reinterpret_cast<int32_t*>(w + L.deltas_off);
  pa.index = reinterpret_cast<int32_t*>(w + L.deltas_off);
  pa.count = counts;
  pa.cap = L.cap;
  void* pargs[] = {&pa};
  const int64_t nwin = (n + ta::kPlanWin - 1) / ta::kPlanWin;
  if (nwin > INT32_MAX) return fail(TA_EUNSUPPORTED, "block list too long");
  TA_HIP(hipLaunchKernel(ta::desc_plan_kernel(f32), dim3((unsigned)nwin), dim3(ta::kPlanThreads), pargs, 0, s));
  // the planned kernel over the lists: int16, one resident grid taking tiles
  // from the schedule counters; fp32 (its kernel has a static stride), 8,192
  // workgroups
  const void* fn = ta::batch_kernel(inv, 0, f32);
  int res = 0, e;
  if (f32)
    res = 8192;
  else if ((e = resident_groups(fn, 256, c->device, &res)))
    return e;
  ta::BatchArgs args{};
  args.tiles = pa.tiles;
  args.ntiles = ta::kXcds * L.cap;
  for (int x = 0; x <= ta::kXcds; ++x) args.xstart[x] = x * L.cap;
  args.xcount = counts;
  args.deltas = pa.deltas;
  args.blocks = blocks;
  args.order = f32 ? pa.index : nullptr;
  args.sched = f32 ? nullptr : sched;
  args.in = static_cast<const int16_t*>(in);
  args.out = static_cast<int16_t*>(out);
  args.bd = c->bd;
  args.m = c->m;
  args.a = c->a;
  void* kargs[] = {&args};
  TA_HIP(hipLaunchKernel(fn, dim3((unsigned)std::max(res, ta::kXcds)), dim3(256), kargs, 0, s));
  if (c->ngeneral > 0) {
    // descriptors with an axis outside the fast kinds: the general kernel
    // over the same list (it skips the others), as for unplanned lists
    const int64_t sortwin = (int64_t)ta::kDescWindow * ta::kSortQuarters;
    const int64_t units = (n + sortwin - 1) / sortwin * ta::kSortQuarters;
    const int64_t g = std::max<int64_t>(ta::kXcds, std::min<int64_t>(units, 0x7fffffff));
    ta::GenArgs ga{};
    ga.blocks = blocks;
    ga.in = in;
    ga.out = out;
    ga.inv = inv;
    ga.bd = c->bd;
    ga.m = c->m;
    ga.a = c->a;
    ga.nblocks = n;
    ga.progs = c->gprogs_dev[f32];
    ga.fast = c->axes_dev;
    void* gargs[] = {&ga};
    TA_HIP(hipLaunchKernel(ta::gen_kernel(1, f32), dim3((unsigned)g), dim3(256), gargs, 0, s));
  }
  return TA_OK;
}

// Last element (exclusive) a block touches at (off, stride), or -1 past `limit`.
int64_t block_end(int64_t off, int32_t stride, int w, int h, int64_t limit) {
  if (off > limit) return -1;
  const int64_t end = off + (int64_t)(h - 1) * stride + w;   // off <= limit < 2^63 - 2^37
  return end > limit ? -1 : end;
}

}  // namespace

extern "C" {

int ta_transform_fwd(ta_ctx* c, const ta_block* blocks_dev, int64_t nblocks, const void* in, void* out, int dtype,
                     ta_stream_t stream) {
  return run_blocks(c, 0, blocks_dev, nblocks, in, out, dtype, stream);
}

int ta_transform_inv(ta_ctx* c, const ta_block* blocks_dev, int64_t nblocks, const void* in, void* out, int dtype,
                     ta_stream_t stream) {
  return run_blocks(c, 1, blocks_dev, nblocks, in, out, dtype, stream);
}

int ta_transform_workspace(int64_t nblocks, int64_t* bytes) {
  if (!bytes || nblocks < 0) return fail(TA_EINVAL, "null argument or negative block count");
  if (nblocks > (int64_t(1) << 40)) return fail(TA_EINVAL, "block count above 2^40");
  *bytes = nblocks ? ws_layout(nblocks).bytes : 0;
  return TA_OK;
}

int ta_transform_fwd_ws(ta_ctx* c, const ta_block* blocks_dev, int64_t nblocks, const void* in, void* out, int dtype,
                        void* workspace, int64_t workspace_bytes, ta_stream_t stream) {
  return run_blocks_ws(c, 0, blocks_dev, nblocks, in, out, dtype, workspace, workspace_bytes, stream);
}

int ta_transform_inv_ws(ta_ctx* c, const ta_block* blocks_dev, int64_t nblocks, const void* in, void* out, int dtype,
                        void* workspace, int64_t workspace_bytes, ta_stream_t stream) {
  return run_blocks_ws(c, 1, blocks_dev, nblocks, in, out, dtype, workspace, workspace_bytes, stream);
}

int ta_validate_blocks(ta_ctx* c, const ta_block* blocks_dev, int64_t n, int64_t in_elems, int64_t out_elems,
                       int64_t* first_bad) {
  return guard([&]() -> int {
    if (!c || !first_bad) return fail(TA_EINVAL, "null argument");
    *first_bad = -1;
    if (n < 0 || in_elems < 0 || out_elems < 0) return fail(TA_EINVAL, "negative count");
    if (n == 0) return TA_OK;
    if (!blocks_dev) return fail(TA_EINVAL, "null descriptors");
    if (in_elems > ((int64_t)1 << 62) || out_elems > ((int64_t)1 << 62)) return fail(TA_EINVAL, "buffer size above 2^62");
    std::vector<ta_block> host((size_t)n);
    TA_ON_DEVICE(c->device);
    TA_HIP(hipMemcpy(host.data(), blocks_dev, (size_t)n * sizeof(ta_block), hipMemcpyDeviceToHost));
    std::lock_guard<std::mutex> lk(c->mu);
    for (int64_t i = 0; i < n; ++i) {
      const ta_block& b = host[(size_t)i];
      Resolved rh, rv;
      int kh, kv, e;
      if ((e = check_block(c, b, i, TA_I16, &rh, &rv, &kh, &kv))) {
        *first_bad = i;
        return e;
      }
      const int w = 1 << b.log2w, h = 1 << b.log2h;
      if (block_end(b.in_off, b.in_stride, w, h, in_elems) < 0 || block_end(b.out_off, b.out_stride, w, h, out_elems) < 0) {
        *first_bad = i;
        return fail(TA_EINVAL, "block %lld: extends past the input (%lld elements) or output (%lld elements)",
                    (long long)i, (long long)in_elems, (long long)out_elems);
      }
    }
    return TA_OK;
  });
}

int ta_set_axis_cfg(ta_ctx* c, int axis_id, const ta_axis_cfg* cfg) {
  if (!c || !cfg) return fail(TA_EINVAL, "null argument");
  if (cfg->adj == TA_ADJ_NONE) {
    if (cfg->log2n != 0 && (cfg->log2n < 2 || cfg->log2n > 6)) return fail(TA_EUNSUPPORTED, "log2n %d", cfg->log2n);
    if (cfg->k_or_b != 0) return fail(TA_EINVAL, "an axis without adjustment has no K or B");
  } else {
    if (cfg->param_id < 0 || cfg->param_id >= kMaxIds) return fail(TA_EINVAL, "parameter id %d outside 0..255", cfg->param_id);
    const ParamSet& ps = c->params[cfg->param_id];
    if (ps.kind != cfg->adj) return fail(TA_ENOPARAMS, "parameter set %d not registered for this adjustment", cfg->param_id);
    if (cfg->log2n != 0 && (1 << std::min(std::max(cfg->log2n, 0), 30)) != ps.n)
      return fail(TA_EINVAL, "log2n %d does not match parameter set %d (size %d)", cfg->log2n, cfg->param_id, ps.n);
    if (cfg->k_or_b != 0 && cfg->k_or_b != ps.kb)
      return fail(TA_EINVAL, "K/B %d does not match parameter set %d (%d)", cfg->k_or_b, cfg->param_id, ps.kb);
  }
  const ta_axis ax{cfg->base, cfg->adj, cfg->flip, cfg->param_id};
  return ta_set_axis(c, axis_id, &ax);
}

int ta_set_params(ta_ctx* c, int param_id, const int16_t* int_taps, const float* f32_params, const int32_t* layout,
                  int64_t n) {
  if (!c || !layout) return fail(TA_EINVAL, "null argument");
  const int adj = layout[0], size = layout[1], kb = layout[2];
  if (adj == TA_ADJ_BAND) {
    if (size < 1 || size > 64 || n != (int64_t)size * size)
      return fail(TA_EINVAL, "band of size %d takes %d x %d entries, got %lld", size, size, size, (long long)n);
    return ta_set_band(c, param_id, size, kb, int_taps, f32_params);
  }
  if (adj == TA_ADJ_POST) {
    if (kb < 1 || kb > 64 || n != (int64_t)kb * kb)
      return fail(TA_EINVAL, "sub-block of side %d takes %d x %d entries, got %lld", kb, kb, kb, (long long)n);
    return ta_set_post(c, param_id, size, kb, int_taps, f32_params);
  }
  return fail(TA_EINVAL, "layout kind %d is not a band or sub-block adjustment", adj);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Differentiable Givens-band path
// ---------------------------------------------------------------------------
namespace {
int givens_check(ta_ctx* c, int base, int n, int taps, const float* theta, int64_t nvec) {
  if (!c || !theta) return fail(TA_EINVAL, "null argument");
  if (nvec < 0) return fail(TA_EINVAL, "negative vector count");
  if ((n != 16 && n != 32) || (taps != 4 && taps != 6) || (base != TA_DCT2 && base != TA_DST3))
    return fail(TA_EUNSUPPORTED, "differentiable path: n in {16, 32}, taps in {4, 6}, base DCT-2 or DST-3");
  return TA_OK;
}
}  // namespace

extern "C" {

int ta_fwd_multi(ta_ctx* c, int param_id, int log2n, int64_t nblocks, const void* in, void* out,
                 ta_stream_t stream) {
  if (!c) return fail(TA_EINVAL, "null context");
  if (nblocks < 0) return fail(TA_EINVAL, "negative block count");
  if (param_id < 0 || param_id >= kMaxIds) return fail(TA_EINVAL, "parameter id %d outside 0..255", param_id);
  const ParamSet& ps = c->params[param_id];
  if (ps.kind != TA_ADJ_POST || !ps.fx_eo) return fail(TA_ENOPARAMS, "parameter set %d is not a sub-block set", param_id);
  if (ps.n != (1 << log2n)) return fail(TA_EINVAL, "parameter set %d is for size %d, not %d", param_id, ps.n, 1 << log2n);
  if (c->m != 8) return fail(TA_EUNSUPPORTED, "simultaneous evaluation is built for m = 8");
  int threads = 0, per_wg = 0;
  const void* fn = ta::multi_kernel(log2n, ps.kb, &threads, &per_wg);
  if (!fn) return fail(TA_EUNSUPPORTED, "simultaneous evaluation is built for 32x32 with B = 8 and 64x64 with B = 16");
  if (nblocks == 0) return TA_OK;
  if (!in || !out) return fail(TA_EINVAL, "null buffer");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(TA_EINVAL, "buffers must be 16-byte aligned");
  const size_t bytes_in = (size_t)nblocks << (2 * log2n + 1);
  const char* ib = static_cast<const char*>(in);
  const char* ob = static_cast<const char*>(out);
  if (ib < ob + 5 * bytes_in && ob < ib + bytes_in) return fail(TA_EINVAL, "input and output overlap");
  ta::MultiArgs a{static_cast<const int16_t*>(in), static_cast<int16_t*>(out), nblocks, ps.fx_eo,
                  log2n + c->bd + c->m - 15, log2n + c->m, c->a};
  const int64_t groups = (nblocks + per_wg - 1) / per_wg;
  if (groups > 0x7fffffff) return fail(TA_EUNSUPPORTED, "batch too large for one launch");
  void* kargs[] = {&a};
  TA_ON_DEVICE(c->device);
  TA_HIP(hipLaunchKernel(fn, dim3((unsigned)groups), dim3(threads), kargs, 0, reinterpret_cast<hipStream_t>(stream)));
  return TA_OK;
}

int ta_givens_workspace(int64_t nvec, int64_t* bytes) {
  if (!bytes || nvec < 0) return fail(TA_EINVAL, "bad argument");
  *bytes = ((nvec + 255) / 256) * ta::kMaxAng * (int64_t)sizeof(float);
  return TA_OK;
}

int ta_givens_fwd(ta_ctx* c, int base, int n, int taps, const float* theta, int64_t nvec, const float* x,
                  float* y, ta_stream_t stream) {
  int e;
  if ((e = givens_check(c, base, n, taps, theta, nvec))) return e;
  if (nvec == 0) return TA_OK;
  if (!x || !y) return fail(TA_EINVAL, "null buffer");
  ta::GivensArgs a{theta, x, nullptr, y, nullptr, nullptr, nvec};
  void* kargs[] = {&a};
  TA_ON_DEVICE(c->device);
  TA_HIP(hipLaunchKernel(ta::givens_kernel(0, n, taps / 2, base), dim3((unsigned)((nvec + 255) / 256)), dim3(256),
                         kargs, 0, reinterpret_cast<hipStream_t>(stream)));
  return TA_OK;
}

}  // extern "C"

namespace {

// The backward's two launches with the partial rows in `part` (the caller's
// workspace, or the static scratch of the allocation-free entry point).
int givens_bwd_launch(ta_ctx* c, int base, int n, int taps, const float* theta, int64_t nvec, const float* x,
                      const float* gy, float* gx, float* gtheta, float* part, ta_stream_t stream) {
  const int64_t groups = (nvec + 255) / 256;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TA_ON_DEVICE(c->device);
  if (groups > 0) {
    ta::GivensArgs a{theta, x, gy, nullptr, gx, part, nvec};
    void* kargs[] = {&a};
    TA_HIP(hipLaunchKernel(ta::givens_kernel(1, n, taps / 2, base), dim3((unsigned)groups), dim3(256), kargs, 0, s));
  }
  int na = 0;
  for (int l = 0; l < taps / 2; ++l) na += (n - 2 - (l & 1)) / 2 + 1;
  const float* cpart = part;
  int64_t g64 = groups;
  void* rargs[] = {&cpart, &g64, &na, &gtheta};
  TA_HIP(hipLaunchKernel(ta::givens_reduce_kernel(), dim3((unsigned)na), dim3(256), rargs, 0, s));
  return TA_OK;
}

}  // namespace

extern "C" {

int ta_givens_bwd(ta_ctx* c, int base, int n, int taps, const float* theta, int64_t nvec, const float* x,
                  const float* gy, float* gx, float* gtheta, void* workspace, ta_stream_t stream) {
  int e;
  if ((e = givens_check(c, base, n, taps, theta, nvec))) return e;
  if (!gtheta) return fail(TA_EINVAL, "null gradient buffer");
  if (nvec > 0 && (!x || !gy || !gx || !workspace)) return fail(TA_EINVAL, "null buffer");
  return givens_bwd_launch(c, base, n, taps, theta, nvec, x, gy, gx, gtheta, static_cast<float*>(workspace),
                           stream);
}

int ta_givens_bwd_noalloc(ta_ctx* c, int base, int n, int taps, const float* theta, int64_t nvec, const float* x,
                          const float* gy, float* gx, float* gtheta, ta_stream_t stream) {
  int e;
  if ((e = givens_check(c, base, n, taps, theta, nvec))) return e;
  if (!gtheta) return fail(TA_EINVAL, "null gradient buffer");
  if (nvec > 0 && (!x || !gy || !gx)) return fail(TA_EINVAL, "null buffer");
  if (nvec > ta::kNoAllocGroups * 256)
    return fail(TA_EINVAL, "%lld vectors: the allocation-free backward takes at most %lld", (long long)nvec,
                (long long)(ta::kNoAllocGroups * 256));
  if (!c->scratch) return fail(TA_EHIP, "static scratch of device %d not available", c->device);
  return givens_bwd_launch(c, base, n, taps, theta, nvec, x, gy, gx, gtheta, c->scratch, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Quantised-coefficient statistics
// ---------------------------------------------------------------------------
extern "C" {

}  // extern "C"

namespace {

// Geometry of the statistics launch: workgroups of 4 waves own 64 positions
// and a range of blocks; the range count fills the device once and keeps
// every 16-bit LDS counter below 2^16.
int stats_plan(ta_ctx* c, int64_t nblocks, int log2h, int log2w, ta::StatsArgs* a, int64_t* ws_bytes) {
  if (!c) return fail(TA_EINVAL, "null context");
  if (log2h < 2 || log2h > 6 || log2w < 2 || log2w > 6) return fail(TA_EUNSUPPORTED, "block sides 4..64");
  if (nblocks < 0) return fail(TA_EINVAL, "negative block count");
  const int positions = 1 << (log2h + log2w);
  if (nblocks > ((int64_t)1 << 34) / positions) return fail(TA_EINVAL, "more than 2^34 coefficients");
  *a = ta::StatsArgs{};
  a->nblocks = nblocks;
  a->positions = positions;
  a->log2h = log2h;
  a->log2w = log2w;
  a->total = nblocks * positions;
  const int np = std::min(positions, 64);
  a->slabs = positions / np;
  a->wstride = std::max(positions, 64);
  a->wave_steps = positions >= 64 ? nblocks : (a->total + 63) / 64;
  const int64_t full_waves = positions >= 64 ? nblocks : a->total / 64;
  a->steps = (a->wave_steps + 3) / 4;
  a->full_steps = full_waves / 4;
  a->ranges = 0;
  a->steps_per_wg = 0;
  if (a->steps > 0) {
    ta::KernelEntry k{};
    k.fn = ta::stats_kernel(1);
    k.threads = 256;
    int resident = 0, e;
    if ((e = resident_groups(&k, c->device, &resident))) return e;
    int64_t ranges = std::max<int64_t>(1, (resident + a->slabs - 1) / a->slabs);
    const int64_t cap = 65535 / (256 / np);   // samples per position per workgroup < 2^16
    a->steps_per_wg = std::min<int64_t>((a->steps + ranges - 1) / ranges, cap);
    a->ranges = (a->steps + a->steps_per_wg - 1) / a->steps_per_wg;
    if (a->ranges * a->slabs > 0x7fffffff) return fail(TA_EUNSUPPORTED, "batch too large for one launch");
  }
  // packed counters, then (8-byte aligned) the three sums per slot
  const int64_t slots = a->ranges * positions;
  *ws_bytes = ((slots * ta::kStatsPartDwords * 4 + 7) & ~(int64_t)7) + slots * 3 * (int64_t)sizeof(uint64_t) +
              positions * (int64_t)sizeof(double);
  return TA_OK;
}

}  // namespace

extern "C" {

int ta_coef_stats_workspace(ta_ctx* c, int64_t nblocks, int log2h, int log2w, int64_t* bytes) {
  if (!bytes) return fail(TA_EINVAL, "null argument");
  ta::StatsArgs a;
  return stats_plan(c, nblocks, log2h, log2w, &a, bytes);
}

int ta_coef_stats(ta_ctx* c, const int16_t* coef, int64_t nblocks, int log2h, int log2w, int32_t step,
                  int32_t offset, uint32_t* hist, uint64_t* esc_bits, uint64_t* energy, uint64_t* dist, double* rate,
                  double* summary, void* workspace, int64_t workspace_bytes, ta_stream_t stream) {
  ta::StatsArgs a;
  int64_t need = 0;
  int e;
  if ((e = stats_plan(c, nblocks, log2h, log2w, &a, &need))) return e;
  if (step < 1 || step > 32768 || offset < 0 || offset >= step)
    return fail(TA_EINVAL, "need 1 <= step <= 32768 and 0 <= offset < step");
  if (!hist || !esc_bits || !energy || !dist || !rate || !summary || (nblocks > 0 && !coef))
    return fail(TA_EINVAL, "null buffer");
  if (workspace_bytes < need || (need > 0 && !workspace))
    return fail(TA_EINVAL, "workspace of %lld bytes needed", (long long)need);
  if (((uintptr_t)hist & 3) || (((uintptr_t)esc_bits | (uintptr_t)energy | (uintptr_t)dist | (uintptr_t)rate |
                                 (uintptr_t)summary | (uintptr_t)workspace) & 7) || ((uintptr_t)coef & 1))
    return fail(TA_EINVAL, "misaligned buffer");
  a.in = coef;
  a.step = step;
  a.offset = offset;
  int cl = 0;
  while ((1 << cl) < step) ++cl;
  a.magic_shift = 16 + cl;
  a.magic = (uint32_t)((((uint64_t)1 << a.magic_shift) + (uint64_t)step - 1) / (uint64_t)step);
  a.hist = hist;
  a.esc_bits = esc_bits;
  a.energy = energy;
  a.dist = dist;
  a.rate = rate;
  a.summary = summary;
  const int64_t slots = a.ranges * a.positions;
  a.part = static_cast<uint32_t*>(workspace);
  a.part_e = reinterpret_cast<uint64_t*>(static_cast<char*>(workspace) +
                                         ((slots * ta::kStatsPartDwords * 4 + 7) & ~(int64_t)7));
  a.part_d = a.part_e + slots;
  a.part_b = a.part_d + slots;
  a.log_energy = reinterpret_cast<double*>(a.part_b + slots);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TA_ON_DEVICE(c->device);
  void* kargs[] = {&a};
  if (a.steps > 0) {
    TA_HIP(hipLaunchKernel(ta::stats_kernel(1), dim3((unsigned)(a.ranges * a.slabs)), dim3(256), kargs, 0, s));
    const int64_t threads = (int64_t)a.positions * (ta::kStatsPartDwords + 3);
    TA_HIP(hipLaunchKernel(ta::stats_kernel(4), dim3((unsigned)((threads + 255) / 256)), dim3(256), kargs, 0, s));
  } else {
    // empty batch: zero the accumulated outputs with a fill kernel
    // (capturable, no memset node)
    const void* zero = ta::stats_kernel(0);
    auto fill = [&](void* p, int64_t words) -> int {
      uint32_t* q = static_cast<uint32_t*>(p);
      int64_t n = words;
      void* zargs[] = {&q, &n};
      TA_HIP(hipLaunchKernel(zero, dim3((unsigned)((words + 255) / 256)), dim3(256), zargs, 0, s));
      return TA_OK;
    };
    if ((e = fill(hist, (int64_t)a.positions * ta::kStatsSymbols))) return e;
    if ((e = fill(esc_bits, 2 * (int64_t)a.positions))) return e;
    if ((e = fill(energy, 2 * (int64_t)a.positions))) return e;
    if ((e = fill(dist, 2 * (int64_t)a.positions))) return e;
  }
  TA_HIP(hipLaunchKernel(ta::stats_kernel(2), dim3((unsigned)((a.positions + 3) / 4)), dim3(256), kargs, 0, s));
  TA_HIP(hipLaunchKernel(ta::stats_kernel(3), dim3(1), dim3(256), kargs, 0, s));
  return TA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched adjustment design search
// ---------------------------------------------------------------------------
extern "C" {

int ta_design_search(ta_ctx* c, int n, int nmat, const double* mats, int64_t ncand, const int32_t* cands,
                     double* theta, int steps, double lr, double lam, double* grad, double* obj, double* adj,
                     ta_stream_t stream) {
  if (!c) return fail(TA_EINVAL, "null context");
  int threads = 0;
  const void* fn = ta::design_kernel(n, &threads);
  if (!fn) return fail(TA_EUNSUPPORTED, "design search is built for n in {4, 8, 16, 32}");
  if (ncand < 0 || nmat < 1 || steps < 0) return fail(TA_EINVAL, "need ncand >= 0, nmat >= 1, steps >= 0");
  if (!(lr > 0.0) || !std::isfinite(lr) || !(lam >= 0.0) || !std::isfinite(lam))
    return fail(TA_EINVAL, "need a finite lr > 0 and lam >= 0");
  if (ncand > 0x7fffffff) return fail(TA_EUNSUPPORTED, "too many candidates for one launch");
  if (ncand == 0) return TA_OK;
  if (!mats || !cands || !theta || !obj) return fail(TA_EINVAL, "null buffer");
  if ((((uintptr_t)mats | (uintptr_t)theta | (uintptr_t)obj | (uintptr_t)grad | (uintptr_t)adj) & 7) ||
      ((uintptr_t)cands & 3))
    return fail(TA_EINVAL, "misaligned buffer");
  ta::DesignArgs a{mats, nmat, cands, theta, steps, lr, lam, 0.9, 0.999, 1e-8, grad, obj, adj};
  void* kargs[] = {&a};
  TA_ON_DEVICE(c->device);
  TA_HIP(hipLaunchKernel(fn, dim3((unsigned)ncand), dim3(threads), kargs, 0, reinterpret_cast<hipStream_t>(stream)));
  return TA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Angle-parametrised parameter sets and the backward of the block-list
// transform
// ---------------------------------------------------------------------------
namespace {

// Rotation (p, q) by t applied from the left to the rows of a row-major
// n x n matrix: v_p = c u_p - s u_q, v_q = s u_p + c u_q.
void rotate_rows(std::vector<double>& m, int n, int p, int q, double t) {
  const double c = std::cos(t), s = std::sin(t);
  for (int j = 0; j < n; ++j) {
    const double a = m[(size_t)p * n + j], b = m[(size_t)q * n + j];
    m[(size_t)p * n + j] = c * a - s * b;
    m[(size_t)q * n + j] = s * a + c * b;
  }
}

int band_angle_count(int n, int taps) {
  int c = 0;
  for (int l = 0; l < taps / 2; ++l) c += (n - 2 - (l & 1)) / 2 + 1;
  return c;
}

// After a set was registered from its angles: keep the angles (and Q0) on
// the device and size the backward's workspace for the resident grid.
int attach_angles(ta_ctx* c, int id, const std::vector<double>& ang, const std::vector<double>* q0, int ne) {
  ParamSet& ps = c->params[id];
  int e, groups = 0;
  if ((e = resident_groups(ta::bwd_kernel(0), 256, c->device, &groups))) return e;
  void* p = nullptr;
  if ((e = upload(c, ang.data(), ang.size() * sizeof(double), &p))) return e;
  ps.ang_dev = static_cast<double*>(p);
  if (q0) {
    if ((e = upload(c, q0->data(), q0->size() * sizeof(double), &p))) return e;
    ps.q0_dev = static_cast<double*>(p);
  }
  std::vector<float> zero((size_t)groups * ne, 0.0f);
  if ((e = upload(c, zero.data(), zero.size() * sizeof(float), &p))) return e;
  ps.part_dev = static_cast<float*>(p);
  ps.part_groups = groups;
  ps.nang = (int)ang.size();
  return TA_OK;
}

}  // namespace

extern "C" {

int ta_set_band_angles(ta_ctx* c, int id, int n, int taps, const double* theta) {
  return guard([&]() -> int {
    if (!c || !theta) return fail(TA_EINVAL, "null argument");
    if (id < 0 || id >= kMaxIds) return fail(TA_EINVAL, "parameter id %d outside 0..255", id);
    if (log2_exact(n) < 2 || n > 64) return fail(TA_EUNSUPPORTED, "band size %d", n);
    if (taps != 2 && taps != 4 && taps != 6 && taps != 8) return fail(TA_EUNSUPPORTED, "band taps %d", taps);
    const int na = band_angle_count(n, taps);
    std::vector<double> ang(theta, theta + na);
    // A = G_{L-1} ... G_0: layer l applied after the layers before it
    std::vector<double> a((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) a[(size_t)i * n + i] = 1.0;
    int r = 0;
    for (int l = 0; l < taps / 2; ++l)
      for (int p = (l & 1); p + 1 < n; p += 2) rotate_rows(a, n, p, p + 1, ang[r++]);
    std::vector<int16_t> ai((size_t)n * n);
    std::vector<float> af((size_t)n * n);
    for (size_t k = 0; k < a.size(); ++k) {
      ai[k] = (int16_t)round_half_away(std::ldexp(a[k], c->a));
      af[k] = (float)a[k];
    }
    int e;
    if ((e = ta_set_band(c, id, n, taps, ai.data(), af.data()))) return e;
    std::lock_guard<std::mutex> lk(c->mu);
    return attach_angles(c, id, ang, nullptr, n * taps);
  });
}

int ta_set_post_angles(ta_ctx* c, int id, int n, int b, const double* q0, const double* phi) {
  return guard([&]() -> int {
    if (!c || !phi) return fail(TA_EINVAL, "null argument");
    if (id < 0 || id >= kMaxIds) return fail(TA_EINVAL, "parameter id %d outside 0..255", id);
    if (log2_exact(n) < 2 || n > 64) return fail(TA_EUNSUPPORTED, "post size %d", n);
    if ((b != 4 && b != 8 && b != 16) || b > n)
      return fail(TA_EUNSUPPORTED, "angle-parametrised sub-blocks take B in {4, 8, 16} (B <= n), got %d", b);
    const int na = b * (b - 1) / 2;
    std::vector<double> ang(phi, phi + na);
    std::vector<double> q0v((size_t)b * b, 0.0);
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) q0v[(size_t)i * b + j] = q0 ? q0[i * b + j] : (i == j ? 1.0 : 0.0);
    // R(phi): the rotations over the pairs (p, q), p < q in lexicographic
    // order, each applied after the previous ones; Q = Q0 R
    std::vector<double> rm((size_t)b * b, 0.0);
    for (int i = 0; i < b; ++i) rm[(size_t)i * b + i] = 1.0;
    int r = 0;
    for (int p = 0; p < b; ++p)
      for (int q = p + 1; q < b; ++q) rotate_rows(rm, b, p, q, ang[r++]);
    std::vector<int16_t> qi((size_t)b * b);
    std::vector<float> qf((size_t)b * b);
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) {
        double v = 0.0;
        for (int k = 0; k < b; ++k) v += q0v[(size_t)i * b + k] * rm[(size_t)k * b + j];
        qi[(size_t)i * b + j] = (int16_t)round_half_away(std::ldexp(v, c->a));
        qf[(size_t)i * b + j] = (float)v;
      }
    int e;
    if ((e = ta_set_post(c, id, n, b, qi.data(), qf.data()))) return e;
    std::lock_guard<std::mutex> lk(c->mu);
    return attach_angles(c, id, ang, q0 ? &q0v : nullptr, b * b);
  });
}

int ta_transform_bwd(ta_ctx* c, const ta_block* blocks_dev, int64_t nblocks, const float* x_dev, const float* gy_dev,
                     float* gx_dev, float* gtheta_dev, int param_id, ta_stream_t stream) {
  if (!c) return fail(TA_EINVAL, "null context");
  if (nblocks < 0) return fail(TA_EINVAL, "negative block count");
  if (param_id < 0 || param_id >= kMaxIds) return fail(TA_EINVAL, "parameter id %d outside 0..255", param_id);
  const ParamSet& ps = c->params[param_id];
  if (!ps.ang_dev || !ps.part_dev)
    return fail(TA_ENOPARAMS, "parameter set %d was not registered by its angles", param_id);
  if (!gtheta_dev) return fail(TA_EINVAL, "null gradient buffer");
  if (nblocks > 0 && (!blocks_dev || !x_dev || !gy_dev || !gx_dev)) return fail(TA_EINVAL, "null buffer");
  if ((uintptr_t)blocks_dev & 7) return fail(TA_EINVAL, "descriptors must be 8-byte aligned");
  if (gx_dev && (gx_dev == x_dev || gx_dev == gy_dev)) return fail(TA_EINVAL, "gx must not alias x or gy");
  const int ne = ps.kind == TA_ADJ_BAND ? ps.n * ps.kb : ps.kb * ps.kb;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nblocks, ps.part_groups));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TA_ON_DEVICE(c->device);
  ta::BwdArgs a{};
  a.blocks = blocks_dev;
  a.nblocks = nblocks;
  a.x = x_dev;
  a.gy = gy_dev;
  a.gx = gx_dev;
  a.progs = c->gprogs_dev[1];
  a.axis_use = c->axis_use_dev;
  a.pid = param_id;
  a.kind = ps.kind;
  a.n = ps.n;
  a.k_or_b = ps.kb;
  a.ne = ne;
  a.part = ps.part_dev;
  void* kargs[] = {&a};
  TA_HIP(hipLaunchKernel(ta::bwd_kernel(0), dim3((unsigned)grid), dim3(256), kargs, 0, s));
  ta::BwdChainArgs ch{ps.part_dev, grid, ne, ps.kind, ps.n, ps.kb, ps.nang, ps.ang_dev, ps.q0_dev, gtheta_dev};
  void* cargs[] = {&ch};
  TA_HIP(hipLaunchKernel(ta::bwd_kernel(1), dim3(1), dim3(256), cargs, 0, s));
  return TA_OK;
}

}  // extern "C"
