// Host runtime and C ABI of the DPLR long-range PPPM step (see include/dplr_lr.h).
#include "../../include/dplr_lr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pppm_kernels.hpp"
#include "mixed_radix_kernels.hpp"

using namespace dplr;

namespace {

// Messages of failed calls.  Fixed buffers: recording an error allocates
// nothing (the no-allocation entry point shares them).
constexpr size_t kErrLen = 512;
thread_local char g_global_error[kErrLen] = "";

void set_msg(char* dst, const char* m) { std::snprintf(dst, kErrLen, "%s", m ? m : ""); }
void set_global_error(const char* m) { set_msg(g_global_error, m); }

#ifndef DPLR_SPREAD_MIN_THREADS
#define DPLR_SPREAD_MIN_THREADS 256
#endif
#ifndef DPLR_GATHER_MIN_THREADS
#define DPLR_GATHER_MIN_THREADS 256
#endif
// spread blocks the x splits aim for (two per compute unit on a 256-CU part)
#ifndef DPLR_SPREAD_TARGET_BLOCKS
#define DPLR_SPREAD_TARGET_BLOCKS 512
#endif
#ifndef DPLR_SPREAD_MAX_SPLIT
#define DPLR_SPREAD_MAX_SPLIT 8
#endif
// particle chunks of the counting sort (one LDS histogram each) and the
// granularity of the chunk length; the per-bin chunk scan handles at most
// 16 x 16 chunks
#ifndef DPLR_SORT_CHUNKS
#define DPLR_SORT_CHUNKS 256
#endif
static_assert(DPLR_SORT_CHUNKS >= 1 && DPLR_SORT_CHUNKS <= 256, "sort chunk count out of range");
// rows per sort bin in plane mode (log2): the gather walks the particles in bin order
#ifndef DPLR_PLANE_QSHIFT
#define DPLR_PLANE_QSHIFT 4
#endif
#ifndef DPLR_SORT_CHUNK_ALIGN
#define DPLR_SORT_CHUNK_ALIGN 256
#endif
// launch shapes of the transform passes (complex elements per y-pass block,
// y rows per inverse-x block, columns per z-pass block)
#ifndef DPLR_FFTY_ELEMS
#define DPLR_FFTY_ELEMS 4096
#endif
#ifndef DPLR_IFFTX_ROWS
#define DPLR_IFFTX_ROWS 16
#endif
#ifndef DPLR_IXY_MIN_THREADS
#define DPLR_IXY_MIN_THREADS 64
#endif
#ifndef DPLR_IXY_AD_THREADS
#define DPLR_IXY_AD_THREADS 64
#endif
#ifndef DPLR_MIXED_QSHIFT
#define DPLR_MIXED_QSHIFT 4
#endif
#ifndef DPLR_MIXED_FUSED
#define DPLR_MIXED_FUSED 1
#endif
#ifndef DPLR_MIXED_ZCOLS
#define DPLR_MIXED_ZCOLS 16
#endif
#ifndef DPLR_FFTZ_COLS
#define DPLR_FFTZ_COLS 8
#endif

constexpr int kMinMesh = 16;
constexpr int kMaxMesh = 512;
constexpr int kMaxOrder = 8;
constexpr int kMinOrder = 2;
constexpr int kMaxQ32Mesh = 256;  // int32-quantised transforms are direct sums, O(K) per output
constexpr int64_t kMixedSplitMinParticles = 65536;  // split plane spread from this many particles

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// sizes with no prime factor other than 2, 3 and 5
bool is_235(int v) {
  if (v <= 0) return false;
  for (int f : {2, 3, 5})
    while (v % f == 0) v /= f;
  return v == 1;
}

// The plane/pencil kernels take power-of-two meshes of 16 to 512 points per
// axis; other 2-3-5 meshes run on the mixed-radix kernels.
bool tuned_mesh(const int* K) {
  for (int a = 0; a < 3; ++a)
    if (!is_pow2(K[a]) || K[a] < kMinMesh || K[a] > kMaxMesh) return false;
  return true;
}

int round_threads(long elems) {
  long t = (elems + kEPT - 1) / kEPT;
  t = ((t + 63) / 64) * 64;
  if (t < 64) t = 64;
  if (t > 1024) t = 1024;
  return (int)t;
}

dplr_lr_status validate(const dplr_lr_config* c, const char*& msg) {
  msg = "";
  if (!c) { msg = "config is NULL"; return DPLR_LR_E_INVALID; }
  for (int a = 0; a < 3; ++a) {
    if (c->mesh[a] <= 0) { msg = "mesh sizes must be positive"; return DPLR_LR_E_INVALID; }
    if (!is_235(c->mesh[a]) || c->mesh[a] > kMaxMesh) {
      msg = "mesh sizes must have no prime factors other than 2, 3 and 5 and be at most 512";
      return DPLR_LR_E_UNSUPPORTED;
    }
  }
  if (c->order < kMinOrder || c->order > kMaxOrder) {
    msg = "order must be in [2, 8]";
    return c->order <= 0 ? DPLR_LR_E_INVALID : DPLR_LR_E_UNSUPPORTED;
  }
  if (!tuned_mesh(c->mesh)) {
    for (int a = 0; a < 3; ++a) {
      if (c->mesh[a] < c->order) {
        msg = "mesh sizes below 16 or not powers of two must be at least the order";
        return DPLR_LR_E_UNSUPPORTED;
      }
    }
    if (c->flags & DPLR_LR_DIFF_AD) {
      msg = "analytic differentiation needs power-of-two meshes of 16 to 512 points";
      return DPLR_LR_E_UNSUPPORTED;
    }
  }
  if (!(c->beta > 0.0) || !std::isfinite(c->beta)) { msg = "beta must be positive and finite"; return DPLR_LR_E_INVALID; }
  if (!std::isfinite(c->coulomb_k)) { msg = "coulomb_k must be finite"; return DPLR_LR_E_INVALID; }
  if (c->precision != DPLR_LR_FP32 && c->precision != DPLR_LR_FP64) { msg = "precision must be FP32 or FP64"; return DPLR_LR_E_INVALID; }
  if (c->alias_range < 0 || c->alias_range > 4) { msg = "alias_range must be in [0, 4]"; return DPLR_LR_E_INVALID; }
  if (c->capacity < 0 || c->capacity > 0x7fffffffLL) { msg = "capacity must be in [0, 2^31-1]"; return DPLR_LR_E_INVALID; }
  if (c->flags & ~(uint32_t)(DPLR_LR_ACCUMULATE | DPLR_LR_NO_VIRIAL | DPLR_LR_DIFF_AD)) {
    msg = "unknown flag bits";
    return DPLR_LR_E_INVALID;
  }
  return DPLR_LR_OK;
}

}  // namespace

struct dplr_lr_plan_s {
  dplr_lr_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;
  bool fp64 = false;
  size_t tsize = 4;
  Geo geo{};
  double box[3] = {0, 0, 0};
  bool has_box = false;
  size_t lds_budget = 65536;
  size_t lds_spread = 0, lds_ffty = 0, lds_z = 0, lds_ifftx = 0, lds_ixy = 0;
  bool plane = false;         // whole z planes fit in LDS: spread + x and y transforms in one kernel
  bool ixy = false;           // inverse y and x transforms of a plane component in one kernel
  bool mixed = false;         // mesh outside the tuned kernels: mixed-radix path
  long long* mmesh = nullptr; // mixed-radix path: fixed-point mesh [Kz][Ky][Kx]
  void* mspec = nullptr;      // ... its full complex spectrum
  void* mfield = nullptr;     // ... three full field spectra, transformed back in place
  void* mpacked = nullptr;    // ... the three real fields interleaved (x, y, z, unused) per mesh point
  int mblk = 0;               // ... blocks (and partials) of the ik multiply
  size_t lds_mplane = 0;      // ... LDS of the plane spread (0: the plane does not fit; global atomics)
  void* mrec = nullptr;       // ... per-particle stencil offsets and charge (plane spread)
  int* mspk = nullptr;        // ... per-particle packed stencil starts (plane spread)
  int msplit = 1;             // ... particle ranges per plane of the split plane spread (partials in mmesh)
  size_t mfused = 0;          // ... LDS of the fused plane kernels (0: the per-axis transforms)
  int mzc = 1;                // ... columns per block of the fused z pass
  int mzblk = 0;              // ... blocks (and partials) of the fused z pass
  int q32_nodes[3] = {0, 0, 0};  // int32-quantised transforms: node blocks per axis (0: off)
  double q32_scale = 0.0;
  unsigned long long* q32_clamped = nullptr;  // saturated partial values of the last compute
  int thr_spread = 256, thr_ffty = 256, thr_z = 256, thr_ifftx = 256, thr_ixy = 256;
  // device workspace
  int* bin_count = nullptr;
  int* bin_start = nullptr;
  int* bin_cursor = nullptr;
  int* bin_hist = nullptr;    // [max chunks][nbins]
  unsigned* qmax = nullptr;   // max |q| bits: per sort chunk, or one word (global-atomic sort)
  bool block_hist = false;    // bins fit in LDS: sort without global atomics
  int max_chunks = DPLR_SORT_CHUNKS;
  void* sorted = nullptr;
  int* perm = nullptr;
  int* sidx = nullptr;
  void* spec = nullptr;
  void* fspec = nullptr;
  void* field = nullptr;   // real fields [Kz][Ky][Kx] x (Ex, Ey, Ez)
  double* G = nullptr;
  double* partials = nullptr;
  void* twiddle = nullptr;
  int64_t ws_bytes = 0;
  std::vector<void*> allocs;
  char err[kErrLen] = "";
  // instrumentation: HIP event pairs around each kernel of compute
  bool prof = false;
  struct ProfRec { int stage; hipEvent_t a, b; };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[16] = {0};
  int64_t prof_calls[16] = {0};
};

namespace {

const char* const kStageNames[] = {"bin_count", "bin_scan", "bin_scatter", "spread_fftx", "ffty_fwd",
                                   "fftz_poisson", "ffty_inv_reduce", "ifftx", "gather", "spread_xy",
                                   "ifft_xy_reduce", "mixed_spread", "mixed_fft_fwd", "mixed_poisson",
                                   "mixed_fft_inv", "mixed_gather"};
constexpr int kNumStages = 16;
static_assert(kNumStages <= 16, "profile slots");

hipEvent_t prof_event(dplr_lr_plan p) {
  if (!p->prof_pool.empty()) {
    hipEvent_t e = p->prof_pool.back();
    p->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Records an event pair around one kernel launch when instrumentation is on.
struct ProfScope {
  dplr_lr_plan p;
  int stage;
  hipEvent_t a = nullptr;
  ProfScope(dplr_lr_plan p_, int s) : p(p_), stage(s) {
    if (p->prof) {
      a = prof_event(p);
      (void)hipEventRecord(a, p->stream);
    }
  }
  ~ProfScope() {
    if (p->prof && a) {
      hipEvent_t b = prof_event(p);
      (void)hipEventRecord(b, p->stream);
      p->prof_pending.push_back({stage, a, b});
    }
  }
};

dplr_lr_status fail(dplr_lr_plan p, dplr_lr_status st, const char* m) {
  set_msg(p ? p->err : g_global_error, m);
  return st;
}

dplr_lr_status hip_fail(dplr_lr_plan p, hipError_t e, const char* what) {
  char m[kErrLen];
  std::snprintf(m, sizeof(m), "%s: %s", what, hipGetErrorString(e));
  return fail(p, e == hipErrorOutOfMemory ? DPLR_LR_E_NOMEM : DPLR_LR_E_DEVICE, m);
}

template <typename T>
size_t cpx_bytes() { return sizeof(cpx<T>); }

// Choose tilings that fit the LDS budget.
bool choose_geometry(dplr_lr_plan p) {
  Geo& g = p->geo;
  const int Kx = p->cfg.mesh[0], Ky = p->cfg.mesh[1], Kz = p->cfg.mesh[2];
  const int P = p->cfg.order;
  const size_t ts = p->tsize, cs = 2 * ts;
  g.K[0] = Kx; g.K[1] = Ky; g.K[2] = Kz;
  g.Kh = Kx / 2 + 1;
  g.qshift = 2;
  g.split_by_index = 0;
  g.NQ = Ky >> g.qshift;
  g.twN = std::max(Kx, std::max(Ky, Kz));
  const size_t twb = g.twN * cs;
  const size_t budget = p->lds_budget - 1024;  // static LDS (ranges, reductions)

  // plane spread: one z plane of 64-bit accumulators (rows of Kx + p - 1),
  // reused for the x- and y-transform tiles, 1024 threads holding at most 16
  // values each
  {
    const size_t b_acc = (size_t)Ky * (Kx + P - 1) * sizeof(long long);
    const size_t b_tx = (size_t)(Ky / 2) * (padded_len(Kx) + 1) * cs;
    const size_t b_ty = (size_t)g.Kh * (padded_len(Ky) + 1) * cs;
    const size_t b = std::max(b_acc, std::max(b_tx, b_ty)) + twb;
    p->plane = b <= budget && (long)Kx * Ky <= 16L * 1024 && (long)g.Kh * Ky <= 16L * 1024;
    if (p->plane) {
      p->lds_spread = b;
      p->thr_spread = 1024;
      const int per_cu = std::max<int>(1, (int)(p->lds_budget / (b + 1024)));
      const int target = std::min(1024, 256 * per_cu);
      g.nsplit = 1;
      while (Kz * g.nsplit < target && g.nsplit < DPLR_SPREAD_MAX_SPLIT && Kx / (2 * g.nsplit) >= 4) g.nsplit *= 2;
      g.xs = Kx / g.nsplit;
      // particles are split by index parity: each split still covers the
      // whole plane, so its LDS atomics spread over every row and column
      g.split_by_index = 1;
      // a plane visits all row groups of its planes: coarse groups keep the
      // sort small while consecutive particles stay close in y
      g.qshift = std::min(DPLR_PLANE_QSHIFT, 31 - __builtin_clz((unsigned)Ky));
      g.NQ = Ky >> g.qshift;
      g.nbins = g.nsplit * Kz * g.NQ;
      g.scy = Ky; g.scz = 1; g.spy = 1; g.spz = Kz;
    }
  }
  // spread pencils: two blocks of at most 512 threads per compute unit, so a
  // block gets half of the LDS; the largest cross-section that fits wins
  // (fewest particles visited twice)
  const size_t sbudget = std::min(budget, p->lds_budget / 2 - 1024);
  const int cand[][2] = {{16, 8}, {16, 4}, {8, 4}, {16, 2}, {8, 2}, {4, 4}, {4, 2}, {8, 1}, {4, 1}};
  if (!p->plane) g.scy = 0;
  for (auto& c : cand) {
    if (p->plane) break;
    const int cy = c[0], cz = c[1];
    if (cy > Ky || cz > Kz || (cy * cz) % 2) continue;
    // 64-bit fixed-point accumulators (rows of Kx + p - 1), converted in
    // place to padded complex pairs
    const size_t accb = (size_t)cy * cz * (Kx + P - 1) * sizeof(long long);
    const size_t cpxb = (size_t)(cy * cz / 2) * (padded_len(Kx) + 1) * cs;
    const size_t b = std::max(accb, cpxb) + twb;
    const long long elems = (long long)cy * cz * Kx;
    if (b <= sbudget && elems <= 16LL * 512) {
      g.scy = cy; g.scz = cz; p->lds_spread = b;
      break;
    }
  }
  if (!p->plane) {
    if (!g.scy) return false;
    g.spy = Ky / g.scy; g.spz = Kz / g.scz;
    // the in-place fixed-point conversion holds at most 16 values per thread
    p->thr_spread = std::max(DPLR_SPREAD_MIN_THREADS, round_threads((long)g.scy * g.scz / 2 * Kx));
    while ((long)p->thr_spread * 16 < (long)g.scy * g.scz * Kx && p->thr_spread < 512) p->thr_spread += 64;
    if ((long)p->thr_spread * 16 < (long)g.scy * g.scz * Kx || p->thr_spread > 512) return false;
    // x splits: more blocks when the pencils alone do not fill the device
    g.nsplit = 1;
    while (g.spy * g.spz * g.nsplit < DPLR_SPREAD_TARGET_BLOCKS && g.nsplit < DPLR_SPREAD_MAX_SPLIT &&
           Kx / (2 * g.nsplit) >= 8)
      g.nsplit *= 2;
    g.xs = Kx / g.nsplit;
    g.nbins = g.nsplit * Kz * g.NQ;
  }

  // inverse x pass: xyb rows of y of the three fields per block
  g.xyb = std::min(DPLR_IFFTX_ROWS, Ky);
  while (g.xyb > 2 && ((size_t)(3 * g.xyb / 2) * (padded_len(Kx) + 1) * cs + twb > budget ||
                       (long)(3 * g.xyb / 2) * Kx > (long)kEPT * 512))
    g.xyb /= 2;
  p->lds_ifftx = (size_t)(3 * g.xyb / 2) * (padded_len(Kx) + 1) * cs + twb;
  p->thr_ifftx = std::max(round_threads((long)(3 * g.xyb / 2) * Kx), ((3 * g.xyb / 2 + 63) / 64) * 64);
  if (p->thr_ifftx > 512) return false;

  // y pass: blocks of zb contiguous rows, about 1024 complex elements
  g.zb = std::max(1, std::min(Kz, DPLR_FFTY_ELEMS / Ky));
  while (g.zb > 1 && ((size_t)g.zb * (padded_len(Ky) + 1) * cs + twb > budget ||
                      round_threads((long)g.zb * Ky) > kFftyThreads))
    g.zb /= 2;
  p->thr_ffty = round_threads((long)g.zb * Ky);
  if (p->thr_ffty > kFftyThreads) return false;
  // the inverse pass also hosts the final reduction: 7 doubles per thread
  p->lds_ffty = std::max((size_t)g.zb * (padded_len(Ky) + 1) * cs + twb, (size_t)7 * p->thr_ffty * sizeof(double));

  // z pass: yb columns x Kz x 3 fields
  g.yb = std::min(DPLR_FFTZ_COLS, Ky);
  while (g.yb > 1 && ((size_t)3 * g.yb * Kz * cs + twb > budget || (long)3 * g.yb * Kz > (long)kEPT * 1024)) g.yb /= 2;
  p->lds_z = (size_t)3 * g.yb * Kz * cs + twb;
  p->thr_z = round_threads((long)3 * g.yb * Kz);
  g.nzblk = g.Kh * (Ky / g.yb);
  g.zgroup = std::max<int>(1, (int)(128 / (g.yb * cs)));

  // fused inverse y + x pass (plane mode): one block per (z plane, component)
  p->ixy = false;
  if (p->plane && Kz % 8 == 0) {
    const long e_y = (long)g.Kh * Ky, e_x = (long)(Ky / 2) * Kx;
    // analytic differentiation has one component per plane (Kz blocks): more threads per block
    const int thr_min = (p->cfg.flags & DPLR_LR_DIFF_AD) ? DPLR_IXY_AD_THREADS : DPLR_IXY_MIN_THREADS;
    const int thr = std::max(thr_min, (int)(((std::max(e_y, e_x) + kEPT - 1) / kEPT + 63) / 64 * 64));
    const size_t b_y = (size_t)g.Kh * (padded_len(Ky) + 1) * cs, b_x = (size_t)(Ky / 2) * (padded_len(Kx) + 1) * cs;
    const size_t lds = std::max(std::max(b_y, b_x) + twb, (size_t)7 * thr * sizeof(double));
    if (thr <= 1024 && lds <= budget) {
      p->ixy = true;
      p->thr_ixy = thr;
      p->lds_ixy = lds;
    }
  }
  return true;
}

template <typename T>
void fill_twiddles(std::vector<unsigned char>& out, int N) {
  out.resize(sizeof(cpx<T>) * N);
  cpx<T>* w = reinterpret_cast<cpx<T>*>(out.data());
  for (int k = 0; k < N; ++k) {
    const double th = -2.0 * M_PI * (double)k / (double)N;
    w[k].x = (T)std::cos(th);
    w[k].y = (T)std::sin(th);
  }
}

dplr_lr_status alloc(dplr_lr_plan p, void** ptr, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) return hip_fail(p, e, what);
  p->allocs.push_back(*ptr);
  p->ws_bytes += (int64_t)bytes;
  return DPLR_LR_OK;
}

void free_all(dplr_lr_plan p) {
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
}

// Raises a kernel's dynamic-LDS limit to at least `bytes`, never lowering a
// limit that another plan set (all plans share the kernels).  Returns false
// when the runtime refuses (the error is cleared).
bool raise_lds_limit(const void* f, size_t bytes) {
  static std::mutex mu;
  static std::vector<std::pair<const void*, size_t>> set;
  std::lock_guard<std::mutex> lock(mu);
  for (auto& e : set)
    if (e.first == f && e.second >= bytes) return true;
  if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  for (auto& e : set)
    if (e.first == f) { e.second = bytes; return true; }
  set.emplace_back(f, bytes);
  return true;
}

template <typename T>
void set_lds_attrs(dplr_lr_plan p) {
  // kernels whose dynamic LDS can exceed the 64 KiB default
  // a refusal is cleared here: a kernel that needed it then fails at its own launch
  auto attr = [&](const void* f, size_t b) {
    if (b > 65536) (void)raise_lds_limit(f, b);
  };
  switch (p->cfg.order) {
#define DPLR_ATTR(PP)                                                        \
  case PP:                                                                   \
    attr((const void*)k_spread_fftx<T, PP>, p->lds_spread);                  \
    attr((const void*)k_spread_xy<T, PP>, p->lds_spread);                    \
    break;
    DPLR_ATTR(2) DPLR_ATTR(3) DPLR_ATTR(4) DPLR_ATTR(5) DPLR_ATTR(6) DPLR_ATTR(7) DPLR_ATTR(8)
#undef DPLR_ATTR
  }
  // LDS histograms and placement ranks: only when the bins fit (block_hist)
  if (p->block_hist) switch (p->cfg.order) {
#define DPLR_ATTR2(PP)                                                                   \
  case PP:                                                                               \
    attr((const void*)k_bin_hist<T, PP>, sizeof(int) * (size_t)p->geo.nbins);           \
    attr((const void*)k_bin_place<T, PP>, 2 * sizeof(int) * (size_t)p->geo.nbins);      \
    break;
    DPLR_ATTR2(2) DPLR_ATTR2(3) DPLR_ATTR2(4) DPLR_ATTR2(5) DPLR_ATTR2(6) DPLR_ATTR2(7) DPLR_ATTR2(8)
#undef DPLR_ATTR2
  }
  attr((const void*)k_ffty<T, false>, p->lds_ffty);
  attr((const void*)k_ffty<T, true>, p->lds_ffty);
  attr((const void*)k_fftz_poisson<T>, p->lds_z);
  attr((const void*)k_ifftx<T>, p->lds_ifftx);
  if (p->ixy) attr((const void*)k_ifft_xy<T>, p->lds_ixy);
}

template <typename T, int P>
dplr_lr_status launch_step(dplr_lr_plan p, int64_t n_ion, const void* ion_pos, const void* ion_q, int64_t n_wc,
                           const void* wc_pos, const void* wc_q, void* ion_force, void* wc_force, double* energy,
                           double* virial) {
  const Geo& g = p->geo;
  hipStream_t s = p->stream;
  const int64_t n = n_ion + n_wc;
  const double ih[3] = {g.K[0] / p->box[0], g.K[1] / p->box[1], g.K[2] / p->box[2]};
  const cpx<T>* tw = reinterpret_cast<const cpx<T>*>(p->twiddle);
  T4<T>* sorted = reinterpret_cast<T4<T>*>(p->sorted);
  cpx<T>* spec = reinterpret_cast<cpx<T>*>(p->spec);
  cpx<T>* fspec = reinterpret_cast<cpx<T>*>(p->fspec);
  const size_t nspec = (size_t)g.Kh * g.K[1] * g.K[2];
  const T* ip = (const T*)ion_pos;
  const T* wp = (const T*)wc_pos;

  int nqpart = 1;  // charge-maximum words the spread reads
  if (p->block_hist) {
    // chunk size: a multiple of DPLR_SORT_CHUNK_ALIGN, at most max_chunks chunks
    constexpr int64_t ca = DPLR_SORT_CHUNK_ALIGN;
    int64_t chunk = std::max<int64_t>(ca, ((n + p->max_chunks - 1) / p->max_chunks + ca - 1) / ca * ca);
    const int nblk = (int)((n + chunk - 1) / chunk);
    const size_t lds = sizeof(int) * g.nbins;
    if (n > 0) {
      ProfScope ps(p, 0);
      hipLaunchKernelGGL((k_bin_hist<T, P>), dim3(nblk), dim3(1024), lds, s, ip, wp, n_ion, n, ih[0], ih[1], ih[2],
                         p->bin_hist, (int)chunk, g);
    }
    {
      ProfScope ps(p, 1);
      // per-bin chunk offsets and bin totals; the placement scans the totals
      if (n > 0) {
        hipLaunchKernelGGL(k_bin_colscan, dim3((g.nbins + 63) / 64), dim3(1024), 0, s, p->bin_hist, p->bin_count,
                           nblk, g.nbins);
      } else {
        hipLaunchKernelGGL(k_fill_int, dim3((g.nbins + 1 + 255) / 256), dim3(256), 0, s, p->bin_start, g.nbins + 1,
                           0);
      }
    }
    if (n > 0) {
      ProfScope ps(p, 2);
      hipLaunchKernelGGL((k_bin_place<T, P>), dim3(nblk), dim3(1024), 2 * lds, s, ip, wp, (const T*)ion_q,
                         (const T*)wc_q, n_ion, n, ih[0], ih[1], ih[2], p->bin_hist, p->bin_count, p->bin_start,
                         sorted, p->sidx, p->perm, p->qmax, (int)chunk, g);
    }
    nqpart = n > 0 ? nblk : 0;
  } else {
    if (n > 0) {
      const int nb = (int)((n + 255) / 256);
      ProfScope ps(p, 0);
      hipLaunchKernelGGL((k_bin_count<T, P>), dim3(nb), dim3(256), 0, s, ip, wp, n_ion, n, ih[0], ih[1], ih[2],
                         p->bin_count, g);
    }
    {
      ProfScope ps(p, 1);
      hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, p->bin_count, p->bin_start, p->bin_cursor,
                         g.nbins, p->qmax);
    }
    if (n > 0) {
      const int nb = (int)((n + 255) / 256);
      ProfScope ps(p, 2);
      hipLaunchKernelGGL((k_bin_scatter<T, P>), dim3(nb), dim3(256), 0, s, ip, wp, (const T*)ion_q, (const T*)wc_q,
                         n_ion, n, ih[0], ih[1], ih[2], p->bin_cursor, sorted, p->sidx, p->perm, p->qmax, g);
    }
  }
  if (p->plane) {
    ProfScope ps(p, 9);
    hipLaunchKernelGGL((k_spread_xy<T, P>), dim3(g.K[2] * g.nsplit), dim3(p->thr_spread), p->lds_spread, s, sorted,
                       p->sidx, p->bin_start, (const unsigned*)p->qmax, nqpart, spec, nspec, tw, g);
  } else {
    {
      ProfScope ps(p, 3);
      hipLaunchKernelGGL((k_spread_fftx<T, P>), dim3(g.spy * g.spz * g.nsplit), dim3(p->thr_spread), p->lds_spread,
                         s, sorted, p->sidx, p->bin_start, (const unsigned*)p->qmax, nqpart, spec, nspec, tw, g);
    }
    {
      ProfScope ps(p, 4);
      hipLaunchKernelGGL((k_ffty<T, false>), dim3(g.Kh * (g.K[2] / g.zb)), dim3(p->thr_ffty), p->lds_ffty, s, spec, tw,
                         g, g.nsplit, nspec, (const double*)nullptr, 0.0, (double*)nullptr, (double*)nullptr);
    }
  }
  PoissonConsts pc;
  for (int a = 0; a < 3; ++a) pc.two_pi_over_L[a] = 2.0 * M_PI / p->box[a];
  pc.inv_4beta2 = 1.0 / (4.0 * p->cfg.beta * p->cfg.beta);
  // field components: three (ik) or the potential alone (analytic differentiation)
  const bool ad = (p->cfg.flags & DPLR_LR_DIFF_AD) != 0;
  const int ncomp = ad ? 1 : 3;
  {
    ProfScope ps(p, 5);
    hipLaunchKernelGGL((k_fftz_poisson<T>), dim3((g.nzblk + 8 * g.zgroup - 1) / (8 * g.zgroup) * 8 * g.zgroup),
                       dim3(p->thr_z), p->lds_z, s, spec,
                       p->plane ? g.nsplit : 1, nspec, ncomp, fspec, p->G, p->partials, tw, g, pc);
  }
  const double V = p->box[0] * p->box[1] * p->box[2];
  const bool want_virial = !(p->cfg.flags & DPLR_LR_NO_VIRIAL) && virial;
  if (p->ixy) {
    ProfScope ps(p, 10);
    hipLaunchKernelGGL((k_ifft_xy<T>), dim3(ncomp * g.K[2]), dim3(p->thr_ixy), p->lds_ixy, s, fspec,
                       reinterpret_cast<T*>(p->field), ncomp, ad ? kGatherAdPad : 0, tw, g, (const double*)p->partials,
                       p->cfg.coulomb_k / (2.0 * V), energy, want_virial ? virial : (double*)nullptr);
  } else {
    ProfScope ps(p, 6);
    hipLaunchKernelGGL((k_ffty<T, true>), dim3(ncomp * g.Kh * (g.K[2] / g.zb)), dim3(p->thr_ffty), p->lds_ffty, s,
                       fspec, tw, g, 1, (size_t)0, (const double*)p->partials, p->cfg.coulomb_k / (2.0 * V), energy,
                       want_virial ? virial : (double*)nullptr);
  }
  if (n > 0) {
    if (!p->ixy) {
      ProfScope ps(p, 7);
      hipLaunchKernelGGL((k_ifftx<T>), dim3(g.K[2] * (g.K[1] / g.xyb)), dim3(p->thr_ifftx), p->lds_ifftx, s, fspec,
                         reinterpret_cast<T*>(p->field), ncomp, tw, g);
    }
    {
      ProfScope ps(p, 8);
      constexpr int kXcd = 8;  // MI355X: 8 XCDs, blocks dealt round-robin
      const int per_block = 4 * (64 / P);
      const int nchunks = (int)((n + per_block - 1) / per_block);
      const int nblk = (nchunks + kXcd - 1) / kXcd * kXcd;
      const int acc = (p->cfg.flags & DPLR_LR_ACCUMULATE) ? 1 : 0;
      if (ad && P <= 6) {
        // one particle per lane, chunks of 256 sorted particles
        const int nch = (int)((n + 255) / 256);
        const int nb = (nch + kXcd - 1) / kXcd * kXcd;
        hipLaunchKernelGGL((k_gather_ad<T, P>), dim3(nb), dim3(256), 0, s, reinterpret_cast<const T*>(p->field),
                           sorted, p->sidx, p->perm, (int)n, nch, (T*)ion_force, (T*)wc_force, n_ion,
                           (T)(p->cfg.coulomb_k / V), (T)(g.K[0] / p->box[0]), (T)(g.K[1] / p->box[1]),
                           (T)(g.K[2] / p->box[2]), acc, kXcd, g);
      } else if (ad) {
        hipLaunchKernelGGL((k_gather_ad_lanes<T, P>), dim3(nblk), dim3(256), 0, s,
                           reinterpret_cast<const T*>(p->field), sorted, p->sidx, p->perm, (int)n, nchunks,
                           (T*)ion_force, (T*)wc_force, n_ion, (T)(p->cfg.coulomb_k / V), (T)(g.K[0] / p->box[0]),
                           (T)(g.K[1] / p->box[1]), (T)(g.K[2] / p->box[2]), acc, kXcd, g);
      } else {
        hipLaunchKernelGGL((k_gather<T, P>), dim3(nblk), dim3(256), 0, s, reinterpret_cast<const F3<T>*>(p->field),
                           sorted, p->sidx, p->perm, (int)n, nchunks, (T*)ion_force, (T*)wc_force, n_ion,
                           (T)(p->cfg.coulomb_k / V), acc, kXcd, g);
      }
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(p, e, "kernel launch");
  return DPLR_LR_OK;
}

// Mixed-radix path: spread, forward x/y/z transforms, ik multiply, the three
// inverse x/y/z transforms, energy/virial reduction, gather.
// packed: the last (z) pass writes the real parts interleaved there
template <typename T>
void launch_mixed_fft(dplr_lr_plan p, cpx<T>* data, int ncomp, int sign, T* packed) {
  const int K[3] = {p->geo.K[0], p->geo.K[1], p->geo.K[2]};
  const int64_t ntot = (int64_t)K[0] * K[1] * K[2];
  const int64_t stride[3] = {1, K[0], (int64_t)K[0] * K[1]};
  for (int a = 0; a < 3; ++a) {
    const int64_t rows = ntot / K[a];
    // columns per block: side by side in memory for the y and z passes, at
    // most 16 and 32 KiB of LDS per buffer
    int C = 1;
    if (a > 0)
      while (C < 16 && stride[a] % (2 * C) == 0 && 2 * (size_t)C * K[a] * sizeof(cpx<T>) <= 32768) C *= 2;
    else  // x rows: several consecutive rows per block, at most about 256 threads' work
      while (C < 16 && rows % (2 * C) == 0 && 2 * C * K[a] <= 1024 && 2 * (size_t)C * K[a] * sizeof(cpx<T>) <= 32768)
        C *= 2;
    const int thr = std::min(256, std::max(64, (C * K[a] / 2 + 63) / 64 * 64));
    hipLaunchKernelGGL(k_mixed_fft_axis<T>, dim3((unsigned)(rows / C), (unsigned)ncomp), dim3(thr),
                       (2 * C + 1) * sizeof(cpx<T>) * K[a], p->stream, data, K[a], stride[a], ntot, sign,
                       a == 2 ? packed : (T*)nullptr, C);
  }
}

template <typename T>
void launch_mixed_dft_q32(dplr_lr_plan p, cpx<T>* data, int ncomp, int sign, T* packed) {
  const int K[3] = {p->geo.K[0], p->geo.K[1], p->geo.K[2]};
  const int64_t ntot = (int64_t)K[0] * K[1] * K[2];
  const int64_t stride[3] = {1, K[0], (int64_t)K[0] * K[1]};
  for (int a = 0; a < 3; ++a) {
    const int64_t rows = ntot / K[a];
    hipLaunchKernelGGL(k_mixed_dft_q32<T>, dim3((unsigned)rows, (unsigned)ncomp), dim3(64), sizeof(cpx<T>) * K[a],
                       p->stream, data, K[a], stride[a], ntot, sign, p->q32_nodes[a], p->q32_scale,
                       a == 2 ? packed : (T*)nullptr, p->q32_clamped);
  }
}

template <typename T, int P>
dplr_lr_status launch_mixed(dplr_lr_plan p, int64_t n_ion, const void* ion_pos, const void* ion_q, int64_t n_wc,
                            const void* wc_pos, const void* wc_q, void* ion_force, void* wc_force, double* energy,
                            double* virial) {
  const Geo& g = p->geo;
  hipStream_t s = p->stream;
  const int64_t n = n_ion + n_wc;
  const int64_t ntot = (int64_t)g.K[0] * g.K[1] * g.K[2];
  const double ih[3] = {g.K[0] / p->box[0], g.K[1] / p->box[1], g.K[2] / p->box[2]};
  cpx<T>* spec = reinterpret_cast<cpx<T>*>(p->mspec);
  cpx<T>* field = reinterpret_cast<cpx<T>*>(p->mfield);
  // quantised transforms: the field spectra carry k_e / V so that the inverse
  // transforms work on the field itself (O(1) values)
  const bool q32 = p->q32_nodes[0] > 0;
  // spread: one thread per (particle, stencil plane); gather: 256 / P particles per block
  const unsigned nbp = (unsigned)((n * P + 255) / 256);
  const int nchg = (int)((n + mixed_gather_per_block<P>() - 1) / mixed_gather_per_block<P>());  // gather chunks; grid a multiple of the XCDs
  const unsigned nbg = (unsigned)((nchg + kNumXcd - 1) / kNumXcd * kNumXcd);
  // split the particles over S blocks per plane when the planes alone
  // leave most compute units idle and there are enough particles
  // fused plane kernels (not for the int32 transforms, which run per axis)
  const bool fused = p->mfused > 0 && !q32;
  const int S = n >= kMixedSplitMinParticles ? p->msplit : 1;
  const int npart = fused ? p->mzblk : p->mblk;  // energy/virial block partials of this call
  if (p->lds_mplane) {
    // counting sort by (particle split, stencil-start plane) with the plane
    // kernels' sort, then one block per (z plane, split): spread in LDS,
    // written straight into the spectrum buffer (or integer partial planes)
    ProfScope ps(p, 11);
    Geo gs = g;
    gs.nsplit = S;
    gs.nbins = S * g.K[2] * g.NQ;
    const int64_t ca = DPLR_SORT_CHUNK_ALIGN;
    const int64_t chunk = std::max<int64_t>(ca, ((n + p->max_chunks - 1) / p->max_chunks + ca - 1) / ca * ca);
    const int nblk = (int)((n + chunk - 1) / chunk);
    const size_t lds = sizeof(int) * gs.nbins;
    if (n > 0) {
      hipLaunchKernelGGL((k_bin_hist<T, P>), dim3(nblk), dim3(1024), lds, s, (const T*)ion_pos, (const T*)wc_pos,
                         n_ion, n, ih[0], ih[1], ih[2], p->bin_hist, (int)chunk, gs);
      hipLaunchKernelGGL(k_bin_colscan, dim3((gs.nbins + 63) / 64), dim3(1024), 0, s, p->bin_hist, p->bin_count,
                         nblk, gs.nbins);
      hipLaunchKernelGGL((k_bin_place<T, P>), dim3(nblk), dim3(1024), 2 * lds, s, (const T*)ion_pos,
                         (const T*)wc_pos, (const T*)ion_q, (const T*)wc_q, n_ion, n, ih[0], ih[1], ih[2],
                         p->bin_hist, p->bin_count, p->bin_start, (T4<T>*)p->mrec, p->mspk, p->perm, p->qmax,
                         (int)chunk, gs);
    } else {
      hipLaunchKernelGGL(k_fill_int, dim3((gs.nbins + 1 + 255) / 256), dim3(256), 0, s, p->bin_start, gs.nbins + 1,
                         0);
    }
    if (fused)
      hipLaunchKernelGGL((k_mixed_spread_xy<T, P>), dim3(g.K[2], S), dim3(1024), p->mfused, s,
                         (const T4<T>*)p->mrec, (const int*)p->mspk, (const int*)p->bin_start, gs,
                         (const unsigned*)p->qmax, n > 0 ? nblk : 0, reinterpret_cast<cpx<T>*>(p->mmesh));
    else
      hipLaunchKernelGGL((k_mixed_spread_sorted<T, P>), dim3(g.K[2], S), dim3(1024), p->lds_mplane, s,
                         (const T4<T>*)p->mrec, (const int*)p->mspk, (const int*)p->bin_start, gs, spec, p->mmesh);
    if (S > 1 && !fused)
      hipLaunchKernelGGL(k_mixed_combine<T>, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s,
                         (const long long*)p->mmesh, S, ntot, spec);
  } else if (n > 0) {
    ProfScope ps(p, 11);
    hipLaunchKernelGGL((k_mixed_spread<T, P>), dim3(nbp), dim3(256), 0, s, (const T*)ion_pos, (const T*)ion_q,
                       (const T*)wc_pos, (const T*)wc_q, n_ion, n, ih[0], ih[1], ih[2], g.K[0], g.K[1], g.K[2],
                       (unsigned long long*)p->mmesh);
  }
  if (q32) {
    // the saturation count of this call starts at zero (a fill kernel, not a memset)
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, reinterpret_cast<int*>(p->q32_clamped), 2, 0);
  }
  if (!fused) {
    ProfScope ps(p, 12);
    if (!p->lds_mplane)
      hipLaunchKernelGGL(k_mixed_unfix<T>, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, p->mmesh, spec,
                         ntot);
    if (q32) launch_mixed_dft_q32<T>(p, spec, 1, -1, (T*)nullptr);
    else launch_mixed_fft<T>(p, spec, 1, -1, (T*)nullptr);
  }
  PoissonConsts pc;
  for (int a = 0; a < 3; ++a) pc.two_pi_over_L[a] = 2.0 * M_PI / p->box[a];
  pc.inv_4beta2 = 1.0 / (4.0 * p->cfg.beta * p->cfg.beta);
  const double V = p->box[0] * p->box[1] * p->box[2];
  const bool want_virial = !(p->cfg.flags & DPLR_LR_NO_VIRIAL) && virial;
  {
    ProfScope ps(p, 13);
    if (fused) {
      const int C = p->mzc;
      hipLaunchKernelGGL(k_mixed_fftz_poisson<T>, dim3((unsigned)p->mzblk), dim3(kFusedZThreads),
                         (size_t)(2 * C + 1) * g.K[2] * sizeof(cpx<T>), s, (const cpx<T>*)p->mmesh, S, field,
                         field + ntot, p->G, g.K[0], g.K[1], g.K[2], C, pc, 1.0, p->partials);
    } else {
      hipLaunchKernelGGL(k_mixed_poisson<T>, dim3((unsigned)p->mblk), dim3(256), 0, s, spec, field, p->G, g.K[0],
                         g.K[1], g.K[2], pc, q32 ? p->cfg.coulomb_k / V : 1.0, p->partials);
    }
    // with particles, block 0 of the gather reduces the partials instead
    if (n == 0)
      hipLaunchKernelGGL(k_mixed_reduce, dim3(1), dim3(256), 0, s, (const double*)p->partials, npart,
                         p->cfg.coulomb_k / (2.0 * V), energy, want_virial ? virial : (double*)nullptr);
  }
  if (n > 0) {
    {
      ProfScope ps(p, 14);
      if (fused)
        hipLaunchKernelGGL(k_mixed_ifft_xy<T>, dim3(g.K[2], 2), dim3(1024), p->mfused, s, (const cpx<T>*)field,
                           (const cpx<T>*)(field + ntot), g.K[0], g.K[1], (T*)p->mpacked);
      else if (q32) launch_mixed_dft_q32<T>(p, field, 3, +1, (T*)p->mpacked);
      else launch_mixed_fft<T>(p, field, 3, +1, (T*)p->mpacked);
    }
    ProfScope ps(p, 15);
    if (p->lds_mplane)  // the sorted records of the spread
      hipLaunchKernelGGL((k_mixed_gather_sorted<T, P>), dim3(nbg), dim3(256), 0, s, (const T4<T>*)p->mrec,
                         (const int*)p->mspk, (const int*)p->perm, n_ion, n, g.K[0], g.K[1], g.K[2],
                         (const T4<T>*)p->mpacked, (T*)ion_force, (T*)wc_force,
                         q32 ? (T)1 : (T)(p->cfg.coulomb_k / V), (p->cfg.flags & DPLR_LR_ACCUMULATE) ? 1 : 0,
                         (const double*)p->partials, npart, p->cfg.coulomb_k / (2.0 * V), energy,
                         want_virial ? virial : (double*)nullptr, nchg);
    else
      hipLaunchKernelGGL((k_mixed_gather<T, P>), dim3(nbg), dim3(256), 0, s, (const T*)ion_pos, (const T*)ion_q,
                         (const T*)wc_pos, (const T*)wc_q, n_ion, n, ih[0], ih[1], ih[2], g.K[0], g.K[1], g.K[2],
                         (const T4<T>*)p->mpacked, (T*)ion_force, (T*)wc_force,
                         q32 ? (T)1 : (T)(p->cfg.coulomb_k / V), (p->cfg.flags & DPLR_LR_ACCUMULATE) ? 1 : 0,
                         (const double*)p->partials, npart, p->cfg.coulomb_k / (2.0 * V), energy,
                         want_virial ? virial : (double*)nullptr, nchg);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(p, e, "kernel launch");
  return DPLR_LR_OK;
}

template <typename T>
dplr_lr_status dispatch_order(dplr_lr_plan p, int64_t n_ion, const void* a, const void* b, int64_t n_wc,
                              const void* c, const void* d, void* e, void* f, double* en, double* vir) {
  if (p->mixed) {
    switch (p->cfg.order) {
      case 2: return launch_mixed<T, 2>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
      case 3: return launch_mixed<T, 3>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
      case 4: return launch_mixed<T, 4>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
      case 5: return launch_mixed<T, 5>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
      case 6: return launch_mixed<T, 6>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
      case 7: return launch_mixed<T, 7>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
      case 8: return launch_mixed<T, 8>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
    }
    return fail(p, DPLR_LR_E_UNSUPPORTED, "order");
  }
  switch (p->cfg.order) {
    case 2: return launch_step<T, 2>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
    case 3: return launch_step<T, 3>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
    case 4: return launch_step<T, 4>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
    case 5: return launch_step<T, 5>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
    case 6: return launch_step<T, 6>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
    case 7: return launch_step<T, 7>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
    case 8: return launch_step<T, 8>(p, n_ion, a, b, n_wc, c, d, e, f, en, vir);
  }
  return fail(p, DPLR_LR_E_UNSUPPORTED, "order");
}

// The per-call buffers of the plane/pencil path (everything but the twiddle
// and influence tables), sized for `cap` particles, taken in a fixed order
// from get(&ptr, bytes, what): hipMalloc for plans, consecutive pieces of the
// static scratch array for the no-allocation entry point.
template <typename Get>
dplr_lr_status carve_workspace(dplr_lr_plan p, size_t cap, Get&& get) {
  const Geo& g = p->geo;
  const size_t ts = p->tsize, cs = 2 * ts;
  const size_t nspec = (size_t)g.Kh * g.K[1] * g.K[2];
  dplr_lr_status s2 = DPLR_LR_OK;
#define DPLR_ALLOC(ptr, bytes, what)                                  \
  if (s2 == DPLR_LR_OK) {                                             \
    void* tmp__ = nullptr;                                            \
    s2 = get(&tmp__, (bytes), what);                                  \
    ptr = reinterpret_cast<decltype(ptr)>(tmp__);                     \
  }
  DPLR_ALLOC(p->bin_count, sizeof(int) * (g.nbins + 1), "bin_count");
  DPLR_ALLOC(p->bin_start, sizeof(int) * (g.nbins + 1), "bin_start");
  DPLR_ALLOC(p->bin_cursor, sizeof(int) * (g.nbins + 1), "bin_cursor");
  p->block_hist = (size_t)g.nbins * sizeof(int) <= std::min<size_t>(p->lds_budget, 65536);
  if (p->block_hist) DPLR_ALLOC(p->bin_hist, sizeof(int) * (size_t)p->max_chunks * g.nbins, "bin histograms");
  DPLR_ALLOC(p->sorted, 4 * ts * cap, "sorted");
  DPLR_ALLOC(p->perm, sizeof(int) * cap, "perm");
  DPLR_ALLOC(p->sidx, sizeof(int) * cap, "stencil starts");
  DPLR_ALLOC(p->spec, cs * nspec * g.nsplit, "spectrum (one partial per particle split)");
  DPLR_ALLOC(p->qmax, sizeof(unsigned) * (size_t)std::max(p->max_chunks, 1), "charge maxima");
  DPLR_ALLOC(p->fspec, 3 * cs * nspec, "field spectra");
  // three interleaved field components, or (analytic differentiation) the
  // potential in rows padded by kGatherAdPad
  DPLR_ALLOC(p->field, ts * std::max<size_t>(3 * (size_t)g.K[0], (size_t)g.K[0] + kGatherAdPad) * g.K[1] * g.K[2],
             "fields");
  DPLR_ALLOC(p->partials, sizeof(double) * 8 * g.nzblk, "partials");
#undef DPLR_ALLOC
  return s2;
}

}  // namespace

extern "C" {

int32_t dplr_lr_abi_version(void) { return DPLR_LR_ABI_VERSION; }

void dplr_lr_config_default(dplr_lr_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->mesh[0] = cfg->mesh[1] = cfg->mesh[2] = 32;
  cfg->order = 5;
  cfg->beta = 0.4;
  cfg->coulomb_k = 14.399645;
  cfg->precision = DPLR_LR_FP32;
  cfg->alias_range = 2;
  cfg->capacity = 0;
  cfg->flags = 0;
}

dplr_lr_status dplr_lr_config_validate(const dplr_lr_config* cfg, char* msg, int64_t msg_len) {
  const char* m = "";
  dplr_lr_status st = validate(cfg, m);
  if (st != DPLR_LR_OK) set_global_error(m);
  if (msg && msg_len > 0) {
    std::snprintf(msg, (size_t)msg_len, "%s", m);
  }
  return st;
}

dplr_lr_status dplr_lr_plan_create(const dplr_lr_config* cfg, void* hip_stream, dplr_lr_plan* out) {
  if (!out) return fail(nullptr, DPLR_LR_E_INVALID, "out is NULL");
  *out = nullptr;
  const char* m = "";
  dplr_lr_status st = validate(cfg, m);
  if (st != DPLR_LR_OK) return fail(nullptr, st, m);

  dplr_lr_plan p = new (std::nothrow) dplr_lr_plan_s();
  if (!p) return fail(nullptr, DPLR_LR_E_NOMEM, "host allocation");
  p->cfg = *cfg;
  p->stream = (hipStream_t)hip_stream;
  p->fp64 = cfg->precision == DPLR_LR_FP64;
  p->tsize = p->fp64 ? sizeof(double) : sizeof(float);

  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; return hip_fail(nullptr, e, "hipGetDevice"); }
  int lds = 0;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
  if (e != hipSuccess) { delete p; return hip_fail(nullptr, e, "hipDeviceGetAttribute"); }
  p->lds_budget = (size_t)std::min(lds, 160 * 1024);
  if (!tuned_mesh(cfg->mesh)) {
    p->mixed = true;
    Geo& g = p->geo;
    for (int a = 0; a < 3; ++a) g.K[a] = cfg->mesh[a];
    g.Kh = g.K[0] / 2 + 1;
    const size_t ts = p->tsize, cs = 2 * ts;
    const size_t ntot = (size_t)g.K[0] * g.K[1] * g.K[2];
    const size_t ng = (size_t)g.Kh * (g.K[1] / 2 + 1) * (g.K[2] / 2 + 1);
    p->mblk = (int)((ntot + 255) / 256);
    dplr_lr_status sm = DPLR_LR_OK;
    void* tmp = nullptr;
    // particle ranges per plane of the split plane spread: enough blocks for 256 CUs, at most 8
    // (a power of two: the sort assigns particles to splits by index bits)
    p->msplit = 1;
    while (2 * p->msplit <= std::min(8, 256 / g.K[2])) p->msplit *= 2;
    // fused z pass: C (x, y) columns per block, a power of two dividing Kx Ky,
    // at most 16 and C Kz <= kFusedZMaxPts
    const size_t nxy = (size_t)g.K[0] * g.K[1];
    while (p->mzc < DPLR_MIXED_ZCOLS && nxy % (2 * p->mzc) == 0 && 2 * (size_t)p->mzc * g.K[2] <= (size_t)kFusedZMaxPts)
      p->mzc *= 2;
    p->mzblk = (int)(nxy / p->mzc);
    // the sort's bins: one per (split, stencil-start plane, group of
    // 2^qshift stencil-start rows); columns are not binned
    g.qshift = DPLR_MIXED_QSHIFT;
    g.NQ = (g.K[1] + (1 << g.qshift) - 1) >> g.qshift;
    g.split_by_index = 1;
    g.nsplit = p->msplit;
    g.xs = g.K[0];
    g.nbins = p->msplit * g.K[2] * g.NQ;
    if (sm == DPLR_LR_OK) {
      // integer partial meshes, or the split spectra of the fused spread
      sm = alloc(p, &tmp, std::max(sizeof(long long), cs) * ntot * p->msplit,
                 "mixed-radix mesh (or split partial meshes)");
      p->mmesh = (long long*)tmp;
    }
    if (sm == DPLR_LR_OK) { sm = alloc(p, &p->mspec, cs * ntot, "mixed-radix spectrum"); }
    if (sm == DPLR_LR_OK) { sm = alloc(p, &p->mfield, 3 * cs * ntot, "mixed-radix field spectra"); }
    if (sm == DPLR_LR_OK) { sm = alloc(p, &p->mpacked, 4 * ts * ntot, "mixed-radix fields"); }
    if (sm == DPLR_LR_OK) { sm = alloc(p, &tmp, sizeof(double) * ng, "influence"); p->G = (double*)tmp; }
    if (sm == DPLR_LR_OK) {
      sm = alloc(p, &tmp, sizeof(double) * 8 * std::max(p->mblk, p->mzblk), "partials");
      p->partials = (double*)tmp;
    }
    if (sm == DPLR_LR_OK) {
      sm = alloc(p, &tmp, sizeof(unsigned long long), "int32 saturation count");
      p->q32_clamped = (unsigned long long*)tmp;
    }
    if (sm == DPLR_LR_OK) {
      hipError_t e2 = hipMemset(p->mmesh, 0, sizeof(long long) * ntot);
      if (e2 == hipSuccess) e2 = hipMemset(p->G, 0, sizeof(double) * ng);
      if (e2 == hipSuccess) e2 = hipMemset(p->q32_clamped, 0, sizeof(unsigned long long));
      if (e2 != hipSuccess) sm = hip_fail(p, e2, "workspace init");
    }
    if (sm != DPLR_LR_OK) {
      set_global_error(p->err);
      free_all(p);
      delete p;
      return sm;
    }
    // plane spread when an xy plane of 64-bit accumulators fits in LDS
    const size_t lp = sizeof(unsigned long long) * (size_t)g.K[0] * g.K[1];
    if (lp + 10240 <= p->lds_budget) {
      const void* f = nullptr;
      switch (cfg->order) {
#define DPLR_PLANE(PP)                                                                                       \
  case PP:                                                                                                   \
    f = p->fp64 ? (const void*)k_mixed_spread_sorted<double, PP> : (const void*)k_mixed_spread_sorted<float, PP>; \
    break;
        DPLR_PLANE(2) DPLR_PLANE(3) DPLR_PLANE(4) DPLR_PLANE(5) DPLR_PLANE(6) DPLR_PLANE(7) DPLR_PLANE(8)
#undef DPLR_PLANE
      }
      p->lds_mplane = lp;
      if (lp > 65536 && !raise_lds_limit(f, lp)) p->lds_mplane = 0;
      // fused plane kernels when an xy plane of complex values (and its roots
      // of unity) fits in LDS
      const size_t lf = (nxy + g.K[0] + g.K[1]) * cs;
      const size_t lz = (size_t)(2 * p->mzc + 1) * g.K[2] * cs;
      const size_t fmax = p->fp64 ? FusedPlane<double>::kMaxPts : FusedPlane<float>::kMaxPts;
      if (DPLR_MIXED_FUSED && p->lds_mplane && nxy <= fmax && lf + 2048 <= p->lds_budget) {
        const void* fs = nullptr;
        switch (cfg->order) {
#define DPLR_FUSED(PP)                                                                                   \
  case PP:                                                                                               \
    fs = p->fp64 ? (const void*)k_mixed_spread_xy<double, PP> : (const void*)k_mixed_spread_xy<float, PP>; \
    break;
          DPLR_FUSED(2) DPLR_FUSED(3) DPLR_FUSED(4) DPLR_FUSED(5) DPLR_FUSED(6) DPLR_FUSED(7) DPLR_FUSED(8)
#undef DPLR_FUSED
        }
        const void* fi = p->fp64 ? (const void*)k_mixed_ifft_xy<double> : (const void*)k_mixed_ifft_xy<float>;
        const void* fzk = p->fp64 ? (const void*)k_mixed_fftz_poisson<double> : (const void*)k_mixed_fftz_poisson<float>;
        if (raise_lds_limit(fs, lf) && raise_lds_limit(fi, lf) && (lz <= 60000 || raise_lds_limit(fzk, lz)))
          p->mfused = lf;
      }
      const size_t capn = (size_t)std::max<int64_t>(cfg->capacity, 1);
      void* t2 = nullptr;
      dplr_lr_status sr = DPLR_LR_OK;
      if (p->lds_mplane) sr = alloc(p, &p->mrec, 4 * ts * capn, "mixed-radix stencil records");
      if (p->lds_mplane && sr == DPLR_LR_OK) { sr = alloc(p, &t2, sizeof(int) * capn, "mixed-radix stencil starts"); p->mspk = (int*)t2; }
      // the counting sort's buffers (bins of every split count up to msplit)
      const size_t nb1 = (size_t)p->geo.nbins + 1;
      if (p->lds_mplane && sr == DPLR_LR_OK) { sr = alloc(p, &t2, sizeof(int) * capn, "perm"); p->perm = (int*)t2; }
      if (p->lds_mplane && sr == DPLR_LR_OK) { sr = alloc(p, &t2, sizeof(int) * nb1, "bin_count"); p->bin_count = (int*)t2; }
      if (p->lds_mplane && sr == DPLR_LR_OK) { sr = alloc(p, &t2, sizeof(int) * nb1, "bin_start"); p->bin_start = (int*)t2; }
      if (p->lds_mplane && sr == DPLR_LR_OK) {
        sr = alloc(p, &t2, sizeof(int) * (size_t)p->max_chunks * p->geo.nbins, "bin histograms");
        p->bin_hist = (int*)t2;
      }
      if (p->lds_mplane && sr == DPLR_LR_OK) {
        sr = alloc(p, &t2, sizeof(unsigned) * (size_t)p->max_chunks, "charge maxima");
        p->qmax = (unsigned*)t2;
      }
      if (sr != DPLR_LR_OK) {
        set_global_error(p->err);
        free_all(p);
        delete p;
        return sr;
      }
    }
    *out = p;
    return DPLR_LR_OK;
  }
  if (!choose_geometry(p)) {
    delete p;
    return fail(nullptr, DPLR_LR_E_UNSUPPORTED, "no tiling fits the device's LDS for this mesh/order/precision");
  }
  const Geo& g = p->geo;
  const size_t ng = (size_t)g.Kh * (g.K[1] / 2 + 1) * (g.K[2] / 2 + 1);
  dplr_lr_status s2 = alloc(p, &p->twiddle, 2 * p->tsize * g.twN, "twiddles");
  if (s2 == DPLR_LR_OK) {
    void* t = nullptr;
    s2 = alloc(p, &t, sizeof(double) * ng, "influence");
    p->G = (double*)t;
  }
  if (s2 == DPLR_LR_OK)
    s2 = carve_workspace(p, (size_t)std::max<int64_t>(cfg->capacity, 1),
                         [p](void** ptr, size_t bytes, const char* what) { return alloc(p, ptr, bytes, what); });
  if (s2 != DPLR_LR_OK) {
    set_global_error(p->err);
    free_all(p);
    delete p;
    return s2;
  }
  std::vector<unsigned char> tw;
  if (p->fp64) fill_twiddles<double>(tw, g.twN); else fill_twiddles<float>(tw, g.twN);
  e = hipMemcpy(p->twiddle, tw.data(), tw.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p->bin_count, 0, sizeof(int) * (g.nbins + 1));
  if (e == hipSuccess) e = hipMemset(p->G, 0, sizeof(double) * ng);
  if (e != hipSuccess) {
    dplr_lr_status r = hip_fail(nullptr, e, "workspace init");
    free_all(p);
    delete p;
    return r;
  }
  if (p->fp64) set_lds_attrs<double>(p); else set_lds_attrs<float>(p);
  *out = p;
  return DPLR_LR_OK;
}

dplr_lr_status dplr_lr_set_fft_int32(dplr_lr_plan p, const int32_t nodes[3], double scale) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  if (!nodes) {
    for (int a = 0; a < 3; ++a) p->q32_nodes[a] = 0;
    p->q32_scale = 0.0;
    return DPLR_LR_OK;
  }
  if (!p->mixed) return fail(p, DPLR_LR_E_UNSUPPORTED, "int32 transforms are available on mixed-radix plans only");
  if (!(scale > 0.0) || !(scale <= 2147483648.0)) return fail(p, DPLR_LR_E_INVALID, "scale must be in (0, 2^31]");
  for (int a = 0; a < 3; ++a) {
    if (nodes[a] < 1 || p->geo.K[a] % nodes[a]) return fail(p, DPLR_LR_E_INVALID, "node counts must divide the mesh sizes");
    if (p->geo.K[a] > kMaxQ32Mesh) return fail(p, DPLR_LR_E_UNSUPPORTED, "int32 transforms take mesh sizes up to 256");
  }
  for (int a = 0; a < 3; ++a) p->q32_nodes[a] = nodes[a];
  p->q32_scale = scale;
  return DPLR_LR_OK;
}

dplr_lr_status dplr_lr_set_stream(dplr_lr_plan p, void* hip_stream) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  p->stream = (hipStream_t)hip_stream;
  return DPLR_LR_OK;
}

dplr_lr_status dplr_lr_set_box(dplr_lr_plan p, const double box_len[3]) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  if (!box_len) return fail(p, DPLR_LR_E_INVALID, "box_len is NULL");
  for (int a = 0; a < 3; ++a) {
    if (!(box_len[a] > 0.0) || !std::isfinite(box_len[a])) return fail(p, DPLR_LR_E_INVALID, "box lengths must be positive and finite");
  }
  for (int a = 0; a < 3; ++a) p->box[a] = box_len[a];
  const Geo& g = p->geo;
  const int64_t ng = (int64_t)g.Kh * (g.K[1] / 2 + 1) * (g.K[2] / 2 + 1);
  hipLaunchKernelGGL(k_influence, dim3((unsigned)((ng + 127) / 128)), dim3(128), 0, p->stream, p->G, g, p->box[0],
                     p->box[1], p->box[2], p->cfg.beta, p->cfg.order, p->cfg.alias_range);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(p, e, "influence launch");
  p->has_box = true;
  return DPLR_LR_OK;
}

dplr_lr_status dplr_lr_compute_energy_forces_virial(dplr_lr_plan p, int64_t n_ion, const void* ion_pos,
                                                    const void* ion_q, int64_t n_wc, const void* wc_pos,
                                                    const void* wc_q, void* ion_force, void* wc_force,
                                                    double* energy, double* virial6) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  if (n_ion < 0 || n_wc < 0) return fail(p, DPLR_LR_E_INVALID, "negative particle count");
  if (n_ion > 0 && (!ion_pos || !ion_q || !ion_force)) return fail(p, DPLR_LR_E_INVALID, "ion pointer is NULL");
  if (n_wc > 0 && (!wc_pos || !wc_q || !wc_force)) return fail(p, DPLR_LR_E_INVALID, "wc pointer is NULL");
  if (!energy) return fail(p, DPLR_LR_E_INVALID, "energy is NULL");
  if (!virial6 && !(p->cfg.flags & DPLR_LR_NO_VIRIAL)) return fail(p, DPLR_LR_E_INVALID, "virial6 is NULL");
  if (!p->has_box) return fail(p, DPLR_LR_E_NO_BOX, "set_box has not been called");
  if (n_ion + n_wc > p->cfg.capacity) return fail(p, DPLR_LR_E_CAPACITY, "n_ion + n_wc exceeds the plan capacity");
  if (p->fp64) return dispatch_order<double>(p, n_ion, ion_pos, ion_q, n_wc, wc_pos, wc_q, ion_force, wc_force, energy, virial6);
  return dispatch_order<float>(p, n_ion, ion_pos, ion_q, n_wc, wc_pos, wc_q, ion_force, wc_force, energy, virial6);
}

dplr_lr_status dplr_lr_scale_grad(dplr_lr_plan p, const double* grad_energy, int64_t n_ion, const void* ion_force,
                                  void* ion_grad, int64_t n_wc, const void* wc_force, void* wc_grad) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  if (!grad_energy) return fail(p, DPLR_LR_E_INVALID, "grad_energy is NULL");
  if (n_ion < 0 || n_wc < 0) return fail(p, DPLR_LR_E_INVALID, "negative particle count");
  if (n_ion > 0 && (!ion_force || !ion_grad)) return fail(p, DPLR_LR_E_INVALID, "ion pointer is NULL");
  if (n_wc > 0 && (!wc_force || !wc_grad)) return fail(p, DPLR_LR_E_INVALID, "wc pointer is NULL");
  const int64_t m[2] = {3 * n_ion, 3 * n_wc};
  const void* src[2] = {ion_force, wc_force};
  void* dst[2] = {ion_grad, wc_grad};
  for (int i = 0; i < 2; ++i) {
    if (m[i] == 0) continue;
    const unsigned nb = (unsigned)((m[i] + 255) / 256);
    if (p->fp64)
      hipLaunchKernelGGL(k_scale_grad<double>, dim3(nb), dim3(256), 0, p->stream, grad_energy, (const double*)src[i], (double*)dst[i], m[i]);
    else
      hipLaunchKernelGGL(k_scale_grad<float>, dim3(nb), dim3(256), 0, p->stream, grad_energy, (const float*)src[i], (float*)dst[i], m[i]);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(p, e, "scale_grad launch");
  return DPLR_LR_OK;
}

dplr_lr_status dplr_lr_plan_destroy(dplr_lr_plan p) {
  if (!p) return DPLR_LR_OK;
  (void)hipStreamSynchronize(p->stream);
  for (auto& r : p->prof_pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : p->prof_pool) (void)hipEventDestroy(e);
  free_all(p);
  delete p;
  return DPLR_LR_OK;
}

dplr_lr_status dplr_lr_profile_enable(dplr_lr_plan p, int32_t enable) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  p->prof = enable != 0;
  return DPLR_LR_OK;
}

dplr_lr_status dplr_lr_profile_read(dplr_lr_plan p, double* ms, int64_t* calls, int32_t max, int32_t* n,
                                    int32_t reset) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  if (max < 0 || (max > 0 && (!ms || !calls))) return fail(p, DPLR_LR_E_INVALID, "bad output arrays");
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "profile sync");
  for (auto& r : p->prof_pending) {
    float t = 0.f;
    e = hipEventElapsedTime(&t, r.a, r.b);
    if (e == hipSuccess) {
      p->prof_ms[r.stage] += t;
      p->prof_calls[r.stage] += 1;
    }
    p->prof_pool.push_back(r.a);
    p->prof_pool.push_back(r.b);
  }
  p->prof_pending.clear();
  for (int i = 0; i < kNumStages && i < max; ++i) {
    ms[i] = p->prof_ms[i];
    calls[i] = p->prof_calls[i];
  }
  if (n) *n = kNumStages;
  if (reset) {
    for (int i = 0; i < 16; ++i) { p->prof_ms[i] = 0; p->prof_calls[i] = 0; }
  }
  return DPLR_LR_OK;
}

const char* dplr_lr_profile_stage_name(int32_t i) {
  return (i >= 0 && i < kNumStages) ? kStageNames[i] : "";
}

const char* dplr_lr_last_error(dplr_lr_plan p) {
  return p ? p->err : g_global_error;
}

int64_t dplr_lr_workspace_bytes(dplr_lr_plan p) { return p ? p->ws_bytes : 0; }

int64_t dplr_lr_debug_size(dplr_lr_plan p, int32_t which) {
  if (!p) return -1;
  const Geo& g = p->geo;
  const size_t cs = 2 * p->tsize;
  const size_t nspec = (size_t)g.Kh * g.K[1] * g.K[2];
  if (which == DPLR_LR_BUF_Q32_CLAMPED) return p->mixed ? (int64_t)sizeof(unsigned long long) : -1;
  if (p->mixed && which != DPLR_LR_BUF_INFLUENCE) return -1;
  switch (which) {
    case DPLR_LR_BUF_SPECTRUM: return (int64_t)(cs * nspec);
    case DPLR_LR_BUF_INFLUENCE: return (int64_t)(sizeof(double) * g.Kh * (g.K[1] / 2 + 1) * (g.K[2] / 2 + 1));
    case DPLR_LR_BUF_FIELD_SPECTRA: return (int64_t)(3 * cs * nspec);
  }
  return -1;
}

dplr_lr_status dplr_lr_debug_copy(dplr_lr_plan p, int32_t which, void* dst, int64_t bytes) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  const int64_t size = dplr_lr_debug_size(p, which);
  if (size < 0) return fail(p, DPLR_LR_E_INVALID, "unknown buffer");
  if (!dst || bytes < 0 || bytes > size) return fail(p, DPLR_LR_E_INVALID, "bad destination or size");
  const void* src = which == DPLR_LR_BUF_SPECTRUM    ? p->spec
                    : which == DPLR_LR_BUF_INFLUENCE ? (const void*)p->G
                    : which == DPLR_LR_BUF_Q32_CLAMPED ? (const void*)p->q32_clamped
                                                      : p->fspec;
  if (which == DPLR_LR_BUF_SPECTRUM && p->plane && p->geo.nsplit > 1) {
    // the plane spread leaves one partial spectrum per particle split: report their sum
    const size_t cs = 2 * p->tsize;
    if ((size_t)bytes % cs) return fail(p, DPLR_LR_E_INVALID, "size must be a whole number of complex values");
    const size_t n = (size_t)bytes / cs, nspec = (size_t)size / cs;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (n > 0) {
      if (p->fp64)
        hipLaunchKernelGGL(k_sum_partials<double>, dim3(nb), dim3(256), 0, p->stream, (cpx<double>*)dst,
                           (const cpx<double>*)p->spec, p->geo.nsplit, nspec, n);
      else
        hipLaunchKernelGGL(k_sum_partials<float>, dim3(nb), dim3(256), 0, p->stream, (cpx<float>*)dst,
                           (const cpx<float>*)p->spec, p->geo.nsplit, nspec, n);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(p, e, "debug copy");
    return DPLR_LR_OK;
  }
  hipError_t e = hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "debug copy");
  return DPLR_LR_OK;
}

dplr_lr_status dplr_lr_debug_dft_q32(dplr_lr_plan p, int32_t axis, int32_t sign, void* data, int32_t ncomp) {
  if (!p) return fail(nullptr, DPLR_LR_E_INVALID, "plan is NULL");
  if (!p->mixed || p->q32_nodes[0] <= 0) return fail(p, DPLR_LR_E_UNSUPPORTED, "int32 transforms are not enabled on this plan");
  if (axis < 0 || axis > 2 || (sign != 1 && sign != -1) || ncomp < 1 || ncomp > 3 || !data)
    return fail(p, DPLR_LR_E_INVALID, "axis in 0..2, sign +-1, ncomp in 1..3, data not NULL");
  const int K[3] = {p->geo.K[0], p->geo.K[1], p->geo.K[2]};
  const int64_t ntot = (int64_t)K[0] * K[1] * K[2];
  const int64_t stride[3] = {1, K[0], (int64_t)K[0] * K[1]};
  const int64_t rows = ntot / K[axis];
  if (p->fp64)
    hipLaunchKernelGGL(k_mixed_dft_q32<double>, dim3((unsigned)rows, (unsigned)ncomp), dim3(64),
                       sizeof(cpx<double>) * K[axis], p->stream, (cpx<double>*)data, K[axis], stride[axis], ntot,
                       (int)sign, p->q32_nodes[axis], p->q32_scale, (double*)nullptr,
                       (unsigned long long*)nullptr);
  else
    hipLaunchKernelGGL(k_mixed_dft_q32<float>, dim3((unsigned)rows, (unsigned)ncomp), dim3(64),
                       sizeof(cpx<float>) * K[axis], p->stream, (cpx<float>*)data, K[axis], stride[axis], ntot,
                       (int)sign, p->q32_nodes[axis], p->q32_scale, (float*)nullptr, (unsigned long long*)nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(p, e, "int32 transform launch");
  return DPLR_LR_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Step without device allocation (dplr_lr_compute_noalloc).  Its working
// buffers live in one file-scope device array, `scratch`; each GPU the library
// runs on holds its own copy from module load to process exit.  Host code
// never passes the array's name to a kernel (in host code the name is a
// host-side stand-in, not a device address): set-up looks up each device's
// address of it once, with hipGetSymbolAddress, and every kernel argument,
// fill and copy uses that address.
//
// Layout of each device's copy: [FP32 twiddle tables for N = 16 .. 512]
// [FP64 twiddle tables] (written once, at set-up) [influence table of the
// last box] [the per-call buffers of carve_workspace].
// ----------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)DPLR_LR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kTwMin = kMinMesh, kTwMax = kMaxMesh;
constexpr size_t kTwEntries = 2 * kTwMax - kTwMin;  // 16 + 32 + ... + 512
// the table of size N (a power of two) starts at entry N - 16
size_t tw_entry(int N) { return (size_t)N - kTwMin; }
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t kTwF32Bytes = (kTwEntries * sizeof(cpx<float>) + 255) & ~(size_t)255;
constexpr size_t kTwF64Bytes = (kTwEntries * sizeof(cpx<double>) + 255) & ~(size_t)255;
constexpr size_t kScratchHead = kTwF32Bytes + kTwF64Bytes;

struct NoallocDevice {
  bool ready = false;
  unsigned char* ptr = nullptr;  // this device's address of `scratch`
  size_t lds_budget = 0;
  // what the influence table in scratch was computed for
  bool g_valid = false;
  int K[3] = {0, 0, 0};
  int order = 0, alias = 0;
  double beta = 0.0, box[3] = {0, 0, 0};
};
constexpr int kMaxDevices = 64;
NoallocDevice g_noalloc[kMaxDevices];
std::mutex g_noalloc_mu;

template <typename T>
void twiddle_tables(cpx<T>* w) {
  for (int N = kTwMin; N <= kTwMax; N *= 2) {
    cpx<T>* t = w + tw_entry(N);
    for (int k = 0; k < N; ++k) {  // the values fill_twiddles gives plans
      const double th = -2.0 * M_PI * (double)k / (double)N;
      t[k].x = (T)std::cos(th);
      t[k].y = (T)std::sin(th);
    }
  }
}

// Once per device, with that device current: the device address of scratch
// and the twiddle tables (synchronous copies from host stack memory).
dplr_lr_status noalloc_setup(int dev, NoallocDevice& d) {
  if (d.ready) return DPLR_LR_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_fail(nullptr, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  int lds = 0;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipDeviceGetAttribute");
  cpx<float> tf[kTwEntries];
  cpx<double> td[kTwEntries];
  twiddle_tables<float>(tf);
  twiddle_tables<double>(td);
  unsigned char* base = (unsigned char*)ptr;
  e = hipMemcpy(base, tf, sizeof(tf), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(base + kTwF32Bytes, td, sizeof(td), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(nullptr, e, "scratch set-up");
  d.ptr = base;
  d.lds_budget = (size_t)std::min(lds, 160 * 1024);
  d.ready = true;
  return DPLR_LR_OK;
}

}  // namespace

extern "C" {

dplr_lr_status dplr_lr_compute_noalloc(const dplr_lr_config* cfg, const double box_len[3], int64_t n_ion,
                                       const void* ion_pos, const void* ion_q, int64_t n_wc, const void* wc_pos,
                                       const void* wc_q, void* ion_force, void* wc_force, double* energy,
                                       double* virial6, void* hip_stream) {
  if (!cfg) return fail(nullptr, DPLR_LR_E_INVALID, "config is NULL");
  dplr_lr_config cf = *cfg;
  cf.capacity = 0;  // not used: the call's particle count sizes the buffers
  cfg = &cf;
  const char* m = "";
  dplr_lr_status st = validate(cfg, m);
  if (st != DPLR_LR_OK) return fail(nullptr, st, m);
  if (!tuned_mesh(cfg->mesh))
    return fail(nullptr, DPLR_LR_E_UNSUPPORTED, "the no-allocation step takes power-of-two meshes of 16 to 512 points");
  if (!box_len) return fail(nullptr, DPLR_LR_E_INVALID, "box_len is NULL");
  for (int a = 0; a < 3; ++a)
    if (!(box_len[a] > 0.0) || !std::isfinite(box_len[a]))
      return fail(nullptr, DPLR_LR_E_INVALID, "box lengths must be positive and finite");
  if (n_ion < 0 || n_wc < 0) return fail(nullptr, DPLR_LR_E_INVALID, "negative particle count");
  if (n_ion + n_wc > 0x7fffffffLL) return fail(nullptr, DPLR_LR_E_CAPACITY, "more than 2^31 - 1 particles");
  if (n_ion > 0 && (!ion_pos || !ion_q || !ion_force)) return fail(nullptr, DPLR_LR_E_INVALID, "ion pointer is NULL");
  if (n_wc > 0 && (!wc_pos || !wc_q || !wc_force)) return fail(nullptr, DPLR_LR_E_INVALID, "wc pointer is NULL");
  if (!energy) return fail(nullptr, DPLR_LR_E_INVALID, "energy is NULL");
  if (!virial6 && !(cfg->flags & DPLR_LR_NO_VIRIAL)) return fail(nullptr, DPLR_LR_E_INVALID, "virial6 is NULL");

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, DPLR_LR_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoallocDevice& d = g_noalloc[dev];
  if ((st = noalloc_setup(dev, d)) != DPLR_LR_OK) return st;

  // a plan on the host stack whose buffers are pieces of scratch
  dplr_lr_plan_s pl;
  dplr_lr_plan p = &pl;
  p->cfg = *cfg;
  p->cfg.capacity = n_ion + n_wc;
  p->stream = (hipStream_t)hip_stream;
  p->device = dev;
  p->fp64 = cfg->precision == DPLR_LR_FP64;
  p->tsize = p->fp64 ? sizeof(double) : sizeof(float);
  p->lds_budget = d.lds_budget;
  if (!choose_geometry(p))
    return fail(nullptr, DPLR_LR_E_UNSUPPORTED, "no tiling fits the device's LDS for this mesh/order/precision");
  const Geo& g = p->geo;
  const size_t ng = (size_t)g.Kh * (g.K[1] / 2 + 1) * (g.K[2] / 2 + 1);
  const size_t g_off = kScratchHead;
  size_t off = align256(g_off + sizeof(double) * ng);
  const size_t cap = (size_t)std::max<int64_t>(n_ion + n_wc, 1);
  // sizes first: reject before touching the device
  {
    size_t need = off;
    dplr_lr_plan_s dry;
    dry.cfg = p->cfg; dry.fp64 = p->fp64; dry.tsize = p->tsize; dry.lds_budget = p->lds_budget; dry.geo = p->geo;
    (void)carve_workspace(&dry, cap, [&need](void** ptr, size_t bytes, const char*) {
      *ptr = nullptr;
      need = align256(need + std::max<size_t>(bytes, 16));
      return DPLR_LR_OK;
    });
    if (need > kScratchBytes) {
      char msg[kErrLen];
      std::snprintf(msg, sizeof(msg),
                    "the no-allocation step needs %zu bytes of scratch for this mesh and %lld particles; "
                    "it has %zu (DPLR_LR_NOALLOC_SCRATCH_BYTES)",
                    need, (long long)(n_ion + n_wc), kScratchBytes);
      return fail(nullptr, DPLR_LR_E_CAPACITY, msg);
    }
  }
  p->twiddle = d.ptr + (p->fp64 ? kTwF32Bytes + sizeof(cpx<double>) * tw_entry(g.twN)
                                : sizeof(cpx<float>) * tw_entry(g.twN));
  p->G = reinterpret_cast<double*>(d.ptr + g_off);
  (void)carve_workspace(p, cap, [&](void** ptr, size_t bytes, const char*) {
    *ptr = d.ptr + off;
    off = align256(off + std::max<size_t>(bytes, 16));
    return DPLR_LR_OK;
  });
  // kernels with more than 64 KiB of dynamic LDS (limits are only ever raised)
  if (p->fp64) set_lds_attrs<double>(p); else set_lds_attrs<float>(p);
  // the influence table is kept from the last call on this device when the
  // mesh, order, alias range, beta and box are the same
  const bool same_g = d.g_valid && d.K[0] == g.K[0] && d.K[1] == g.K[1] && d.K[2] == g.K[2] &&
                      d.order == cfg->order && d.alias == cfg->alias_range && d.beta == cfg->beta &&
                      d.box[0] == box_len[0] && d.box[1] == box_len[1] && d.box[2] == box_len[2];
  for (int a = 0; a < 3; ++a) p->box[a] = box_len[a];
  p->has_box = true;
  if (!same_g) {
    d.g_valid = false;
    hipLaunchKernelGGL(k_influence, dim3((unsigned)((ng + 127) / 128)), dim3(128), 0, p->stream, p->G, g, p->box[0],
                       p->box[1], p->box[2], cfg->beta, cfg->order, cfg->alias_range);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(nullptr, e, "influence launch");
    d.g_valid = true;
    for (int a = 0; a < 3; ++a) { d.K[a] = g.K[a]; d.box[a] = box_len[a]; }
    d.order = cfg->order;
    d.alias = cfg->alias_range;
    d.beta = cfg->beta;
  }
  // the global-atomic sort counts into bin_count, which must start at zero
  // (scratch keeps the previous call's contents); a fill kernel, not a memset
  if (!p->block_hist) {
    hipLaunchKernelGGL(k_fill_int, dim3((g.nbins + 1 + 255) / 256), dim3(256), 0, p->stream, p->bin_count,
                       g.nbins + 1, 0);
  }
  st = p->fp64 ? dispatch_order<double>(p, n_ion, ion_pos, ion_q, n_wc, wc_pos, wc_q, ion_force, wc_force, energy,
                                        virial6)
               : dispatch_order<float>(p, n_ion, ion_pos, ion_q, n_wc, wc_pos, wc_q, ion_force, wc_force, energy,
                                       virial6);
  if (st != DPLR_LR_OK) set_global_error(p->err);
  return st;
}

}  // extern "C"

#include "learned_api.inc"
