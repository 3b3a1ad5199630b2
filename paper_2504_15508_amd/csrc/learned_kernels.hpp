// Learned coarse-mesh correction: neighbour descriptor, a 128-64-64-64-32
// SiLU MLP on BF16 MFMA with FP32 accumulation, the equivariant force head,
// and training (loss, backward, Adam) - all as gfx950 kernels.
//
//   T_i[k, a] = sum_{j: r_ij < rc} q_j T_k(2 r_ij / rc - 1) s(r_ij) u_a(i -> j),
//               u = (1, unit vector), s(r) = (1 + cos(pi r / rc)) / 2, k < 32;
//   D_i[4k + l] = sum_a T_i[k, a] T_i[l, a] (l < 4);  x_i = (D_i - mu) * inv_sigma;
//   h1 = silu(x W1 + b1), h2 = silu(h1 W2 + b2), h3 = silu(h2 W3 + b3),
//   c = h3 W4 + b4;  dF_i = s_out q_i sum_k c_ik T_i[k, 1:4].
//
// Packed parameter vector (FP32 master copy, the layout of the C ABI):
//   W1[128][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64][32] b4[32]
//   mu[128] inv_sigma[128]                                   (18912 floats)
#pragma once

#include "pppm_kernels.hpp"

namespace dplr {
namespace mlp {

constexpr int kIn = 128, kH = 64, kOut = 32;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kIn * kH;
constexpr int kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH * kH;
constexpr int kOffW4 = kOffB3 + kH, kOffB4 = kOffW4 + kH * kOut;
constexpr int kNTrain = kOffB4 + kOut;                // trainable parameters
constexpr int kOffMu = kNTrain, kOffIsd = kOffMu + kIn;
constexpr int kNParams = kOffIsd + kIn;               // packed total
constexpr int kNWeights = kIn * kH + 2 * kH * kH + kH * kOut;  // bf16 weight copy
constexpr int kRows = 128;                            // particles per MLP block (4 waves x 32)
constexpr int kMlpThreads = 256;                      // threads of the MLP forward and backward blocks

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// silu with the hardware reciprocal (1 ulp): the result is rounded to bf16
// before it is used, so the last FP32 bits do not matter
__device__ __forceinline__ float silu(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// row / column of accumulator register r of this lane in the 32 x 32 tile
__device__ __forceinline__ int acc_row(int r) { return 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3); }
__device__ __forceinline__ int acc_col() { return threadIdx.x & 31; }

__device__ __forceinline__ void zero(f32x16& a) {
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = 0.0f;
}

// ---------------------------------------------------------------------------
// Cell list: cells of edge >= rc per axis (at least 3 per axis).
// ---------------------------------------------------------------------------
struct CellGeo {
  int nc[3];
  float L[3], invL[3], cinv[3];  // box, 1/box, cells per Angstrom
  float rc;
  int ncells;
};

__device__ __forceinline__ float wrapf(float v, float L, float invL) {
  v -= L * floorf(v * invL);
  if (v >= L) v -= L;
  if (!(v >= 0.0f && v < L)) v = 0.0f;
  return v;
}

__device__ __forceinline__ int cell_of(float x, float y, float z, const CellGeo& c) {
  int cx = min((int)(x * c.cinv[0]), c.nc[0] - 1);
  int cy = min((int)(y * c.cinv[1]), c.nc[1] - 1);
  int cz = min((int)(z * c.cinv[2]), c.nc[2] - 1);
  return (cz * c.nc[1] + cy) * c.nc[0] + cx;
}

__global__ void k_cell_count(const float* __restrict__ ion_pos, const float* __restrict__ wc_pos, int64_t n_ion,
                             int64_t n, int* __restrict__ count, CellGeo c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* r = (i < n_ion) ? ion_pos + 3 * i : wc_pos + 3 * (i - n_ion);
  const float x = wrapf(r[0], c.L[0], c.invL[0]), y = wrapf(r[1], c.L[1], c.invL[1]),
              z = wrapf(r[2], c.L[2], c.invL[2]);
  atomicAdd(count + cell_of(x, y, z, c), 1);
}

__global__ void k_cell_scatter(const float* __restrict__ ion_pos, const float* __restrict__ wc_pos,
                               const float* __restrict__ ion_q, const float* __restrict__ wc_q, int64_t n_ion,
                               int64_t n, int* __restrict__ cursor, float4* __restrict__ cpos,
                               int* __restrict__ cidx, CellGeo c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* r = (i < n_ion) ? ion_pos + 3 * i : wc_pos + 3 * (i - n_ion);
  const float x = wrapf(r[0], c.L[0], c.invL[0]), y = wrapf(r[1], c.L[1], c.invL[1]),
              z = wrapf(r[2], c.L[2], c.invL[2]);
  const float q = (i < n_ion) ? ion_q[i] : wc_q[i - n_ion];
  const int slot = atomicAdd(cursor + cell_of(x, y, z, c), 1);
  cpos[slot] = make_float4(x, y, z, q);
  cidx[slot] = (int)i;
}

// The atomic scatter leaves each cell's particles in arrival order; this puts
// them in order of original index (rank = number of the cell's particles
// with a smaller index), so the cell order and every sum over neighbours
// taken in it are the same on every call.  One thread per particle; a cell
// holds tens of particles, so the O(n^2) ranking per cell is cheap.
__global__ void k_cell_order(const float4* __restrict__ cpos_in, const int* __restrict__ cidx_in,
                             const int* __restrict__ start, int n,
                             float4* __restrict__ cpos, int* __restrict__ cidx, CellGeo c) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float4 p = cpos_in[e];
  const int id = cidx_in[e];
  const int cell = cell_of(p.x, p.y, p.z, c);
  const int j0 = start[cell], j1 = start[cell + 1];
  int rank = 0;
  for (int j = j0; j < j1; ++j) rank += cidx_in[j] < id;
  cpos[j0 + rank] = p;
  cidx[j0 + rank] = id;
}

// Runtime statistics of the learned form's inputs and outputs, read by the
// fallback guard (dplr_lr_mlp_read_stats).  Maxima of non-negative floats are
// kept as their bit patterns (whose unsigned order is the float order), so
// every field is an integer reduction or a fixed-order FP64 sum: the values do
// not depend on the order of the contributions.
struct Stats {
  unsigned max_corr_bits;   // max |dF_i| of the last forward
  unsigned max_force_bits;  // max |F_i| of the forces the last forward added to
  int min_nbr, max_nbr;     // neighbour counts within the cutoff, last forward
  int unseen;               // charges outside the training set, last check
  int audit_valid;
  double audit_num, audit_den;  // sum |F - F_ref|^2, sum |F_ref|^2 of the audits
};

__device__ __forceinline__ unsigned wave_max_bits(unsigned v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, off, 64));
  return v;
}

__global__ void k_stats_reset_forward(Stats* st) {
  if (threadIdx.x == 0) {
    st->max_corr_bits = 0u;
    st->max_force_bits = 0u;
    st->min_nbr = 0x7fffffff;
    st->max_nbr = 0;
  }
}

// Smallest and largest neighbour count: per-block partials, then one block
// reduces them (integer min / max: independent of the order).
__global__ void __launch_bounds__(256) k_nbr_partials(const int* __restrict__ nbr, int n, int* __restrict__ part) {
  __shared__ int lo[256], hi[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  lo[threadIdx.x] = i < n ? nbr[i] : 0x7fffffff;
  hi[threadIdx.x] = i < n ? nbr[i] : 0;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + h]);
      hi[threadIdx.x] = max(hi[threadIdx.x], hi[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = lo[0];
    part[2 * blockIdx.x + 1] = hi[0];
  }
}

__global__ void __launch_bounds__(256) k_nbr_range(const int* __restrict__ part, int nblk, Stats* __restrict__ st) {
  __shared__ int lo[256], hi[256];
  int a = 0x7fffffff, b = 0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    a = min(a, part[2 * k]);
    b = max(b, part[2 * k + 1]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + h]);
      hi[threadIdx.x] = max(hi[threadIdx.x], hi[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->min_nbr = lo[0];
    st->max_nbr = hi[0];
  }
}

// Charges not in the training set (exact float comparison with the set).
constexpr int kMaxTrainCharges = 16;
struct ChargeSet {
  int n;
  float q[kMaxTrainCharges];
};

__global__ void k_check_charges(const float* __restrict__ ion_q, const float* __restrict__ wc_q, int64_t n_ion,
                                int64_t n, ChargeSet cs, Stats* st, int reset) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (reset) {  // single-block launch for an empty input
    if (i == 0) st->unseen = 0;
    return;
  }
  int bad = 0;
  if (i < n) {
    const float q = (i < n_ion) ? ion_q[i] : wc_q[i - n_ion];
    bool seen = false;
    for (int k = 0; k < cs.n; ++k) seen |= (q == cs.q[k]);
    bad = seen ? 0 : 1;
  }
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(&st->unseen, bad);
}

// Audit sums over both particle sets: per-block FP64 partials (fixed order
// inside the block), then one block adds them in block order.
__global__ void __launch_bounds__(256) k_audit_partials(const float* __restrict__ fi, const float* __restrict__ ri,
                                                        int64_t n_ion, const float* __restrict__ fw,
                                                        const float* __restrict__ rw, int64_t n,
                                                        double* __restrict__ part) {
  __shared__ double red[2][256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (i < n) {
    const float* f = (i < n_ion) ? fi + 3 * i : fw + 3 * (i - n_ion);
    const float* r = (i < n_ion) ? ri + 3 * i : rw + 3 * (i - n_ion);
    for (int a = 0; a < 3; ++a) {
      const double d = (double)f[a] - (double)r[a];
      num += d * d;
      den += (double)r[a] * (double)r[a];
    }
  }
  red[0][threadIdx.x] = num;
  red[1][threadIdx.x] = den;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_audit_finish(const double* __restrict__ part, int nblk, Stats* st, int accumulate) {
  if (threadIdx.x != 0) return;
  double num = 0.0, den = 0.0;
  for (int b = 0; b < nblk; ++b) {
    num += part[2 * b];
    den += part[2 * b + 1];
  }
  st->audit_num = accumulate ? st->audit_num + num : num;
  st->audit_den = accumulate ? st->audit_den + den : den;
  st->audit_valid = 1;
}

// Input normalisation from training descriptors: per-block partial sums of
// D_f and D_f^2 and the block maximum of |D| (f < 128), from T [n][128];
// then the block partials are added in block order into acc[2][128] (+ count
// and max), and finish turns them into mu = mean, inv_sigma =
// 1 / (std + 1e-6 (max |D| + 1)) in the parameter vector.
__global__ void __launch_bounds__(128) k_norm_partials(const float* __restrict__ T, int n, int rows_per_block,
                                                       double* __restrict__ part) {
  const int f = threadIdx.x;  // feature 4k + l
  const int k = f >> 2, l = f & 3;
  const int r0 = blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
  double s1 = 0.0, s2 = 0.0;
  float mx = 0.0f;
  for (int r = r0; r < r1; ++r) {
    const float4 tk = reinterpret_cast<const float4*>(T + (size_t)r * 128)[k];
    const float4 tl = reinterpret_cast<const float4*>(T + (size_t)r * 128)[l];
    const float d = tk.x * tl.x + tk.y * tl.y + tk.z * tl.z + tk.w * tl.w;
    s1 += d;
    s2 += (double)d * d;
    mx = fmaxf(mx, fabsf(d));
  }
  double* p = part + (size_t)blockIdx.x * 3 * 128;
  p[f] = s1;
  p[128 + f] = s2;
  p[256 + f] = mx;
}

__global__ void __launch_bounds__(128) k_norm_reduce(const double* __restrict__ part, int nblk, int rows,
                                                     double* __restrict__ acc) {
  // acc: [0,128) sum, [128,256) sum of squares, [256] max |D|, [257] count
  const int f = threadIdx.x;
  double s1 = 0.0, s2 = 0.0, mx = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double* p = part + (size_t)b * 3 * 128;
    s1 += p[f];
    s2 += p[128 + f];
    mx = fmax(mx, p[256 + f]);
  }
  acc[f] += s1;
  acc[128 + f] += s2;
  __shared__ double m[128];
  m[f] = mx;
  __syncthreads();
  if (f == 0) {
    double g = acc[256];
    for (int i = 0; i < 128; ++i) g = fmax(g, m[i]);
    acc[256] = g;
    acc[257] += (double)rows;
  }
}

__global__ void __launch_bounds__(128) k_norm_finish(double* __restrict__ acc, float* __restrict__ params) {
  const int f = threadIdx.x;
  const double cnt = acc[257];
  if (cnt > 0.0) {
    const double mu = acc[f] / cnt;
    const double var = fmax(acc[128 + f] / cnt - mu * mu, 0.0);
    params[kOffMu + f] = (float)mu;
    params[kOffIsd + f] = (float)(1.0 / (sqrt(var) + 1e-6 * (acc[256] + 1.0)));
  }
  __syncthreads();
  acc[f] = 0.0;
  acc[128 + f] = 0.0;
  if (f == 0) {
    acc[256] = 0.0;
    acc[257] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Descriptor: four lanes per (cell-sorted) particle.  Lane g owns the radial
// orders k = g, g+4, ..., g+28, advanced with the stride-4 Chebyshev
// recurrence T_{k+4} = 2 T_4 T_k - T_{k-4}, so a lane holds 8 x 4
// accumulators instead of 32 x 4 (high occupancy hides the memory latency of
// the neighbour scan).  Two phases: the four lanes scan the 27 neighbour cells
// together (candidate jb + g), and the ones inside the cutoff are appended to
// the particle's LDS list in candidate order (ballot + prefix count, so the
// order is deterministic); then every lane accumulates its orders over the
// whole list, the pair quantities formed once per pair (accumulate_pairs).  Writes T [n][128] (FP32, index 4k + a) and the normalised MLP
// input x [n][128] (bf16).
// ---------------------------------------------------------------------------
constexpr int kDescLanes = 4;
constexpr int kDescThreads = 256;
constexpr int kDescParts = kDescThreads / kDescLanes;
constexpr int kNbrMax = 64;

// Pairs per round of the accumulation: the four lanes of a particle form the
// round's pair quantities (weight, unit vector, Chebyshev argument) once, one
// pair each in turn, through the particle's LDS slots, and then every lane
// runs its eight orders over all of them.
constexpr int kPairChunk = 8;  // 4 measured the same, 16 slower (LDS per block)

__device__ __forceinline__ void accumulate_pairs(float (&T)[8][4], const float4 pi, const float4* __restrict__ cpos,
                                                 const int* list, int cnt, int g, const CellGeo& c,
                                                 float (*pq)[5]) {
  const float inv_rc = 1.0f / c.rc;
  for (int t0 = 0; t0 < cnt; t0 += kPairChunk) {
    const int nc = min(kPairChunk, cnt - t0);
    for (int t = g; t < nc; t += kDescLanes) {
      const float4 pj = cpos[list[t0 + t]];
      float d0 = pj.x - pi.x, d1 = pj.y - pi.y, d2 = pj.z - pi.z;
      d0 -= c.L[0] * rintf(d0 * c.invL[0]);
      d1 -= c.L[1] * rintf(d1 * c.invL[1]);
      d2 -= c.L[2] * rintf(d2 * c.invL[2]);
      const float r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const float r = sqrtf(r2), ir = 1.0f / r;
      const float sw = 0.5f * (1.0f + __cosf(3.14159265358979f * r * inv_rc));
      pq[t][0] = pj.w * sw;
      pq[t][1] = d0 * ir;
      pq[t][2] = d1 * ir;
      pq[t][3] = d2 * ir;
      pq[t][4] = 2.0f * r * inv_rc - 1.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the round's slots written
    for (int t = 0; t < nc; ++t) {
      const float w = pq[t][0], u1 = pq[t][1], u2 = pq[t][2], u3 = pq[t][3], x = pq[t][4];
      const float t2 = 2.0f * x * x - 1.0f, t3 = 2.0f * x * t2 - x, t4 = 2.0f * x * t3 - t2;
      // lane g starts from T_g and T_{4-g}
      float cur = (g == 0) ? 1.0f : (g == 1) ? x : (g == 2) ? t2 : t3;
      float prev = (g == 0) ? t4 : (g == 1) ? t3 : (g == 2) ? t2 : x;
      const float t4x2 = 2.0f * t4;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        if (m > 0) {
          const float nxt = t4x2 * cur - prev;
          prev = cur;
          cur = nxt;
        }
        const float wg = w * cur;
        T[m][0] += wg;
        T[m][1] += wg * u1;
        T[m][2] += wg * u2;
        T[m][3] += wg * u3;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // all four lanes done before the next round
  }
}

__global__ void __launch_bounds__(kDescThreads) k_descriptor(const float4* __restrict__ cpos,
                                                             const int* __restrict__ start, int n,
                                                             const float* __restrict__ params,
                                                             float* __restrict__ Tout,
                                                             unsigned short* __restrict__ X, CellGeo c,
                                                             int* __restrict__ nbr) {
  __shared__ int lists[kDescParts][kNbrMax];
  __shared__ float pqs[kDescParts][kPairChunk][5];
  const int g = threadIdx.x & (kDescLanes - 1), p = threadIdx.x / kDescLanes;
  const int lane = threadIdx.x & 63, gbase = lane & ~(kDescLanes - 1);
  const int i = blockIdx.x * kDescParts + p;
  if (i >= n) return;  // the four lanes of a particle leave together
  int* list = lists[p];
  const float4 pi = cpos[i];
  float T[8][4];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
#pragma unroll
    for (int a = 0; a < 4; ++a) T[m][a] = 0.0f;
  }
  const int cx = min((int)(pi.x * c.cinv[0]), c.nc[0] - 1);
  const int cy = min((int)(pi.y * c.cinv[1]), c.nc[1] - 1);
  const int cz = min((int)(pi.z * c.cinv[2]), c.nc[2] - 1);
  const float rc2 = c.rc * c.rc;
  int cnt = 0, total = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = (cz + dz + c.nc[2]) % c.nc[2];
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = (cy + dy + c.nc[1]) % c.nc[1];
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = (cx + dx + c.nc[0]) % c.nc[0];
        const int cell = (zz * c.nc[1] + yy) * c.nc[0] + xx;
        const int j0 = start[cell], j1 = start[cell + 1];
        for (int jb = j0; jb < j1; jb += kDescLanes) {
          const int j = jb + g;
          bool in = false;
          if (j < j1 && j != i) {
            const float4 pj = cpos[j];
            float d0 = pj.x - pi.x, d1 = pj.y - pi.y, d2 = pj.z - pi.z;
            d0 -= c.L[0] * rintf(d0 * c.invL[0]);
            d1 -= c.L[1] * rintf(d1 * c.invL[1]);
            d2 -= c.L[2] * rintf(d2 * c.invL[2]);
            const float r2 = d0 * d0 + d1 * d1 + d2 * d2;
            in = r2 < rc2 && r2 > 0.0f;
          }
          const unsigned gm = (unsigned)(__ballot(in) >> gbase) & ((1u << kDescLanes) - 1u);
          if (in) list[cnt + __popc(gm & ((1u << g) - 1u))] = j;
          cnt += __popc(gm);
          total += __popc(gm);
          if (cnt > kNbrMax - kDescLanes) {  // the same decision on all four lanes
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            accumulate_pairs(T, pi, cpos, list, cnt, g, c, pqs[p]);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            cnt = 0;
          }
        }
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  accumulate_pairs(T, pi, cpos, list, cnt, g, c, pqs[p]);
  if (nbr && g == 0) nbr[i] = total;  // neighbour count, reduced by k_nbr_range
  float* to = Tout + (size_t)i * 128;
#pragma unroll
  for (int m = 0; m < 8; ++m)
    reinterpret_cast<float4*>(to)[g + 4 * m] = make_float4(T[m][0], T[m][1], T[m][2], T[m][3]);
  // invariants D[4k + l] = sum_a T[k][a] T[l][a], l < 4: T[l] is order 0 of lane l
  float Tl[4][4];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
#pragma unroll
    for (int a = 0; a < 4; ++a) Tl[l][a] = __shfl(T[0][a], gbase + l, 64);
  }
  const float* mu = params + kOffMu;
  const float* isd = params + kOffIsd;
  unsigned short* xo = X + (size_t)i * 128;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int k = g + 4 * m;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const float d = T[m][0] * Tl[l][0] + T[m][1] * Tl[l][1] + T[m][2] * Tl[l][2] + T[m][3] * Tl[l][3];
      const int f = 4 * k + l;
      xo[f] = f2bf((d - mu[f]) * isd[f]);
    }
  }
}

// ---------------------------------------------------------------------------
// LDS operand layout for the MFMA tiles: every matrix is stored with the
// contraction index k contiguous and rows padded by 4 bf16 (8 bytes), so a
// lane's eight k values are two 64-bit LDS reads and the 32 rows a half-wave
// reads fall on distinct banks (row pitch / 8 bytes is odd).
// ---------------------------------------------------------------------------
constexpr int kPadIn = kIn + 4;     // 132: rows of 128 bf16
constexpr int kPadH = kH + 4;       // 68: rows of 64 bf16
constexpr int kPadO = kOut + 4;     // 36: rows of 32 bf16
constexpr int kPadRows = kRows + 4; // 132: transposed tiles (rows = features, k = particles)

// acc (32 x 32) += A (32 x K) * B (K x 32) with both operands k-contiguous:
// A(m, k) = A[m * lda + k], B(k, n) = B[n * ldb + k].  One gfx950
// v_mfma_f32_32x32x16_bf16 per 16 values of k: lane l supplies
// A(l % 32, 8 (l / 32) + i) and B(8 (l / 32) + i, l % 32), i < 8, read as two
// 8-byte LDS loads (rows are 8-byte aligned); K is a multiple of 16.
__device__ __forceinline__ void mfma_tile_kc(f32x16& acc, const unsigned short* A, int lda,
                                             const unsigned short* B, int ldb, int K) {
  const int l = threadIdx.x & 63;
  const int mn = l & 31, kh = (l >> 5) * 8;
  const unsigned short* pa = A + mn * lda + kh;
  const unsigned short* pb = B + mn * ldb + kh;
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x4 a0 = *reinterpret_cast<const bf16x4*>(pa + k0);
    const bf16x4 a1 = *reinterpret_cast<const bf16x4*>(pa + k0 + 4);
    const bf16x4 b0 = *reinterpret_cast<const bf16x4*>(pb + k0);
    const bf16x4 b1 = *reinterpret_cast<const bf16x4*>(pb + k0 + 4);
    const bf16x8 a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
    const bf16x8 b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
}

// The same for two B tiles sharing A: acc0 += A B0, acc1 += A B1.
__device__ __forceinline__ void mfma_tile_kc2(f32x16& acc0, f32x16& acc1, const unsigned short* A, int lda,
                                              const unsigned short* B0, const unsigned short* B1, int ldb, int K) {
  const int l = threadIdx.x & 63;
  const int mn = l & 31, kh = (l >> 5) * 8;
  const unsigned short* pa = A + mn * lda + kh;
  const unsigned short* p0 = B0 + mn * ldb + kh;
  const unsigned short* p1 = B1 + mn * ldb + kh;
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x4 a0 = *reinterpret_cast<const bf16x4*>(pa + k0);
    const bf16x4 a1 = *reinterpret_cast<const bf16x4*>(pa + k0 + 4);
    const bf16x4 b00 = *reinterpret_cast<const bf16x4*>(p0 + k0);
    const bf16x4 b01 = *reinterpret_cast<const bf16x4*>(p0 + k0 + 4);
    const bf16x4 b10 = *reinterpret_cast<const bf16x4*>(p1 + k0);
    const bf16x4 b11 = *reinterpret_cast<const bf16x4*>(p1 + k0 + 4);
    const bf16x8 a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
    const bf16x8 b0 = __builtin_shufflevector(b00, b01, 0, 1, 2, 3, 4, 5, 6, 7);
    const bf16x8 b1 = __builtin_shufflevector(b10, b11, 0, 1, 2, 3, 4, 5, 6, 7);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
  }
}

// weight offsets in the padded LDS copies
constexpr int kLW1t = 0, kLW2t = kLW1t + kH * kPadIn, kLW3t = kLW2t + kH * kPadH,
              kLW4t = kLW3t + kH * kPadH, kLWt = kLW4t + kOut * kPadH;  // [out][in] copies
constexpr int kLW1 = 0, kLW2 = kLW1 + kIn * kPadH, kLW3 = kLW2 + kH * kPadH, kLW4 = kLW3 + kH * kPadH,
              kLW = kLW4 + kH * kPadO;                                   // [in][out] copies

// ---------------------------------------------------------------------------
// MLP forward + force head.  Persistent blocks of 4 waves stage the weights
// (bf16, [out][in]) and biases once, then walk tiles of 128 particles; wave w
// owns rows 32w..32w+31 of a tile.  Activations go layer to layer through
// LDS.  In training mode the pre-activations z1..z3 and activations h1..h3
// are stored, and the head also forms the loss and dL/dc.
// ---------------------------------------------------------------------------
struct FwdLds {
  unsigned short wt[kLWt];
  float b[kH * 3 + kOut];
  unsigned short x[kRows][kPadIn];
  unsigned short h[2][kRows][kPadH];
  float c[kRows][kOut + 1];
  double lred[4];
};

template <bool TRAIN>
__global__ void __launch_bounds__(256) k_mlp_fwd(const unsigned short* __restrict__ X, const float* __restrict__ Tin,
                                                 const float4* __restrict__ cpos, const int* __restrict__ cidx,
                                                 int n, int64_t n_ion, const unsigned short* __restrict__ wt_g,
                                                 const float* __restrict__ params, float s_out,
                                                 float* __restrict__ ion_dF, float* __restrict__ wc_dF,
                                                 int accumulate,
                                                 // training
                                                 const float* __restrict__ ion_tgt, const float* __restrict__ wc_tgt,
                                                 const float* __restrict__ ion_base, const float* __restrict__ wc_base,
                                                 float* __restrict__ Z, unsigned short* __restrict__ H,
                                                 float* __restrict__ dC, double* __restrict__ loss_part, float gscale,
                                                 Stats* __restrict__ st) {
  extern __shared__ __align__(16) unsigned char smem[];
  FwdLds& S = *reinterpret_cast<FwdLds*>(smem);
  const int tid = threadIdx.x, wave = tid >> 6;
  // weights: global [out][in] (dense) -> LDS rows padded, in 16-byte chunks
  // of 8 values whose loads are all in flight before the first LDS store (a
  // loop with a run-time trip count would wait for each load in turn)
  {
    const int cols[4] = {kIn, kH, kH, kH};
    const int gofs[4] = {0, kIn * kH, kIn * kH + kH * kH, kIn * kH + 2 * kH * kH};
    const int lofs[4] = {kLW1t, kLW2t, kLW3t, kLW4t}, pitch[4] = {kPadIn, kPadH, kPadH, kPadH};
    constexpr int kChunks = kNWeights / 8, kPer = (kChunks + kMlpThreads - 1) / kMlpThreads;
    uint4 wv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int c = tid + u * kMlpThreads;
      if (c < kChunks) wv[u] = reinterpret_cast<const uint4*>(wt_g)[c];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int c = tid + u * kMlpThreads;
      if (c < kChunks) {
        const int e = 8 * c;
        const int L = e < gofs[1] ? 0 : e < gofs[2] ? 1 : e < gofs[3] ? 2 : 3;
        const int el = e - gofs[L], r = el / cols[L], col = el - r * cols[L];
        uint2* dst = reinterpret_cast<uint2*>(S.wt + lofs[L] + r * pitch[L] + col);  // 8-byte aligned
        dst[0] = make_uint2(wv[u].x, wv[u].y);
        dst[1] = make_uint2(wv[u].z, wv[u].w);
      }
    }
  }
  for (int e = tid; e < kH; e += blockDim.x) {
    S.b[e] = params[kOffB1 + e];
    S.b[kH + e] = params[kOffB2 + e];
    S.b[2 * kH + e] = params[kOffB3 + e];
  }
  for (int e = tid; e < kOut; e += blockDim.x) S.b[3 * kH + e] = params[kOffB4 + e];

  const int wr = wave * 32;  // this wave's first row in the tile
  const unsigned short* wl[4] = {S.wt + kLW1t, S.wt + kLW2t, S.wt + kLW3t, S.wt + kLW4t};
  const int ldw[4] = {kPadIn, kPadH, kPadH, kPadH};
  double lsum = 0.0;
  unsigned mcorr = 0u, mforce = 0u;  // running maxima (float bits) for the guard
  const int ntiles = (n + kRows - 1) / kRows;
  // A tile's inputs travel in 16-byte chunks held in registers: the next
  // tile's loads are issued while the current tile computes (the block's
  // barriers wait on LDS only, so the loads stay in flight across them).
  constexpr int kXc = kRows * kIn / 8, kXper = kXc / kMlpThreads;
  uint4 xv[kXper];
  auto load_x = [&](int tile) {
#pragma unroll
    for (int u = 0; u < kXper; ++u) {
      const int c = tid + u * kMlpThreads, r = c / (kIn / 8), c8 = c % (kIn / 8);
      const int row = tile * kRows + r;
      xv[u] = make_uint4(0u, 0u, 0u, 0u);
      if (tile < ntiles && row < n) xv[u] = reinterpret_cast<const uint4*>(X + (size_t)row * kIn)[c8];
    }
  };
  load_x(blockIdx.x);
  // head: two threads per particle (hp = particle in the tile, hk = which
  // half of the 32 radial orders); the particle's descriptor rows are loaded
  // at the start of the tile, so that they arrive during the layers
  const int hp = tid >> 1, hk = tid & 1;
  constexpr int kHalf = kOut / 2;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int row0 = tile * kRows;
    const bool hon = row0 + hp < n;
    float4 tq[kHalf];
    if (hon) {
      const float4* Tp = reinterpret_cast<const float4*>(Tin + (size_t)(row0 + hp) * 128) + hk * kHalf;
#pragma unroll
      for (int k = 0; k < kHalf; ++k) tq[k] = Tp[k];
    }
    __syncthreads();  // previous tile done with S.x / S.c; weights staged
#pragma unroll
    for (int u = 0; u < kXper; ++u) {
      const int c = tid + u * kMlpThreads, r = c / (kIn / 8), c8 = c % (kIn / 8);
      uint2* dst = reinterpret_cast<uint2*>(&S.x[r][8 * c8]);  // 8-byte aligned rows
      dst[0] = make_uint2(xv[u].x, xv[u].y);
      dst[1] = make_uint2(xv[u].z, xv[u].w);
    }
    __syncthreads();
    load_x(tile + gridDim.x);
    // hidden layers
#pragma unroll
    for (int layer = 0; layer < 3; ++layer) {
      const int K = layer == 0 ? kIn : kH;
      const unsigned short* A = layer == 0 ? &S.x[wr][0] : &S.h[(layer - 1) & 1][wr][0];
      const int lda = layer == 0 ? kPadIn : kPadH;
      unsigned short* Hout = &S.h[layer & 1][wr][0];
      // both 32-column tiles of the layer in one pass over k (two independent
      // accumulation chains in flight)
      static_assert(kH == 64, "two 32-column tiles per hidden layer");
      f32x16 acc2[2];
      zero(acc2[0]);
      zero(acc2[1]);
      mfma_tile_kc2(acc2[0], acc2[1], A, lda, wl[layer], wl[layer] + 32 * ldw[layer], ldw[layer], K);
#pragma unroll
      for (int nt = 0; nt < kH / 32; ++nt) {
        const f32x16& acc = acc2[nt];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = acc_row(r), col = nt * 32 + acc_col();
          const float z = acc[r] + S.b[layer * kH + col];
          const float h = silu(z);
          const unsigned short hb = f2bf(h);
          Hout[row * kPadH + col] = hb;
          if (TRAIN && row0 + wr + row < n) {
            Z[((size_t)layer * n + row0 + wr + row) * kH + col] = z;
            H[((size_t)layer * n + row0 + wr + row) * kH + col] = hb;
          }
        }
      }
      __syncthreads();
    }
    // output layer: c = h3 W4 + b4
    {
      f32x16 acc;
      zero(acc);
      mfma_tile_kc(acc, &S.h[0][wr][0], kPadH, wl[3], ldw[3], kH);
#pragma unroll
      for (int r = 0; r < 16; ++r) S.c[wr + acc_row(r)][acc_col()] = acc[r] + S.b[3 * kH + acc_col()];
    }
    __syncthreads();

    // head: dF = s_out q sum_k c_k T[k, 1:4], each thread over its half of k
    // (in order), the halves added in the order (0, 1)
    {
      float f0 = 0.f, f1 = 0.f, f2 = 0.f;
      if (hon) {
#pragma unroll
        for (int k = 0; k < kHalf; ++k) {
          const float cc = S.c[hp][hk * kHalf + k];
          f0 += cc * tq[k].y;
          f1 += cc * tq[k].z;
          f2 += cc * tq[k].w;
        }
      }
      const float o0 = __shfl_xor(f0, 1, 64), o1 = __shfl_xor(f1, 1, 64), o2 = __shfl_xor(f2, 1, 64);
      // both threads of the pair form the same sums: half 0 first
      f0 = hk == 0 ? f0 + o0 : o0 + f0;
      f1 = hk == 0 ? f1 + o1 : o1 + f1;
      f2 = hk == 0 ? f2 + o2 : o2 + f2;
      if (hon) {
        const int slot = row0 + hp;
        const float q = cpos[slot].w;
        const float sq = s_out * q;
        f0 *= sq; f1 *= sq; f2 *= sq;
        const int src = cidx[slot];
        float* out = (src < n_ion) ? ion_dF + 3 * (int64_t)src : wc_dF + 3 * ((int64_t)src - n_ion);
        if (hk == 0) {
          mcorr = max(mcorr, __float_as_uint(sqrtf(f0 * f0 + f1 * f1 + f2 * f2)));
          if (accumulate) {
            mforce = max(mforce, __float_as_uint(sqrtf(out[0] * out[0] + out[1] * out[1] + out[2] * out[2])));
            out[0] += f0; out[1] += f1; out[2] += f2;
          } else {
            out[0] = f0; out[1] = f1; out[2] = f2;
          }
        }
        if (TRAIN) {
          // target: the residual target - base (fine minus coarse forces) when a base is given
          const int64_t o3 = (src < n_ion) ? 3 * (int64_t)src : 3 * ((int64_t)src - n_ion);
          const float* tg = ((src < n_ion) ? ion_tgt : wc_tgt) + o3;
          const float* bs = (src < n_ion) ? ion_base : wc_base;
          float t0 = tg[0], t1 = tg[1], t2 = tg[2];
          if (bs) { t0 -= bs[o3]; t1 -= bs[o3 + 1]; t2 -= bs[o3 + 2]; }
          const float e0 = f0 - t0, e1 = f1 - t1, e2 = f2 - t2;
          if (hk == 0) lsum += (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
          // dL/d dF = gscale * e (gscale = 2 / (3 n)); dL/dc_k = s_out q (g . T[k, 1:4])
          const float g0 = gscale * e0 * sq, g1 = gscale * e1 * sq, g2 = gscale * e2 * sq;
#pragma unroll
          for (int k = 0; k < kHalf; ++k)
            dC[(size_t)slot * kOut + hk * kHalf + k] = g0 * tq[k].y + g1 * tq[k].z + g2 * tq[k].w;
        }
      }
    }
  }
  if (st) {
    mcorr = wave_max_bits(mcorr);
    mforce = wave_max_bits(mforce);
    if ((tid & 63) == 0) {
      if (mcorr) atomicMax(&st->max_corr_bits, mcorr);
      if (mforce) atomicMax(&st->max_force_bits, mforce);
    }
  }
  if (TRAIN) {
    // deterministic block sum of the squared errors (the even threads hold them)
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
    __syncthreads();
    if ((tid & 63) == 0) S.lred[wave] = lsum;
    __syncthreads();
    if (tid == 0) loss_part[blockIdx.x] = S.lred[0] + S.lred[1] + S.lred[2] + S.lred[3];
  }
}

// ---------------------------------------------------------------------------
// MLP backward for one block of 128 particles: per-block partial gradients of
// every weight and bias, written to gpart[block][kNTrain] (summed later in a
// fixed order).  Weights are staged in LDS in their natural [in][out] layout
// (the k of dh = dz W^T is the output index); the layer input and dz are
// also kept transposed (features x particles) for dW = act^T dz, whose k is
// the particle index.  dz / dz^T are double-buffered across layers.
// ---------------------------------------------------------------------------
struct BwdLds {
  unsigned short w[kLW];                  // W1 [128][68], W2 [64][68], W3 [64][68], W4 [64][36]
  unsigned short actT[kIn][kPadRows];     // layer input, transposed
  unsigned short dz[2][kRows][kPadH];     // gradient at the layer output (bf16)
  unsigned short dzT[2][kH][kPadRows];    // the same, transposed
};

__global__ void __launch_bounds__(256) k_mlp_bwd(const unsigned short* __restrict__ X, const float* __restrict__ Z,
                                                 const unsigned short* __restrict__ H, const float* __restrict__ dC,
                                                 int n, const unsigned short* __restrict__ w_g,
                                                 float* __restrict__ gpart) {
  extern __shared__ __align__(16) unsigned char smem[];
  BwdLds& S = *reinterpret_cast<BwdLds*>(smem);
  const int row0 = blockIdx.x * kRows;
  const int tid = threadIdx.x, wave = tid >> 6;
  float* gp = gpart + (size_t)blockIdx.x * kNTrain;
  {
    const int rows[4] = {kIn, kH, kH, kH}, cols[4] = {kH, kH, kH, kOut};
    const int gofs[4] = {0, kIn * kH, kIn * kH + kH * kH, kIn * kH + 2 * kH * kH};
    const int lofs[4] = {kLW1, kLW2, kLW3, kLW4}, pitch[4] = {kPadH, kPadH, kPadH, kPadO};
#pragma unroll
    for (int L = 0; L < 4; ++L)
      for (int e = tid; e < rows[L] * cols[L]; e += blockDim.x) {
        const int r = e / cols[L], c = e - r * cols[L];
        S.w[lofs[L] + r * pitch[L] + c] = w_g[gofs[L] + e];
      }
  }
  // dz <- dC (bf16, zero for rows past n), both layouts
  for (int e = tid; e < kRows * kOut; e += blockDim.x) {
    const int r = e / kOut, k = e % kOut;
    const unsigned short v = (row0 + r < n) ? f2bf(dC[(size_t)(row0 + r) * kOut + k]) : (unsigned short)0;
    S.dz[0][r][k] = v;
    S.dzT[0][k][r] = v;
  }
  const int offW[4] = {kLW1, kLW2, kLW3, kLW4};
  const int pitW[4] = {kPadH, kPadH, kPadH, kPadO};
  const int offGW[4] = {kOffW1, kOffW2, kOffW3, kOffW4};
  const int offGB[4] = {kOffB1, kOffB2, kOffB3, kOffB4};
  const int nin[4] = {kIn, kH, kH, kH};
  const int nout[4] = {kH, kH, kH, kOut};
  int cur = 0;
  for (int layer = 3; layer >= 0; --layer) {
    const int ni = nin[layer], no = nout[layer];
    // layer input activation (x for layer 0, h_layer otherwise), transposed
    for (int e = tid; e < kRows * ni; e += blockDim.x) {
      const int k = e / kRows, r = e - k * kRows;
      unsigned short v = 0;
      if (row0 + r < n) v = layer == 0 ? X[(size_t)(row0 + r) * kIn + k] : H[((size_t)(layer - 1) * n + row0 + r) * kH + k];
      S.actT[k][r] = v;
    }
    __syncthreads();
    // weight gradient tiles: dW (ni x no) = act^T (ni x rows) * dz (rows x no)
    const int tm = ni / 32, tn = no / 32;
    for (int t = wave; t < tm * tn; t += 4) {
      const int mi = t / tn, nj = t % tn;
      f32x16 acc;
      zero(acc);
      mfma_tile_kc(acc, &S.actT[mi * 32][0], kPadRows, &S.dzT[cur][nj * 32][0], kPadRows, kRows);
#pragma unroll
      for (int r = 0; r < 16; ++r)
        gp[offGW[layer] + (mi * 32 + acc_row(r)) * no + nj * 32 + acc_col()] = acc[r];
    }
    // bias gradient: sums of dz over particles (fixed order)
    for (int col = tid; col < no; col += blockDim.x) {
      float s = 0.0f;
      for (int r = 0; r < kRows; ++r) s += bf2f(S.dzT[cur][col][r]);
      gp[offGB[layer] + col] = s;
    }
    if (layer == 0) break;
    // gradient to the layer below: dh (rows x ni) = dz (rows x no) * W^T, then * silu'(z)
    const int nxt = cur ^ 1;
    for (int t = wave; t < (kRows / 32) * (ni / 32); t += 4) {
      const int ri = t / (ni / 32), mj = t % (ni / 32);
      f32x16 acc;
      zero(acc);
      // A(m, k) = dz[r0 + m][k], B(k, n) = W[m0 + n][k]  (W stored [in][out])
      mfma_tile_kc(acc, &S.dz[cur][ri * 32][0], kPadH, S.w + offW[layer] + mj * 32 * pitW[layer], pitW[layer], no);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = ri * 32 + acc_row(r), col = mj * 32 + acc_col();
        float v = 0.0f;
        if (row0 + row < n) v = acc[r] * dsilu(Z[((size_t)(layer - 1) * n + row0 + row) * kH + col]);
        const unsigned short b = f2bf(v);
        S.dz[nxt][row][col] = b;
        S.dzT[nxt][col][row] = b;
      }
    }
    __syncthreads();
    cur = nxt;
  }
}

// Sum of the per-block gradient partials in block order (deterministic) and
// of the loss partials; gscale_loss converts the squared-error sum to the mean.
__global__ void k_grad_reduce(const float* __restrict__ gpart, int nblk, float* __restrict__ grad,
                              const double* __restrict__ loss_part, int nloss, double loss_scale,
                              double* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNTrain) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += gpart[(size_t)b * kNTrain + p];
    grad[p] = s;
  }
  if (p == 0 && loss) {
    double s = 0.0;
    for (int b = 0; b < nloss; ++b) s += loss_part[b];
    *loss = s * loss_scale;
  }
}

// Adam on the FP32 master parameters, then bf16 copies of the weights in
// both layouts ([in][out] for backward, [out][in] for forward).
__global__ void k_adam(float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNTrain) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_weights_to_bf16(const float* __restrict__ params, unsigned short* __restrict__ w,
                                  unsigned short* __restrict__ wt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNWeights) return;
  // locate layer
  int off = 0, pofs = 0, ni = kIn, no = kH;
  if (e < kIn * kH) { off = 0; pofs = kOffW1; ni = kIn; no = kH; }
  else if (e < kIn * kH + kH * kH) { off = kIn * kH; pofs = kOffW2; ni = kH; no = kH; }
  else if (e < kIn * kH + 2 * kH * kH) { off = kIn * kH + kH * kH; pofs = kOffW3; ni = kH; no = kH; }
  else { off = kIn * kH + 2 * kH * kH; pofs = kOffW4; ni = kH; no = kOut; }
  const int loc = e - off;
  const int i = loc / no, o = loc % no;
  const unsigned short b = f2bf(params[pofs + loc]);
  w[e] = b;                      // [in][out]
  wt[off + o * ni + i] = b;      // [out][in]
}

}  // namespace mlp
}  // namespace dplr
