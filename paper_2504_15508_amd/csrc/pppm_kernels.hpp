// PPPM-ik kernels for gfx950.
//
// Data layout in HBM (FP32 plan; FP64 doubles every element):
//   sorted   [n] T4 (d_x, d_y, d_z, q): fractional B-spline offsets and charge,
//            ordered by bin; sidx [n] int: stencil starts s_x | s_y<<10 | s_z<<20;
//            perm [n] int: original index (ions 0..n_ion-1, then WCs).
//   bins     one per (split, stencil-start plane s_z, stencil-start row group
//            s_y >> qshift), in that order of significance; bin_start
//            [nbins+1].  The split is s_x / xs for pencil tiles and the
//            original index mod nsplit for planes.
//   spec     half spectrum [Kx/2+1][Kz][Ky] complex (y fastest); the spread
//            writes one such partial spectrum per particle split; the pass
//            after it adds them in split order.
//   fspec    three field spectra [3][Kx/2+1][Kz][Ky] complex.
//   G        FP64 influence table [Kx/2+1][Ky/2+1][Kz/2+1] (G is even in
//            every wave-vector component).
#pragma once

#include "device_common.hpp"

namespace dplr {

template <typename T>
struct alignas(4 * sizeof(T)) T4 {
  T x, y, z, w;
};

// Mesh/tiling geometry shared by all kernels of a plan (passed by value).
struct Geo {
  int K[3];      // Kx, Ky, Kz
  int Kh;        // Kx/2 + 1
  int qshift;    // rows per bin group = 2^qshift (4 for pencil tiles, 16 for planes)
  int NQ;        // Ky >> qshift
  int nsplit;    // particle splits of the spread (one partial spectrum each)
  int xs;        // Kx / nsplit: split = s_x / xs (pencil tiles) ...
  int split_by_index;  // ... or split = original index mod nsplit (planes)
  int nbins;     // nsplit * Kz * NQ
  int scy, scz;  // spread pencil cross-section (y, z); the pencil spans all x
  int spy, spz;  // spread pencil counts
  int zb;        // rows per block of the y-transform pass
  int yb;        // columns per block of the z-transform pass
  int twN;       // twiddle table length (max K)
  int nzblk;     // z-pass blocks
  int xyb;       // y rows per block of the inverse x pass
  int zgroup;    // z-pass column blocks per 128-byte output line (run on one XCD)
};

struct PoissonConsts {
  double two_pi_over_L[3];
  double inv_4beta2;
};

constexpr int kEPT = 16;  // FFT elements per thread bound
constexpr int kFftyThreads = 256;  // launch bound of the y pass

// Copies n contiguous elements from global memory to LDS with U loads in
// flight per thread before any of them is stored (a loop whose trip count
// the compiler cannot see would otherwise wait for each load in turn).
template <int U, typename V>
__device__ __forceinline__ void copy_g2s(V* __restrict__ dst, const V* __restrict__ src, int n) {
  for (int base = threadIdx.x; base < n; base += U * blockDim.x) {
    V r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * blockDim.x;
      if (e < n) r[u] = src[e];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * blockDim.x;
      if (e < n) dst[e] = r[u];
    }
  }
}

__device__ __forceinline__ int wrapi(int v, int K) {
  v %= K;
  return v < 0 ? v + K : v;
}

// ----------------------------------------------------------------------------
// Wrap + bin: counting sort by stencil-start plane and row quad
// ----------------------------------------------------------------------------
// The mesh coordinate u = r K / L, its wrap into [0, K), the stencil start s
// and the fractional offset d are computed in FP64 for both precisions: an
// FP32 u near K = 128 would carry a rounding of ~1e-5 cells, which water's
// tightly bound charges turn into ~1e-5 relative force error.  The FP32 path
// then stores d in [0, 1] (absolute rounding ~6e-8) next to the integer s.
template <typename T, int P>
__device__ __forceinline__ void particle_bin(const T* __restrict__ ion_pos, const T* __restrict__ wc_pos,
                                             int64_t n_ion, int64_t i, const double invh[3], const Geo& g,
                                             T d_out[3], int& spack, int& bin) {
  const T* r = (i < n_ion) ? (ion_pos + 3 * i) : (wc_pos + 3 * (i - n_ion));
  int s[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double K = (double)g.K[a];
    double v = (double)r[a] * invh[a];
    v = v - K * floor(v / K);
    if (v >= K) v -= K;
    if (!(v >= 0.0 && v < K)) v = 0.0;  // also maps NaN/Inf inputs to 0
    const double av = v - 0.5 * P;
    const double f = floor(av);
    d_out[a] = (T)(av - f);
    int sa = (int)f + 1;
    if (sa < 0) sa += g.K[a];
    if (sa >= g.K[a]) sa -= g.K[a];
    s[a] = sa;
  }
  spack = s[0] | (s[1] << 10) | (s[2] << 20);
  const int split = g.split_by_index ? (int)(i & (g.nsplit - 1)) : s[0] / g.xs;
  bin = (split * g.K[2] + s[2]) * g.NQ + (s[1] >> g.qshift);
}

// |q| as an unsigned integer whose order is that of the float (non-negative
// floats compare as their bit patterns); the wave maximum is formed with
// shuffles so that one lane per wave touches memory.
template <typename T>
__device__ __forceinline__ unsigned abs_q_bits(T q) {
  return __float_as_uint(fabsf((float)q));
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, off, 64));
  return v;
}

template <typename T, int P>
__global__ void __launch_bounds__(256) k_bin_count(const T* __restrict__ ion_pos, const T* __restrict__ wc_pos,
                                                   int64_t n_ion, int64_t n, double ihx, double ihy, double ihz,
                                                   int* __restrict__ count, Geo g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double invh[3] = {ihx, ihy, ihz};
  T d[3];
  int sp, bin;
  particle_bin<T, P>(ion_pos, wc_pos, n_ion, i, invh, g, d, sp, bin);
  atomicAdd(count + bin, 1);
}

// Exclusive scan of the bin counts (one block); also clears the counts for
// the next call and seeds the scatter cursors.
__global__ void __launch_bounds__(1024) k_bin_scan(int* __restrict__ count, int* __restrict__ start,
                                                   int* __restrict__ cursor, int nbins,
                                                   unsigned* __restrict__ qmax_bits = nullptr) {
  // tiles of 4 bins per thread, loaded and stored coalesced; the running
  // offset is carried from tile to tile
  __shared__ int part[1024];
  __shared__ int vals[4096];
  __shared__ int carry;
  if (qmax_bits && threadIdx.x == 0) *qmax_bits = 0u;
  const int t = threadIdx.x, nt = blockDim.x, tile = 4 * nt;
  if (t == 0) carry = 0;
  for (int b0 = 0; b0 < nbins; b0 += tile) {
    int c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * nt + t;  // coalesced
      c[u] = b < nbins ? count[b] : 0;
    }
    __syncthreads();  // carry of the previous tile is final; vals is free
    // this thread's 4 bins are b0 + 4t .. b0 + 4t + 3: exchange through LDS
#pragma unroll
    for (int u = 0; u < 4; ++u) vals[u * nt + t] = c[u];
    __syncthreads();
    int v4[4], s = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) { v4[u] = vals[4 * t + u]; s += v4[u]; }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
      const int x = (t >= off) ? part[t - off] : 0;
      __syncthreads();
      part[t] += x;
      __syncthreads();
    }
    int run = carry + part[t] - s;
#pragma unroll
    for (int u = 0; u < 4; ++u) { vals[4 * t + u] = run; run += v4[u]; }
    __syncthreads();
    const int tot = part[nt - 1];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * nt + t;
      if (b < nbins) {
        start[b] = vals[u * nt + t];
        cursor[b] = vals[u * nt + t];
        count[b] = 0;
      }
    }
    __syncthreads();
    if (t == 0) carry += tot;
  }
  __syncthreads();
  if (t == 0) start[nbins] = carry;
}

template <typename T, int P>
__global__ void __launch_bounds__(256) k_bin_scatter(const T* __restrict__ ion_pos, const T* __restrict__ wc_pos,
                                                     const T* __restrict__ ion_q, const T* __restrict__ wc_q,
                                                     int64_t n_ion, int64_t n, double ihx, double ihy, double ihz,
                                                     int* __restrict__ cursor, T4<T>* __restrict__ sorted,
                                                     int* __restrict__ sidx, int* __restrict__ perm,
                                                     unsigned* __restrict__ qmax_bits, Geo g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned qb = 0u;
  if (i < n) {
    const double invh[3] = {ihx, ihy, ihz};
    T d[3];
    int sp, bin;
    particle_bin<T, P>(ion_pos, wc_pos, n_ion, i, invh, g, d, sp, bin);
    const T q = (i < n_ion) ? ion_q[i] : wc_q[i - n_ion];
    const int slot = atomicAdd(cursor + bin, 1);
    sorted[slot] = T4<T>{d[0], d[1], d[2], q};
    sidx[slot] = sp;
    perm[slot] = (int)i;
    qb = abs_q_bits(q);
  }
  qb = wave_max_u32(qb);
  if ((threadIdx.x & 63) == 0) atomicMax(qmax_bits, qb);
}

// Counting sort without global atomics (used when the bins fit in LDS).
// Particles are cut into chunks of `chunk` consecutive indices; chunk c's
// histogram is built with LDS atomics and stored densely in hist[c][bin];
// a per-bin scan over chunks turns it into the chunk's offset inside the bin,
// a scan over bins (inside the placement kernel) gives bin_start, and the
// scatter places particle i of chunk c at
// bin_start[bin] + hist[c][bin] + (its rank within the chunk).
template <typename T, int P>
__global__ void __launch_bounds__(1024) k_bin_hist(const T* __restrict__ ion_pos, const T* __restrict__ wc_pos,
                                                   int64_t n_ion, int64_t n, double ihx, double ihy, double ihz,
                                                   int* __restrict__ hist, int chunk, Geo g) {
  extern __shared__ int lh[];
  for (int b = threadIdx.x; b < g.nbins; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const double invh[3] = {ihx, ihy, ihz};
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    T d[3];
    int sp, bin;
    particle_bin<T, P>(ion_pos, wc_pos, n_ion, i, invh, g, d, sp, bin);
    atomicAdd(lh + bin, 1);
  }
  __syncthreads();
  int* out = hist + (size_t)blockIdx.x * g.nbins;
  for (int b = threadIdx.x; b < g.nbins; b += blockDim.x) out[b] = lh[b];
}

__global__ void k_fill_int(int* __restrict__ a, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Per bin: exclusive scan of the chunk counts (in place) and the bin total.
// A block of 1024 threads handles 64 bins; its 16 groups of 64 lanes split
// the chunks into 16 consecutive ranges whose sums are combined in LDS.
__global__ void __launch_bounds__(1024) k_bin_colscan(int* __restrict__ hist, int* __restrict__ total, int nblk,
                                                      int nbins) {
  __shared__ int gsum[16][64];
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int b = blockIdx.x * 64 + lane;
  const int per = (nblk + 15) / 16;
  const int k0 = min(nblk, grp * per), k1 = min(nblk, k0 + per);
  int s = 0;
  int c[16];
  const int cnt = k1 - k0;  // at most 16 chunks per group (at most 256 chunks)
#pragma unroll
  for (int u = 0; u < 16; ++u) c[u] = (b < nbins && u < cnt) ? hist[(size_t)(k0 + u) * nbins + b] : 0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s += c[u];
  gsum[grp][lane] = s;
  __syncthreads();
  int run = 0;
  for (int g2 = 0; g2 < grp; ++g2) run += gsum[g2][lane];
  if (b < nbins) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (u < cnt) {
        hist[(size_t)(k0 + u) * nbins + b] = run;
        run += c[u];
      }
    }
    if (grp == 15) total[b] = run;
  }
}

// Exclusive scan of v[0, n) (global) into out[0, n) (LDS) by the whole block,
// one contiguous stretch of bins per thread; returns the total.  wsum: 17
// ints of LDS.
__device__ __forceinline__ int block_exclusive_scan(const int* __restrict__ v, int* out, int n, int* wsum) {
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, w = t >> 6, nw = nt >> 6;
  const int per = (n + nt - 1) / nt;
  const int b0 = min(n, t * per), b1 = min(n, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += v[b];
  int x = s;  // inclusive scan within the wave
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (w == 0) {
    const int ws = lane < nw ? wsum[lane] : 0;
    int xs = ws;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(xs, off, 64);
      if (lane >= off) xs += y;
    }
    if (lane < nw) wsum[lane] = xs - ws;
    if (lane == nw - 1) wsum[16] = xs;
  }
  __syncthreads();
  int run = wsum[w] + x - s;
  for (int b = b0; b < b1; ++b) {
    out[b] = run;
    run += v[b];
  }
  return wsum[16];
}

// Placement.  Every block first turns the bin totals into bin starts (an
// exclusive scan in LDS; block 0 also publishes them as bin_start), then
// scatters its chunk.
template <typename T, int P>
__global__ void __launch_bounds__(1024) k_bin_place(const T* __restrict__ ion_pos, const T* __restrict__ wc_pos,
                                                    const T* __restrict__ ion_q, const T* __restrict__ wc_q,
                                                    int64_t n_ion, int64_t n, double ihx, double ihy, double ihz,
                                                    const int* __restrict__ hist, const int* __restrict__ total,
                                                    int* __restrict__ bin_start,
                                                    T4<T>* __restrict__ sorted, int* __restrict__ sidx,
                                                    int* __restrict__ perm, unsigned* __restrict__ qmax_part,
                                                    int chunk, Geo g) {
  extern __shared__ int lc[];  // [nbins] ranks, then [nbins] bin starts
  int* start = lc + g.nbins;
  __shared__ unsigned qm;
  __shared__ int wsum[17];
  for (int b = threadIdx.x; b < g.nbins; b += blockDim.x) lc[b] = 0;
  if (threadIdx.x == 0) qm = 0u;
  const int all = block_exclusive_scan(total, start, g.nbins, wsum);  // contains barriers
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int b = threadIdx.x; b < g.nbins; b += blockDim.x) bin_start[b] = start[b];
    if (threadIdx.x == 0) bin_start[g.nbins] = all;
  }
  unsigned qb = 0u;
  const double invh[3] = {ihx, ihy, ihz};
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  const int* off = hist + (size_t)blockIdx.x * g.nbins;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    T d[3];
    int sp, bin;
    particle_bin<T, P>(ion_pos, wc_pos, n_ion, i, invh, g, d, sp, bin);
    const T q = (i < n_ion) ? ion_q[i] : wc_q[i - n_ion];
    const int slot = start[bin] + off[bin] + atomicAdd(lc + bin, 1);
    sorted[slot] = T4<T>{d[0], d[1], d[2], q};
    sidx[slot] = sp;
    perm[slot] = (int)i;
    qb = max(qb, abs_q_bits(q));
  }
  qb = wave_max_u32(qb);
  if ((threadIdx.x & 63) == 0) atomicMax(&qm, qb);
  __syncthreads();
  if (threadIdx.x == 0) qmax_part[blockIdx.x] = qm;
}

// ----------------------------------------------------------------------------
// Visit ranges of a pencil: the sorted particles whose stencil-start plane lies
// in [z_lo, z_lo + nplanes) (mod Kz) and whose stencil-start row quad lies in
// [q_lo, q_lo + nq) (mod NQ), as at most 2 contiguous ranges per plane.
// ----------------------------------------------------------------------------
struct Ranges {
  int n;
  int lo[48];
  int pre[49];  // prefix sums of lengths
  int b[48][2]; // scratch: bin bounds, then particle bounds, per candidate range
};

// Candidate ranges (up to two per plane) are resolved one per thread, so the
// block waits for one round of bin_start loads instead of a chain of them.
// range_load issues the loads (no barrier); ranges_finish stores them, then
// thread 0 lists the non-empty ranges, merging ranges that continue each
// other in the sorted order (consecutive planes usually do).
struct RangeLoad {
  int ncand, b0, b1;
};

__device__ __forceinline__ RangeLoad range_load(const int* __restrict__ bin_start, const Geo& g, int xsplit,
                                                int z_lo, int nplanes, int q_lo, int nq) {
  const int t = threadIdx.x;
  const int qa = wrapi(q_lo, g.NQ);
  const bool split = qa + nq > g.NQ;
  RangeLoad L{nplanes * (split ? 2 : 1), 0, 0};
  if (t < L.ncand) {
    const int i = split ? (t >> 1) : t, j = split ? (t & 1) : 0;
    const int z = wrapi(z_lo + i, g.K[2]);
    int q0, q1;
    if (!split) { q0 = qa; q1 = qa + nq; }
    else if (j == 0) { q0 = qa; q1 = g.NQ; }
    else { q0 = 0; q1 = qa + nq - g.NQ; }
    const int b0 = (xsplit * g.K[2] + z) * g.NQ;
    L.b0 = bin_start[b0 + q0];
    L.b1 = bin_start[b0 + q1];
  }
  return L;
}

// Called by every thread of the block (contains barriers).
__device__ __forceinline__ void ranges_finish(Ranges& R, const RangeLoad& L) {
  const int t = threadIdx.x;
  if (t < L.ncand) {
    R.b[t][0] = L.b0;
    R.b[t][1] = L.b1;
  }
  __syncthreads();
  if (t == 0) {
    int n = 0, acc = 0;
    for (int c = 0; c < L.ncand; ++c) {
      const int p0 = R.b[c][0], p1 = R.b[c][1];
      if (p1 > p0) {
        if (n > 0 && R.lo[n - 1] + (acc - R.pre[n - 1]) == p0) {
          acc += p1 - p0;  // continues the previous range
        } else {
          R.lo[n] = p0;
          R.pre[n] = acc;
          acc += p1 - p0;
          ++n;
        }
      }
    }
    R.pre[n] = acc;
    R.n = n;
  }
  __syncthreads();
}

__device__ __forceinline__ void build_ranges(Ranges& R, const int* __restrict__ bin_start, const Geo& g,
                                             int xsplit, int z_lo, int nplanes, int q_lo, int nq) {
  ranges_finish(R, range_load(bin_start, g, xsplit, z_lo, nplanes, q_lo, nq));
}

__device__ __forceinline__ int range_index(const Ranges& R, int v) {
  int r = 0;
  while (r + 1 < R.n && R.pre[r + 1] <= v) ++r;
  return R.lo[r] + (v - R.pre[r]);
}

// The same for at most two ranges (consecutive planes of one split are
// contiguous in the sorted order, so a run of planes is one range, or two
// where it wraps past the last plane); pre[1] is the total when n == 1.
__device__ __forceinline__ int range_index2(const Ranges& R, int v) {
  const int p1 = R.pre[1];
  return v < p1 ? R.lo[0] + v : R.lo[1] + (v - p1);
}

// Blocks are dealt to the 8 XCDs of the device round-robin (block b runs on
// XCD b mod 8).  Block b of a per-plane kernel with Kz planes and nsplit
// particle splits serves (plane z, split): with Kz a multiple of 8, XCD x
// takes the slab of planes [x Kz/8, (x+1) Kz/8) for every split, so its L2
// holds the particles (and mesh rows) of one slab plus its stencil overhang
// instead of every plane.
constexpr int kNumXcd = 8;
__device__ __forceinline__ void plane_of_block(int b, int Kz, int nsplit, int& z, int& split) {
  if ((Kz % kNumXcd) == 0) {
    const int xcd = b % kNumXcd, j = b / kNumXcd;
    split = j % nsplit;
    z = xcd * (Kz / kNumXcd) + j / nsplit;
  } else {
    z = b % Kz;
    split = b / Kz;
  }
}


// ----------------------------------------------------------------------------
// 64-bit fixed-point charge accumulators.  FP32 plans scale every term by a
// power of two S = 2^(30 - e), with 2^e > max |q| over the particles: a term
// q w (|w| <= 1) becomes round(q w S), |q w S| < 2^30, one FP32 multiply and
// one conversion to int32 whose rounding is at most 2^-31 max|q| in charge
// units; the 64-bit sums then hold any total.  FP64 plans use S = 2^40
// (|mesh charge| < 2^23).  Integer sums do not depend on the order of the
// additions, so the mesh is bitwise repeatable.
// ----------------------------------------------------------------------------
__device__ __forceinline__ float fixed_scale_fp32(unsigned qmax_bits) {
  const float qm = __uint_as_float(qmax_bits);
  if (!(qm > 0.0f) || !isfinite(qm)) return 1.0f;
  int e;
  (void)frexpf(qm, &e);  // qm < 2^e
  return ldexpf(1.0f, 30 - e);
}

// c is the already scaled term
template <typename T>
__device__ __forceinline__ long long to_fixed(T c) {
  if constexpr (sizeof(T) == 4) return (long long)(int)rintf(c);
  else return (long long)llrint(c);
}

// ----------------------------------------------------------------------------
// Charge spreading into an LDS pencil (owner computes its halo), then the
// real-to-complex transform along x.
//
// Tile t owns rows y in [y0, y0+scy), z in [z0, z0+scz), all x.  Its blocks
// visit every particle whose stencil touches those rows (its own bins and the
// p-1 planes / one row group below) and add only the owned part of each
// stencil, so every mesh value is complete inside one LDS tile and no block
// writes another's rows.  With nsplit > 1 the particles are further divided
// by stencil-start column (s_x / xs); block (t, split) spreads one part and
// writes its own partial spectrum, and the y pass adds the partial spectra in
// split order (deterministic).  Rows carry p-1 extra columns so the stencil
// never wraps in x inside the hot loop; the overhang is folded back before
// the transform.  Accumulation is in 64-bit fixed point with integer LDS
// atomics (exact, order independent).  After the spread the tile is converted
// in place to complex rows packed in pairs (even row = real part, odd row =
// imaginary part), so one complex FFT transforms two real rows; the two half
// spectra are separated with the Hermitian symmetry of each.
// ----------------------------------------------------------------------------
template <typename T, int P>
__global__ void __launch_bounds__(512) k_spread_fftx(const T4<T>* __restrict__ sorted,
                                                     const int* __restrict__ sidx,
                                                     const int* __restrict__ bin_start,
                                                     const unsigned* __restrict__ qmax_part, int nqpart,
                                                     cpx<T>* __restrict__ spec, size_t split_stride,
                                                     const cpx<T>* __restrict__ twg, Geo g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  const int nrows = g.scy * g.scz;
  const int nrc = nrows >> 1;
  constexpr int XH = P - 1;                                      // x overhang
  const int RX = Kx + XH;                                        // accumulator row length
  long long* acc = reinterpret_cast<long long*>(smem);          // [nrows][RX]
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem);               // [nrc][RS] after conversion
  const int RS = padded_len(Kx) + 1;                             // odd row stride (banks)
  const size_t acc_bytes = (size_t)nrows * RX * sizeof(long long);
  const size_t cpx_bytes = (size_t)nrc * RS * sizeof(cpx<T>);
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem + (acc_bytes > cpx_bytes ? acc_bytes : cpx_bytes));
  __shared__ Ranges R;
  __shared__ unsigned qm_s;

  const int ntiles = g.spy * g.spz;
  const int tile_id = blockIdx.x % ntiles, split = blockIdx.x / ntiles;
  const int py = tile_id % g.spy, pz = tile_id / g.spy;
  const int y0 = py * g.scy, z0 = pz * g.scz;

  if (threadIdx.x == 0) qm_s = 0u;
  for (int e = threadIdx.x; e < nrows * RX; e += blockDim.x) acc[e] = 0;
  copy_g2s<8>(tw, twg, g.twN);
  {
    const int nplanes = min(g.scz + P - 1, Kz);
    const int ylo = y0 - (P - 1);
    const int qm = (1 << g.qshift) - 1;
    const int q_lo = (ylo >= 0) ? (ylo >> g.qshift) : -((qm - ylo) >> g.qshift);
    const int q_hi = (y0 + g.scy - 1) >> g.qshift;
    const int nq = min(q_hi - q_lo + 1, g.NQ);
    build_ranges(R, bin_start, g, split, z0 - (P - 1), nplanes, q_lo, nq);  // contains barriers
  }
  T scale;
  if constexpr (sizeof(T) == 4) {
    unsigned qb = 0u;
    for (int i = threadIdx.x; i < nqpart; i += blockDim.x) qb = max(qb, qmax_part[i]);
    qb = wave_max_u32(qb);
    if ((threadIdx.x & 63) == 0 && qb) atomicMax(&qm_s, qb);
    __syncthreads();
    scale = fixed_scale_fp32(qm_s);
  } else {
    scale = (T)1099511627776.0;  // 2^40
  }

  const int total = R.pre[R.n];
  constexpr int PB = 4;  // particles fetched per thread before processing
  for (int v0 = threadIdx.x; v0 < total; v0 += PB * blockDim.x) {
    T4<T> pts[PB];
    int sps[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int v = v0 + u * blockDim.x;
      if (v < total) {
        const int idx = range_index(R, v);
        pts[u] = sorted[idx];
        sps[u] = sidx[idx];
      }
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      if (v0 + u * blockDim.x >= total) continue;
      const T4<T> pt = pts[u];
      const int sp = sps[u];
      const int sx = sp & 1023, sy = (sp >> 10) & 1023, sz = sp >> 20;
      T wx[P], wy[P], wz[P];
      bspline_weights<T, P>(pt.x, wx);
      bspline_weights<T, P>(pt.y, wy);
      bspline_weights<T, P>(pt.z, wz);
      const T qs = pt.w * scale;
#pragma unroll
      for (int tz = 0; tz < P; ++tz) {
        int gz = sz + tz;
        if (gz >= Kz) gz -= Kz;
        const int lz = gz - z0;
        if (lz < 0 || lz >= g.scz) continue;
        const T qz = qs * wz[tz];
#pragma unroll
        for (int ty = 0; ty < P; ++ty) {
          int gy = sy + ty;
          if (gy >= Ky) gy -= Ky;
          const int ly = gy - y0;
          if (ly < 0 || ly >= g.scy) continue;
          unsigned long long* rp =
              reinterpret_cast<unsigned long long*>(acc + imul(lz * g.scy + ly, RX) + sx);
          const T qyz = qz * wy[ty];
#pragma unroll
          for (int tx = 0; tx < P; ++tx) atomicAdd(rp + tx, (unsigned long long)to_fixed<T>(qyz * wx[tx]));
        }
      }
    }
  }
  __syncthreads();
  // fold the x overhang of every row back to the row start (periodic in x)
  for (int e = threadIdx.x; e < nrows * XH; e += blockDim.x) {
    const int row = e / XH, j = e - row * XH;
    acc[imul(row, RX) + j] += acc[imul(row, RX) + Kx + j];
  }
  __syncthreads();

  // fixed point -> complex row pairs, in place: every thread first reads all
  // of its values, the block synchronises, then it writes
  {
    constexpr int kMaxPer = 16;
    long long v[kMaxPer];
    const int per = (nrows * Kx + blockDim.x - 1) / blockDim.x;
    const int lkx = 31 - __clz(Kx);
#pragma unroll
    for (int c = 0; c < kMaxPer; ++c) {
      const int e = threadIdx.x + c * blockDim.x;
      if (c < per && e < nrows * Kx) v[c] = acc[imul(e >> lkx, RX) + (e & (Kx - 1))];
    }
    __syncthreads();
    const double inv_scale = 1.0 / (double)scale;
    T* out = reinterpret_cast<T*>(tile);
#pragma unroll
    for (int c = 0; c < kMaxPer; ++c) {
      const int e = threadIdx.x + c * blockDim.x;
      if (c < per && e < nrows * Kx) {
        const int row = e >> lkx, x = e & (Kx - 1);
        out[2 * (imul(row >> 1, RS) + lds_pad(x)) + (row & 1)] = (T)((double)v[c] * inv_scale);
      }
    }
    __syncthreads();
  }

  fft_rows<T, false, kEPT, true>(tile, nrc, Kx, RS, 1, false, tw, g.twN);

  const int Kh = g.Kh;
  cpx<T>* sp_out = spec + (size_t)split * split_stride;
  for (int e = threadIdx.x; e < nrows * Kh; e += blockDim.x) {
    const int ly = e % g.scy;
    const int rest = e / g.scy;
    const int lz = rest % g.scz;
    const int k = rest / g.scz;
    const int row = lz * g.scy + ly;
    const cpx<T>* zr = tile + imul(row >> 1, RS);
    const cpx<T> z1 = zr[lds_pad(k)];
    const cpx<T> z2 = cconj(zr[lds_pad((Kx - k) & (Kx - 1))]);
    cpx<T> out;
    if ((row & 1) == 0) {
      out = cpx<T>{(T)0.5 * (z1.x + z2.x), (T)0.5 * (z1.y + z2.y)};
    } else {
      const cpx<T> d = csub(z1, z2);
      out = cpx<T>{(T)0.5 * d.y, (T)-0.5 * d.x};
    }
    sp_out[(unsigned)imul(imul(k, Kz) + z0 + lz, Ky) + (y0 + ly)] = out;
  }
}

#ifndef DPLR_SPREAD_PB
#define DPLR_SPREAD_PB 2
#endif

// ----------------------------------------------------------------------------
// Plane spread with both forward in-plane transforms (used when one z plane
// fits in LDS).  Block (z, split) owns mesh plane z and visits every particle
// whose stencil-start plane is one of z-p+1 .. z (and whose original index
// falls in its split); each visit adds the particle's p x p points of
// that plane with the single z weight of the plane.  With no halo in x or y
// every visit does the same work, and no per-row ownership tests are needed.
// The plane is then converted to complex row pairs, transformed along x
// (real-to-complex, two rows per complex FFT), rearranged to [kx][y] and
// transformed along y, and written as spec[kx][z][y] (one partial spectrum
// per split; the z pass adds them in split order).  Where the register
// transforms apply, the conversion (with the x-overhang fold) is the x
// transform's first read, the rearrangement the y transform's first read,
// and the y transform's last write goes straight to spec.
// ----------------------------------------------------------------------------
template <typename T, int P>
__global__ void __launch_bounds__(1024) k_spread_xy(const T4<T>* __restrict__ sorted,
                                                    const int* __restrict__ sidx,
                                                    const int* __restrict__ bin_start,
                                                    const unsigned* __restrict__ qmax_part, int nqpart,
                                                    cpx<T>* __restrict__ spec, size_t split_stride,
                                                    const cpx<T>* __restrict__ twg, Geo g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2], Kh = g.Kh;
  constexpr int XH = P - 1;
  const int RX = Kx + XH;
  const int RS = padded_len(Kx) + 1;  // x-transform rows (complex pairs of real rows)
  const int RY = padded_len(Ky) + 1;  // y-transform rows ([kx][y])
  long long* acc = reinterpret_cast<long long*>(smem);  // [Ky][RX]
  cpx<T>* tx_tile = reinterpret_cast<cpx<T>*>(smem);    // [Ky/2][RS]
  cpx<T>* ty_tile = reinterpret_cast<cpx<T>*>(smem);    // [Kh][RY]
  const size_t b_acc = (size_t)Ky * RX * sizeof(long long);
  const size_t b_tx = (size_t)(Ky / 2) * RS * sizeof(cpx<T>);
  const size_t b_ty = (size_t)Kh * RY * sizeof(cpx<T>);
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem + max(b_acc, max(b_tx, b_ty)));
  __shared__ Ranges R;
  __shared__ unsigned qm_s;

  int z, split;
  plane_of_block(blockIdx.x, Kz, g.nsplit, z, split);
  // global loads first (range bounds, charge maxima), so that their latencies
  // overlap each other and the clearing of the accumulators
  const RangeLoad rl = range_load(bin_start, g, split, z - (P - 1), min(P, Kz), 0, g.NQ);
  unsigned qb = 0u;
  if constexpr (sizeof(T) == 4) {
    for (int i = threadIdx.x; i < nqpart; i += blockDim.x) qb = max(qb, qmax_part[i]);
  }
  if (threadIdx.x == 0) qm_s = 0u;
  for (int e = threadIdx.x; e < Ky * RX; e += blockDim.x) acc[e] = 0;
  copy_g2s<8>(tw, twg, g.twN);
  if constexpr (sizeof(T) == 4) {
    qb = wave_max_u32(qb);
    __syncthreads();  // qm_s initialised
    if ((threadIdx.x & 63) == 0 && qb) atomicMax(&qm_s, qb);
  }
  ranges_finish(R, rl);  // contains barriers (also publishes qm_s)
  T scale;
  if constexpr (sizeof(T) == 4) {
    scale = fixed_scale_fp32(qm_s);
  } else {
    scale = (T)1099511627776.0;  // 2^40
  }

  const int total = R.pre[R.n];
  constexpr int PB = DPLR_SPREAD_PB;  // particles fetched per thread before processing
  for (int v0 = threadIdx.x; v0 < total; v0 += PB * blockDim.x) {
    T4<T> pts[PB];
    int sps[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int v = v0 + u * blockDim.x;
      if (v < total) {
        const int idx = range_index2(R, v);  // the P planes below z: at most two ranges
        pts[u] = sorted[idx];
        sps[u] = sidx[idx];
      }
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      if (v0 + u * blockDim.x >= total) continue;
      const T4<T> pt = pts[u];
      const int sp = sps[u];
      const int sx = sp & 1023, sy = (sp >> 10) & 1023, sz = sp >> 20;
      int tz = z - sz;
      if (tz < 0) tz += Kz;
      T wx[P], wy[P], wz[P];
      bspline_weights<T, P>(pt.x, wx);
      bspline_weights<T, P>(pt.y, wy);
      bspline_weights<T, P>(pt.z, wz);
      T wzt = wz[0];
#pragma unroll
      for (int q = 1; q < P; ++q) wzt = (tz == q) ? wz[q] : wzt;
      const T qz = pt.w * scale * wzt;
#pragma unroll
      for (int ty = 0; ty < P; ++ty) {
        int gy = sy + ty;
        if (gy >= Ky) gy -= Ky;
        unsigned long long* rp = reinterpret_cast<unsigned long long*>(acc + imul(gy, RX) + sx);
        const T qyz = qz * wy[ty];
#pragma unroll
        for (int tx = 0; tx < P; ++tx) atomicAdd(rp + tx, (unsigned long long)to_fixed<T>(qyz * wx[tx]));
      }
    }
  }
  __syncthreads();
  const int lkx = 31 - __clz(Kx), lky = 31 - __clz(Ky);
  const double inv_scale = 1.0 / (double)scale;
  cpx<T>* out = spec + (size_t)split * split_stride;

  // x transform of the row pairs (2r, 2r+1) as complex rows.  The fused form
  // reads the fixed-point rows directly, folding the x overhang back and
  // converting on the way in.
  auto load_x = [&](int r, int e) {
    const long long* a0 = acc + imul(2 * r, RX);
    const long long* a1 = a0 + RX;
    long long v0 = a0[e], v1 = a1[e];
    if (e < XH) {
      v0 += a0[Kx + e];
      v1 += a1[Kx + e];
    }
    return cpx<T>{(T)((double)v0 * inv_scale), (T)((double)v1 * inv_scale)};
  };
  auto store_tx = [&](int r, int e, const cpx<T>& v) { tx_tile[imul(r, RS) + lds_pad(e)] = v; };
  if (!fft_rows_io<T, false>(tx_tile, Ky / 2, Kx, RS, tw, g.twN, load_x, store_tx)) {
    for (int e = threadIdx.x; e < Ky * XH; e += blockDim.x) {
      const int row = e / XH, j = e - row * XH;
      acc[imul(row, RX) + j] += acc[imul(row, RX) + Kx + j];
    }
    __syncthreads();
    // fixed point -> complex row pairs (in place through registers)
    constexpr int kMaxPer = 16;
    long long v[kMaxPer];
#pragma unroll
    for (int c = 0; c < kMaxPer; ++c) {
      const int e = threadIdx.x + c * blockDim.x;
      if (e < Ky * Kx) v[c] = acc[imul(e >> lkx, RX) + (e & (Kx - 1))];
    }
    __syncthreads();
    T* o = reinterpret_cast<T*>(tx_tile);
#pragma unroll
    for (int c = 0; c < kMaxPer; ++c) {
      const int e = threadIdx.x + c * blockDim.x;
      if (e < Ky * Kx) {
        const int row = e >> lkx, x = e & (Kx - 1);
        o[2 * (imul(row >> 1, RS) + lds_pad(x)) + (row & 1)] = (T)((double)v[c] * inv_scale);
      }
    }
    __syncthreads();
    fft_rows<T, false, kEPT, true>(tx_tile, Ky / 2, Kx, RS, 1, false, tw, g.twN);
  }

  // y transform of the kx rows: the two half spectra of every row pair are
  // separated on the way in, and the fused form writes the spectrum directly
  auto load_y = [&](int k, int y) {
    const cpx<T>* zr = tx_tile + imul(y >> 1, RS);
    const cpx<T> z1 = zr[lds_pad(k)];
    const cpx<T> z2 = cconj(zr[lds_pad((Kx - k) & (Kx - 1))]);
    if ((y & 1) == 0) return cpx<T>{(T)0.5 * (z1.x + z2.x), (T)0.5 * (z1.y + z2.y)};
    const cpx<T> d = csub(z1, z2);
    return cpx<T>{(T)0.5 * d.y, (T)-0.5 * d.x};
  };
  auto store_spec = [&](int k, int y, const cpx<T>& v) { out[(unsigned)imul(imul(k, Kz) + z, Ky) + y] = v; };
  if (fft_rows_io<T, false>(ty_tile, Kh, Ky, RY, tw, g.twN, load_y, store_spec)) return;
  {
    constexpr int kMaxOut = 16;
    cpx<T> o[kMaxOut];
#pragma unroll
    for (int c = 0; c < kMaxOut; ++c) {
      const int e = threadIdx.x + c * blockDim.x;  // e = kx * Ky + y
      if (e < Kh * Ky) o[c] = load_y(e >> lky, e & (Ky - 1));
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxOut; ++c) {
      const int e = threadIdx.x + c * blockDim.x;
      if (e < Kh * Ky) ty_tile[imul(e >> lky, RY) + lds_pad(e & (Ky - 1))] = o[c];
    }
    __syncthreads();
  }
  fft_rows<T, false, kEPT, true>(ty_tile, Kh, Ky, RY, 1, false, tw, g.twN);
  for (int e = threadIdx.x; e < Kh * Ky; e += blockDim.x) {
    const int k = e >> lky, y = e & (Ky - 1);
    out[(unsigned)imul(imul(k, Kz) + z, Ky) + y] = ty_tile[imul(k, RY) + lds_pad(y)];
  }
}

// Sum of the partial spectra of the particle splits in split order (inspection copy).
template <typename T>
__global__ void k_sum_partials(cpx<T>* __restrict__ dst, const cpx<T>* __restrict__ src, int nsum, size_t stride,
                               size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cpx<T> a = src[i];
  for (int s = 1; s < nsum; ++s) a = cadd(a, src[(size_t)s * stride + i]);
  dst[i] = a;
}

// ----------------------------------------------------------------------------
// Transforms along y of contiguous blocks of zb rows (forward on the charge
// spectrum, after adding the partial spectra of the particle splits; inverse on the
// three field spectra).
// Used forward on spec and inverse on the three field spectra.
// ----------------------------------------------------------------------------
// Final FP64 reduction of the z-pass partials with a fixed tree (bitwise
// deterministic); run by block 0 of the inverse y pass, which follows the
// z pass on the stream.
__device__ void reduce_partials(const double* __restrict__ partials, int nblk, double pre,
                                double* __restrict__ energy, double* __restrict__ virial, double* red) {
  // red: 7 * blockDim.x doubles of LDS
  const int t = threadIdx.x, nt = blockDim.x;
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    double a = 0.0;
    for (int b = t; b < nblk; b += nt) a += partials[(size_t)b * 8 + c];
    red[c * nt + t] = a;
  }
  __syncthreads();
  // pairwise tree over the next power of two (any block size)
  int top = 1;
  while (top < nt) top <<= 1;
  for (int h = top >> 1; h > 0; h >>= 1) {
    if (t < h && t + h < nt) {
#pragma unroll
      for (int c = 0; c < 7; ++c) red[c * nt + t] += red[c * nt + t + h];
    }
    __syncthreads();
  }
  if (t == 0) *energy = pre * red[0];
  if (t >= 1 && t < 7 && virial) virial[t - 1] = pre * red[t * nt];
}

template <typename T, bool INV>
__global__ void __launch_bounds__(kFftyThreads) k_ffty(cpx<T>* __restrict__ data, const cpx<T>* __restrict__ twg, Geo g,
                                              int nsum, size_t sum_stride,
                                              const double* __restrict__ partials, double pre,
                                              double* __restrict__ energy, double* __restrict__ virial) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Ky = g.K[1], Kz = g.K[2];
  const int RS = padded_len(Ky) + 1;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* tw = buf + g.zb * RS;
  const int nzb = Kz / g.zb;
  const int plane = blockIdx.x / nzb, zblk = blockIdx.x % nzb;
  cpx<T>* base = data + ((size_t)plane * Kz + (size_t)zblk * g.zb) * Ky;
  const int n = g.zb * Ky, lky = 31 - __clz(Ky);
  for (int b0 = threadIdx.x; b0 < n; b0 += 16 * blockDim.x) {
    cpx<T> r[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = b0 + u * blockDim.x;
      if (e < n) r[u] = base[e];
    }
    // partial spectra of the other particle splits, added in split order
    for (int sp = 1; sp < nsum; ++sp) {
      const cpx<T>* ps = base + (size_t)sp * sum_stride;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = b0 + u * blockDim.x;
        if (e < n) r[u] = cadd(r[u], ps[e]);
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = b0 + u * blockDim.x;
      if (e < n) buf[imul(e >> lky, RS) + lds_pad(e & (Ky - 1))] = r[u];
    }
  }
  copy_g2s<8>(tw, twg, g.twN);
  __syncthreads();
  fft_rows<T, INV, kEPT, true>(buf, g.zb, Ky, RS, 1, false, tw, g.twN);
  for (int e = threadIdx.x; e < n; e += blockDim.x) base[e] = buf[imul(e >> lky, RS) + lds_pad(e & (Ky - 1))];
  if (INV && energy && blockIdx.x == 0) {
    __syncthreads();
    reduce_partials(partials, g.nzblk, pre, energy, virial, reinterpret_cast<double*>(smem));
  }
}

// ----------------------------------------------------------------------------
// Forward transform along z of yb columns of
// one kx plane, the influence-function multiply with ik-differentiation, the
// FP64 energy and virial partial sums, and the three inverse z transforms.
//
//   E^_a(n) = -i k'_a G(n) Q^(n),  k' = k with the Nyquist component zeroed;
//   e  = sum w G |Q^|^2,  w = 1 on the kx = 0 and kx = Kx/2 planes, else 2;
//   v_ab = sum w G |Q^|^2 (delta_ab - 2 (1 + k^2/(4 beta^2)) k_a k_b / k^2)
//   (off-diagonal products use k', since full-spectrum terms with a Nyquist
//   component cancel in +-n pairs).
// ----------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_fftz_poisson(const cpx<T>* __restrict__ spec, int nsum, size_t sum_stride,
                                                       int ncomp, cpx<T>* __restrict__ fspec,
                                                       const double* __restrict__ G, double* __restrict__ partials,
                                                       const cpx<T>* __restrict__ twg, Geo g, PoissonConsts pc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2], Kh = g.Kh;
  const int yb = g.yb, w3 = 3 * yb;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem);  // [Kz][3*yb]
  cpx<T>* tw = buf + Kz * w3;
  __shared__ double red[16][8];

  const int lyb = 31 - __clz(yb);  // yb is a power of two
  const int nyb = Ky >> lyb;
  // XCD-aware order: the f consecutive column blocks that share 128-byte
  // lines of the outputs run on one XCD (blocks are dealt to the 8 XCDs
  // round-robin), so no line is written from two L2s.  The grid is padded to
  // a multiple of 8 f; padding blocks leave at once.
  const int f = g.zgroup;
  const int bg = blockIdx.x / (8 * f), bw = blockIdx.x - bg * 8 * f;
  const int blk = bg * 8 * f + (bw & 7) * f + (bw >> 3);
  if (blk >= g.nzblk) return;
  const int kx = blk / nyb, y0 = (blk - kx * nyb) << lyb;
  const unsigned col0 = (unsigned)imul(imul(kx, Kz), Ky) + y0;  // spec[kx][0][y0]
  const int n = Kz << lyb;                                      // elements (z, yl), yl fastest
  // forward z transform of the yb columns, the partial spectra of the particle
  // splits added in split order on the way in
  copy_g2s<8>(tw, twg, g.twN);
  auto load_s = [&](int yl, int z) {
    const unsigned o = col0 + imul(z, Ky) + yl;
    cpx<T> v = spec[o];
    for (int sp = 1; sp < nsum; ++sp) v = cadd(v, spec[(size_t)sp * sum_stride + o]);
    return v;
  };
  auto store_b = [&](int yl, int z, const cpx<T>& v) { buf[imul(z, w3) + yl] = v; };
  if (!fft_cols_io<T, false>(buf, yb, Kz, w3, tw, g.twN, load_s, store_b)) {
    for (int base = threadIdx.x; base < n; base += 8 * blockDim.x) {
      cpx<T> r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * blockDim.x;
        if (e < n) r[u] = spec[col0 + imul(e >> lyb, Ky) + (e & (yb - 1))];
      }
      // partial spectra of the other particle splits, added in split order
      for (int sp = 1; sp < nsum; ++sp) {
        const cpx<T>* ps = spec + (size_t)sp * sum_stride;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = base + u * blockDim.x;
          if (e < n) r[u] = cadd(r[u], ps[col0 + imul(e >> lyb, Ky) + (e & (yb - 1))]);
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * blockDim.x;
        if (e < n) buf[imul(e >> lyb, w3) + (e & (yb - 1))] = r[u];
      }
    }
    __syncthreads();
    fft_rows<T, false, kEPT>(buf, yb, Kz, 1, w3, true, tw, g.twN);
  }

  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const int Kyh = Ky / 2 + 1, Kzh = Kz / 2 + 1;
  const double wgt = (kx == 0 || kx == Kx / 2) ? 1.0 : 2.0;
  const double kxv = pc.two_pi_over_L[0] * kx;
  const double kxd = (kx == Kx / 2) ? 0.0 : kxv;
  for (int base = threadIdx.x; base < n; base += 8 * blockDim.x) {
    double Gr[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * blockDim.x;
      if (e < n) {
        const int yl = e & (yb - 1), z = e >> lyb, ny = y0 + yl;
        Gr[u] = G[(unsigned)imul(imul(kx, Kyh) + min(ny, Ky - ny), Kzh) + min(z, Kz - z)];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * blockDim.x;
      if (e >= n) continue;
      const int yl = e & (yb - 1), z = e >> lyb;
      const int ny = y0 + yl;
      const double kyv = pc.two_pi_over_L[1] * (ny <= Ky / 2 ? ny : ny - Ky);
      const double kzv = pc.two_pi_over_L[2] * (z <= Kz / 2 ? z : z - Kz);
      const double kyd = (2 * ny == Ky) ? 0.0 : kyv;
      const double kzd = (2 * z == Kz) ? 0.0 : kzv;
      const double Gv = Gr[u];
      cpx<T>* bz = buf + imul(z, w3) + yl;
      const cpx<T> q = bz[0];
      const double s2 = (double)q.x * (double)q.x + (double)q.y * (double)q.y;
      const double t = wgt * Gv * s2;
      const double k2 = kxv * kxv + kyv * kyv + kzv * kzv;
      const double c = (k2 > 0.0) ? 2.0 * (1.0 + k2 * pc.inv_4beta2) / k2 : 0.0;
      acc[0] += t;
      acc[1] += t * (1.0 - c * kxv * kxv);
      acc[2] += t * (1.0 - c * kyv * kyv);
      acc[3] += t * (1.0 - c * kzv * kzv);
      acc[4] += t * (-c * kxd * kyd);
      acc[5] += t * (-c * kxd * kzd);
      acc[6] += t * (-c * kyd * kzd);
      if (ncomp == 1) {
        // analytic differentiation: the potential spectrum G Q^
        const T gv = (T)Gv;
        bz[0] = cpx<T>{gv * q.x, gv * q.y};
      } else {
        // -i k' G Q^ = k' G (q.y, -q.x)
        const T gx = (T)(Gv * kxd), gy = (T)(Gv * kyd), gz = (T)(Gv * kzd);
        bz[0] = cpx<T>{gx * q.y, -gx * q.x};
        bz[yb] = cpx<T>{gy * q.y, -gy * q.x};
        bz[2 * yb] = cpx<T>{gz * q.y, -gz * q.x};
      }
    }
  }
  __syncthreads();
  // ncomp inverse z transforms (three field components, or the potential);
  // the fused form writes the spectra directly
  const unsigned fstride = (unsigned)imul(imul(Kh, Kz), Ky);
  auto store_f = [&](int c, int z, const cpx<T>& v) {
    const int a = c >> lyb, yl = c & (yb - 1);  // column c = a * yb + yl
    fspec[a * fstride + col0 + imul(z, Ky) + yl] = v;
  };
  auto load_b = [&](int c, int z) { return buf[imul(z, w3) + c]; };
  if (!fft_cols_io<T, true>(buf, ncomp * yb, Kz, w3, tw, g.twN, load_b, store_f)) {
    fft_rows<T, true, kEPT>(buf, ncomp * yb, Kz, 1, w3, true, tw, g.twN);
    // store: e = ((z * ncomp + a) << lyb) + yl
    for (int e = threadIdx.x; e < ncomp * n; e += blockDim.x) {
      const int za = e >> lyb, yl = e & (yb - 1);
      const int z = za / ncomp, a = za - ncomp * z;
      fspec[a * fstride + col0 + imul(z, Ky) + yl] = buf[imul(z, w3) + imul(a, yb) + yl];
    }
  }

  // deterministic block reduction of the 7 FP64 partial sums
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    double v = acc[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    double v = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) v += red[w][threadIdx.x];
    partials[(size_t)blk * 8 + threadIdx.x] = v;
  }
}

// ----------------------------------------------------------------------------
// Inverse complex-to-real transform along x of the three field spectra.  A
// workgroup takes one z plane and yb consecutive y rows of all three fields
// (3 * yb real rows, transformed in pairs as complex rows) and writes the
// real fields interleaved, E[z][y][x] = (Ex, Ey, Ez), so the gather reads one
// 3-component record per stencil point.
// ----------------------------------------------------------------------------
#ifndef DPLR_GATHER_OCC
#define DPLR_GATHER_OCC
#endif

template <typename T>
struct F3 {
  T x, y, z;
};

// x padding of the potential's rows (analytic differentiation): covers the
// 16-byte chunks of any stencil of up to 8 points that starts at x <= Kx - 1
// (and keeps rows 16-byte aligned)
constexpr int kGatherAdPad = 8;

// ncomp = 3 writes the interleaved field records; ncomp = 1 (analytic
// differentiation) writes the potential in rows of Kx + kGatherAdPad values,
// the last ones repeating x = 0, 1, ...
template <typename T>
__global__ void __launch_bounds__(512) k_ifftx(const cpx<T>* __restrict__ fspec, T* __restrict__ field, int ncomp,
                                               const cpx<T>* __restrict__ twg, Geo g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2], Kh = g.Kh;
  const int yb = g.xyb;                  // y rows per block
  const int nrc = (ncomp * yb) / 2;      // complex rows: pair (2c, 2c+1) of rows r = a*yb + yl
  const int RS = padded_len(Kx) + 1;
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem);  // [nrc][RS]
  cpx<T>* tw = tile + (size_t)nrc * RS;
  const int nyb = Ky / yb;
  const int z = blockIdx.x / nyb, y0 = (blockIdx.x % nyb) * yb;
  const size_t fstride = (size_t)Kh * Kz * Ky, plane = (size_t)Kz * Ky;
  copy_g2s<8>(tw, twg, g.twN);

  // load: thread -> (pair c, kx = k0, k0 + kstep, ...)
  const int c_t = threadIdx.x % nrc, k_t = threadIdx.x / nrc, kstep = blockDim.x / nrc;
  if (k_t < kstep) {
    const int r0 = 2 * c_t, r1 = r0 + 1;
    const cpx<T>* s0 = fspec + (size_t)(r0 / yb) * fstride + (size_t)z * Ky + y0 + r0 % yb;
    const cpx<T>* s1 = fspec + (size_t)(r1 / yb) * fstride + (size_t)z * Ky + y0 + r1 % yb;
    cpx<T>* zr = tile + imul(c_t, RS);
    for (int kb = k_t; kb < Kh; kb += 4 * kstep) {
      cpx<T> A[4], B[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = kb + u * kstep;
        if (kk < Kh) { A[u] = s0[(size_t)kk * plane]; B[u] = s1[(size_t)kk * plane]; }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = kb + u * kstep;
        if (kk < Kh) {
          cpx<T> av = A[u], bv = B[u];
          if (kk == 0 || kk == Kx / 2) { av.y = (T)0; bv.y = (T)0; }
          zr[lds_pad(kk)] = cpx<T>{av.x - bv.y, av.y + bv.x};
          if (kk > 0 && kk < Kx / 2) zr[lds_pad(Kx - kk)] = cpx<T>{av.x + bv.y, bv.x - av.y};
        }
      }
    }
  }
  __syncthreads();
  fft_rows<T, true, kEPT, true>(tile, nrc, Kx, RS, 1, false, tw, g.twN);

  // store: record (yl, x) gathers component a from row r = a*yb + yl
  const T* tr = reinterpret_cast<const T*>(tile);
  const int lkx = 31 - __clz(Kx);
  if (ncomp == 3) {
    F3<T>* out = reinterpret_cast<F3<T>*>(field) + ((size_t)z * Ky + y0) * Kx;
    for (int e = threadIdx.x; e < yb * Kx; e += blockDim.x) {
      const int yl = e >> lkx, x = e & (Kx - 1);
      const int col = 2 * lds_pad(x);
      T v[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int r = a * yb + yl;
        v[a] = tr[2 * imul(r >> 1, RS) + col + (r & 1)];
      }
      out[e] = F3<T>{v[0], v[1], v[2]};
    }
  } else {
    const int RX = Kx + kGatherAdPad;
    T* out = field + ((size_t)z * Ky + y0) * RX;
    for (int e = threadIdx.x; e < yb * Kx; e += blockDim.x) {
      const int yl = e >> lkx, x = e & (Kx - 1);
      const T v = tr[2 * imul(yl >> 1, RS) + 2 * lds_pad(x) + (yl & 1)];
      out[imul(yl, RX) + x] = v;
      if (x < kGatherAdPad) out[imul(yl, RX) + Kx + x] = v;
    }
  }
}

// ----------------------------------------------------------------------------
// Inverse y and x transforms of one field component on one z plane (used when
// a plane fits in LDS; it replaces the separate inverse y and x passes).  The
// Kh rows (kx, z) of the component's spectrum are transformed along y, then
// recombined into complex pairs of real x rows: row pair (2c, 2c+1) takes
// A + iB for kx <= Kx/2 and conj(A) + i conj(B) at Kx - kx (Hermitian
// symmetry), with the imaginary parts of the kx = 0 and Kx/2 terms dropped.
// One inverse complex FFT per pair along x gives both real rows, written as
// component a of the interleaved field records (ncomp = 3 field components
// for ik differentiation, ncomp = 1 for the potential of analytic
// differentiation).  Block b serves plane z = 8 (b / (8 ncomp)) + b % 8 and
// component (b / 8) % ncomp, so the components of a plane land on the same XCD
// (blocks are dealt round-robin over 8 XCDs) and its L2 merges their partial
// record writes.  Block 0 also performs the final energy/virial reduction.
// ----------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_ifft_xy(const cpx<T>* __restrict__ fspec, T* __restrict__ field,
                                                  int ncomp, int xpad, const cpx<T>* __restrict__ twg, Geo g,
                                                  const double* __restrict__ partials, double pre,
                                                  double* __restrict__ energy, double* __restrict__ virial) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2], Kh = g.Kh;
  const int RS = padded_len(Kx) + 1;  // x rows (complex pairs of real rows)
  const int RY = padded_len(Ky) + 1;  // y rows ([kx][y])
  cpx<T>* ty = reinterpret_cast<cpx<T>*>(smem);  // [Kh][RY]
  cpx<T>* tx = reinterpret_cast<cpx<T>*>(smem);  // [Ky/2][RS]
  const size_t b_ty = (size_t)Kh * RY * sizeof(cpx<T>);
  const size_t b_tx = (size_t)(Ky / 2) * RS * sizeof(cpx<T>);
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem + max(b_ty, b_tx));
  const int zx = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int zg = slot / ncomp, a = slot - ncomp * zg;
  const int z = zg * 8 + zx;
  const int lkx = 31 - __clz(Kx), lky = 31 - __clz(Ky);
  copy_g2s<8>(tw, twg, g.twN);

  // rows (kx, z) of component a: Ky contiguous values each, Kz * Ky apart.
  // The fused form loads them straight into the transform's registers.
  constexpr int kMax = 16;  // host: Kh * Ky <= 16 * blockDim.x
  const cpx<T>* src = fspec + (size_t)a * Kh * Kz * Ky + (size_t)z * Ky;
  const size_t rstride = (size_t)Kz * Ky;
  auto load_g = [&](int k, int y) { return src[(size_t)k * rstride + y]; };
  auto store_ty = [&](int k, int y, const cpx<T>& v) { ty[imul(k, RY) + lds_pad(y)] = v; };
  if (!fft_rows_io<T, true>(ty, Kh, Ky, RY, tw, g.twN, load_g, store_ty)) {
    cpx<T> r[kMax];
#pragma unroll
    for (int c = 0; c < kMax; ++c) {
      const int e = threadIdx.x + c * blockDim.x;
      if (e < Kh * Ky) r[c] = load_g(e >> lky, e & (Ky - 1));
    }
#pragma unroll
    for (int c = 0; c < kMax; ++c) {
      const int e = threadIdx.x + c * blockDim.x;
      if (e < Kh * Ky) store_ty(e >> lky, e & (Ky - 1), r[c]);
    }
    __syncthreads();
    fft_rows<T, true, kEPT, true>(ty, Kh, Ky, RY, 1, false, tw, g.twN);
  }

  // complex row pairs along x: pair pr takes A + iB (A, B: rows 2pr, 2pr+1)
  // for kx <= Kx/2 and conj(A) + i conj(B) at Kx - kx.  The fused form builds
  // them on the way into the transform.
  auto load_r = [&](int pr, int m) {
    const bool up = m > Kx / 2;
    const int k = up ? Kx - m : m;
    const cpx<T>* row = ty + imul(k, RY);
    cpx<T> av = row[lds_pad(2 * pr)], bv = row[lds_pad(2 * pr + 1)];
    if (k == 0 || k == Kx / 2) { av.y = (T)0; bv.y = (T)0; }
    return up ? cpx<T>{av.x + bv.y, bv.x - av.y} : cpx<T>{av.x - bv.y, av.y + bv.x};
  };
  auto store_tx = [&](int pr, int x, const cpx<T>& v) { tx[imul(pr, RS) + lds_pad(x)] = v; };
  if (!fft_rows_io<T, true>(tx, Ky / 2, Kx, RS, tw, g.twN, load_r, store_tx)) {
    const int half = Ky >> 1, lhalf = lky - 1;
    constexpr int kPairs = kMax / 2;  // Kh * Ky / 2 <= 8 * blockDim.x
    cpx<T> A[kPairs], B[kPairs];
#pragma unroll
    for (int c = 0; c < kPairs; ++c) {
      const int i = threadIdx.x + c * blockDim.x;  // i = kx * (Ky/2) + pair
      if (i < Kh * half) {
        const int k = i >> lhalf, pr = i & (half - 1);
        const cpx<T>* row = ty + imul(k, RY);
        A[c] = row[lds_pad(2 * pr)];
        B[c] = row[lds_pad(2 * pr + 1)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kPairs; ++c) {
      const int i = threadIdx.x + c * blockDim.x;
      if (i < Kh * half) {
        const int k = i >> lhalf, pr = i & (half - 1);
        cpx<T> av = A[c], bv = B[c];
        if (k == 0 || k == Kx / 2) { av.y = (T)0; bv.y = (T)0; }
        cpx<T>* zr = tx + imul(pr, RS);
        zr[lds_pad(k)] = cpx<T>{av.x - bv.y, av.y + bv.x};
        if (k > 0 && k < Kx / 2) zr[lds_pad(Kx - k)] = cpx<T>{av.x + bv.y, bv.x - av.y};
      }
    }
    __syncthreads();
    fft_rows<T, true, kEPT, true>(tx, Ky / 2, Kx, RS, 1, false, tw, g.twN);
  }

  // real rows (y even in the real parts, y odd in the imaginary parts) to
  // component a of the field records (ncomp values per mesh point; rows of
  // Kx + xpad records, the last xpad repeating x = 0 .. xpad-1), consecutive
  // threads on consecutive x
  const T* tr = reinterpret_cast<const T*>(tx);
  const int RX = Kx + xpad;
  T* out = field + (size_t)z * Ky * RX * ncomp + a;
  for (int e = threadIdx.x; e < Ky * Kx; e += blockDim.x) {
    const int y = e >> lkx, x = e & (Kx - 1);
    const T v = tr[2 * (imul(y >> 1, RS) + lds_pad(x)) + (y & 1)];
    out[(size_t)(imul(y, RX) + x) * ncomp] = v;
    if (x < xpad) out[(size_t)(imul(y, RX) + Kx + x) * ncomp] = v;
  }
  if (energy && blockIdx.x == 0) {
    __syncthreads();
    reduce_partials(partials, g.nzblk, pre, energy, virial, reinterpret_cast<double*>(smem));
  }
}

// ----------------------------------------------------------------------------
// Force interpolation with the assignment weights of the spread, reading the
// real fields from memory (L1/L2).  P lanes serve one particle: lane tx reads
// the column s_x + tx of all P x P (y, z) rows, so each group's loads cover
// P consecutive records; the P partial sums are then added across the group.
// Blocks walk the sorted particles in order, and consecutive chunks are
// mapped to the same XCD so each XCD's L2 serves one slab of the field.
// ----------------------------------------------------------------------------
template <typename T, int P>
__global__ void __launch_bounds__(256) DPLR_GATHER_OCC k_gather(const F3<T>* __restrict__ field, const T4<T>* __restrict__ sorted,
                                                const int* __restrict__ sidx, const int* __restrict__ perm,
                                                int n, int nchunks, T* __restrict__ ion_f, T* __restrict__ wc_f,
                                                int64_t n_ion, T fscale, int accumulate, int nxcd, Geo g) {
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  constexpr int GPW = 64 / P;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / P, tx = lane - grp * P;
  const bool lane_on = grp < GPW;
  const int per_block = (blockDim.x >> 6) * GPW;
  // XCD-aware order: blocks b, b + nxcd, ... run on one XCD; give them
  // consecutive chunks of the sorted particles.  The grid is a multiple of
  // nxcd, so b -> chunk is a bijection onto [0, gridDim.x); chunks at or
  // beyond nchunks hold no particles.
  const int per_xcd = gridDim.x / nxcd;
  const int chunk = (blockIdx.x % nxcd) * per_xcd + blockIdx.x / nxcd;
  const int v = chunk * per_block + wave * GPW + grp;
  const bool on = lane_on && chunk < nchunks && v < n;
  T part[3] = {(T)0, (T)0, (T)0};
  T qw = (T)0;
  int src = 0;
  if (on) {
    const T4<T> pt = sorted[v];
    const int sp = sidx[v];
    src = perm[v];
    const int sx = sp & 1023, sy = (sp >> 10) & 1023, sz = sp >> 20;
    T wy[P], wz[P], wxt, dxt;
    bspline_weight_at<T, P>(pt.x, tx, wxt, dxt);  // this lane's column only
    bspline_weights<T, P>(pt.y, wy);
    bspline_weights<T, P>(pt.z, wz);
    int gx = sx + tx;
    if (gx >= Kx) gx -= Kx;
    // all loads of a batch of z planes are issued before any of them is used
    // (memory-level parallelism: the loop is latency bound otherwise)
    constexpr int TZB = (P <= 5) ? P : ((P <= 6) ? 3 : 2);
#pragma unroll
    for (int tz0 = 0; tz0 < P; tz0 += TZB) {
      F3<T> r[TZB][P];
#pragma unroll
      for (int dz = 0; dz < TZB; ++dz) {
        if (tz0 + dz < P) {
          int gz = sz + tz0 + dz;
          if (gz >= Kz) gz -= Kz;
          const F3<T>* fz = field + (unsigned)imul(gz, Ky) * (unsigned)Kx + gx;
#pragma unroll
          for (int ty = 0; ty < P; ++ty) {
            int gy = sy + ty;
            if (gy >= Ky) gy -= Ky;
            r[dz][ty] = fz[imul(gy, Kx)];
          }
        }
      }
#pragma unroll
      for (int dz = 0; dz < TZB; ++dz) {
        if (tz0 + dz < P) {
#pragma unroll
          for (int ty = 0; ty < P; ++ty) {
            const T w = wz[tz0 + dz] * wy[ty];
            part[0] += w * r[dz][ty].x;
            part[1] += w * r[dz][ty].y;
            part[2] += w * r[dz][ty].z;
          }
        }
      }
    }
    qw = fscale * pt.w * wxt;
  }
  const int gbase = grp * P;
  T tot[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T mine = qw * part[a];
    T s = (T)0;
#pragma unroll
    for (int q = 0; q < P; ++q) s += __shfl(mine, gbase + q, 64);
    tot[a] = s;
  }
  if (on && tx == 0) {
    T* out = (src < n_ion) ? (ion_f + 3 * (int64_t)src) : (wc_f + 3 * ((int64_t)src - n_ion));
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = accumulate ? out[a] + tot[a] : tot[a];
  }
}

// ----------------------------------------------------------------------------
// Forces by analytic differentiation: F_ja = -(k_e q_j / (V h_a)) times
// sum_g phi(g) dW(u_j - g)/du_a, with the potential phi read as one value per
// mesh point.  One lane serves one particle.  Each of its P x P stencil rows
// is read as the NC aligned 16-byte chunks that cover x = s_x .. s_x+P-1
// (from a = s_x rounded down to a chunk boundary), and the x weights are
// shifted by o = s_x - a once per particle instead (zero outside the
// stencil), so the row needs no data shuffling.  The potential's rows hold
// kGatherAdPad extra values repeating x = 0, 1, ..., so no read wraps in x.
// Per row the lane forms rx = sum wx' phi and rw = sum wx phi
// and adds wy wz rx, wy' wz rw and wy wz' rw to the three components.
// ----------------------------------------------------------------------------
template <typename T>
struct __attribute__((aligned(16))) Chunk16 {
  T v[16 / sizeof(T)];
};



template <typename T, int P>
__global__ void __launch_bounds__(256) k_gather_ad(const T* __restrict__ phi, const T4<T>* __restrict__ sorted,
                                                   const int* __restrict__ sidx, const int* __restrict__ perm,
                                                   int n, int nchunks, T* __restrict__ ion_f, T* __restrict__ wc_f,
                                                   int64_t n_ion, T fscale, T ihx, T ihy, T ihz, int accumulate,
                                                   int nxcd, Geo g) {
  constexpr int C = 16 / (int)sizeof(T);      // values per chunk
  constexpr int NC = (P + 2 * C - 2) / C;     // chunks covering P values at any offset < C
  constexpr int NW = NC * C;
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  // XCD-aware order as in k_gather: consecutive chunks of blockDim.x sorted
  // particles go to the same XCD
  const int per_xcd = gridDim.x / nxcd;
  const int chunk = (blockIdx.x % nxcd) * per_xcd + blockIdx.x / nxcd;
  const int v = chunk * blockDim.x + threadIdx.x;
  if (chunk >= nchunks || v >= n) return;
  const T4<T> pt = sorted[v];
  const int sp = sidx[v];
  const int src = perm[v];
  const int sx = sp & 1023, sy = (sp >> 10) & 1023, sz = sp >> 20;
  T wy[P], wz[P], dy[P], dz[P];
  bspline_weights<T, P>(pt.y, wy);
  bspline_weights<T, P>(pt.z, wz);
  bspline_dweights<T, P>(pt.y, dy);
  bspline_dweights<T, P>(pt.z, dz);
  const int xa = sx & ~(C - 1), o = sx - xa;
  T swx[NW], sdx[NW];  // x weights shifted by o
  {
    T wx[P], dx[P];
    bspline_weights<T, P>(pt.x, wx);
    bspline_dweights<T, P>(pt.x, dx);
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      T a = (T)0, b = (T)0;
#pragma unroll
      for (int oo = 0; oo < C; ++oo) {
        if (j - oo >= 0 && j - oo < P) {
          a = (o == oo) ? wx[j - oo] : a;
          b = (o == oo) ? dx[j - oo] : b;
        }
      }
      swx[j] = a;
      sdx[j] = b;
    }
  }
  static_assert(NW - C <= kGatherAdPad, "row padding too small for this order");
  const int RX = Kx + kGatherAdPad;
  T fx = (T)0, fy = (T)0, fz = (T)0;
  // one plane at a time (not unrolled, so that only its rows are in flight)
#pragma unroll 1
  for (int tz = 0; tz < P; ++tz) {
    T wzt = wz[0], dzt = dz[0];
#pragma unroll
    for (int k = 1; k < P; ++k) {
      wzt = (tz == k) ? wz[k] : wzt;
      dzt = (tz == k) ? dz[k] : dzt;
    }
    int gz = sz + tz;
    if (gz >= Kz) gz -= Kz;
    const T* plane = phi + (size_t)gz * Ky * RX;
    T f[P][NW];
#pragma unroll
    for (int ty = 0; ty < P; ++ty) {
      int gy = sy + ty;
      if (gy >= Ky) gy -= Ky;
      const Chunk16<T>* row = reinterpret_cast<const Chunk16<T>*>(plane + (size_t)gy * RX + xa);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const Chunk16<T> ch = row[c];
#pragma unroll
        for (int k = 0; k < C; ++k) f[ty][c * C + k] = ch.v[k];
      }
    }
#pragma unroll
    for (int ty = 0; ty < P; ++ty) {
      T rx = (T)0, rw = (T)0;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        rx += sdx[j] * f[ty][j];
        rw += swx[j] * f[ty][j];
      }
      fx += wy[ty] * wzt * rx;
      fy += dy[ty] * wzt * rw;
      fz += wy[ty] * dzt * rw;
    }
  }
  const T qs = -fscale * pt.w;
  const T tot[3] = {qs * ihx * fx, qs * ihy * fy, qs * ihz * fz};
  T* out = (src < n_ion) ? (ion_f + 3 * (int64_t)src) : (wc_f + 3 * ((int64_t)src - n_ion));
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = accumulate ? out[a] + tot[a] : tot[a];
}

// ----------------------------------------------------------------------------
// The same forces with P lanes per particle (used for orders above 6, where
// one lane would hold too many stencil rows in flight): lane tx reads the
// column s_x + tx of all P x P (y, z) rows of the padded potential and keeps
// three partial sums, phi wy wz (for the x derivative), phi wy' wz and
// phi wy wz' (for y and z), which it then weights by wx' or wx before the
// sums over the group.
// ----------------------------------------------------------------------------
template <typename T, int P>
__global__ void __launch_bounds__(256) k_gather_ad_lanes(const T* __restrict__ phi, const T4<T>* __restrict__ sorted,
                                                   const int* __restrict__ sidx, const int* __restrict__ perm,
                                                   int n, int nchunks, T* __restrict__ ion_f, T* __restrict__ wc_f,
                                                   int64_t n_ion, T fscale, T ihx, T ihy, T ihz, int accumulate,
                                                   int nxcd, Geo g) {
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  const int RX = Kx + kGatherAdPad;
  constexpr int GPW = 64 / P;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / P, tx = lane - grp * P;
  const bool lane_on = grp < GPW;
  const int per_block = (blockDim.x >> 6) * GPW;
  const int per_xcd = gridDim.x / nxcd;
  const int chunk = (blockIdx.x % nxcd) * per_xcd + blockIdx.x / nxcd;
  const int v = chunk * per_block + wave * GPW + grp;
  const bool on = lane_on && chunk < nchunks && v < n;
  T mine[3] = {(T)0, (T)0, (T)0};
  int src = 0;
  if (on) {
    const T4<T> pt = sorted[v];
    const int sp = sidx[v];
    src = perm[v];
    const int sx = sp & 1023, sy = (sp >> 10) & 1023, sz = sp >> 20;
    T wy[P], wz[P], dy[P], dz[P], wxt, dxt;
    bspline_weight_at<T, P>(pt.x, tx, wxt, dxt);  // this lane's column only
    bspline_weights<T, P>(pt.y, wy);
    bspline_weights<T, P>(pt.z, wz);
    bspline_dweights<T, P>(pt.y, dy);
    bspline_dweights<T, P>(pt.z, dz);
    int gx = sx + tx;
    if (gx >= Kx) gx -= Kx;
    T s0 = (T)0, s1 = (T)0, s2 = (T)0;
    constexpr int TZB = (P <= 5) ? P : ((P <= 6) ? 3 : 2);
#pragma unroll
    for (int tz0 = 0; tz0 < P; tz0 += TZB) {
      T r[TZB][P];
#pragma unroll
      for (int d = 0; d < TZB; ++d) {
        if (tz0 + d < P) {
          int gz = sz + tz0 + d;
          if (gz >= Kz) gz -= Kz;
          const T* fz = phi + (size_t)gz * Ky * RX + gx;
#pragma unroll
          for (int ty = 0; ty < P; ++ty) {
            int gy = sy + ty;
            if (gy >= Ky) gy -= Ky;
            r[d][ty] = fz[imul(gy, RX)];
          }
        }
      }
#pragma unroll
      for (int d = 0; d < TZB; ++d) {
        if (tz0 + d < P) {
          const int tz = tz0 + d;
          T a0 = (T)0, a1 = (T)0;
#pragma unroll
          for (int ty = 0; ty < P; ++ty) {
            a0 += wy[ty] * r[d][ty];
            a1 += dy[ty] * r[d][ty];
          }
          s0 += wz[tz] * a0;
          s1 += wz[tz] * a1;
          s2 += dz[tz] * a0;
        }
      }
    }
    const T qs = -fscale * pt.w;
    mine[0] = qs * ihx * dxt * s0;
    mine[1] = qs * ihy * wxt * s1;
    mine[2] = qs * ihz * wxt * s2;
  }
  const int gbase = grp * P;
  T tot[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T s = (T)0;
#pragma unroll
    for (int k = 0; k < P; ++k) s += __shfl(mine[a], gbase + k, 64);
    tot[a] = s;
  }
  if (on && tx == 0) {
    T* out = (src < n_ion) ? (ion_f + 3 * (int64_t)src) : (wc_f + 3 * ((int64_t)src - n_ion));
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = accumulate ? out[a] + tot[a] : tot[a];
  }
}

// ----------------------------------------------------------------------------
// FP64 optimal influence function for ik-differentiation (per box).
//   G(k) = sum_m (k.k_m) U^2(k_m) phi(k_m) / (|k|^2 [sum_m U^2(k_m)]^2),
//   k_m = k + 2 pi m / h, U(k) = prod_a sinc(k_a h_a / 2)^p,
//   phi(k) = 4 pi exp(-k^2 / (4 beta^2)) / k^2.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double sinc_alias(int n, int K, int m) {
  // sinc(pi (n/K + m)) with sin(pi(n/K + m)) = (-1)^m sin(pi n/K)
  if (n == 0) return (m == 0) ? 1.0 : 0.0;
  const double x = (double)n / (double)K + (double)m;
  const double s = sinpi((double)n / (double)K);
  return ((m & 1) ? -s : s) / (M_PI * x);
}

__global__ void k_influence(double* __restrict__ G, Geo g, double Lx, double Ly, double Lz, double beta, int p,
                            int alias) {
  const int Kxh = g.K[0] / 2 + 1, Kyh = g.K[1] / 2 + 1, Kzh = g.K[2] / 2 + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Kxh * Kyh * Kzh) return;
  const int az = (int)(i % Kzh);
  const int ay = (int)((i / Kzh) % Kyh);
  const int ax = (int)(i / ((int64_t)Kzh * Kyh));
  const int n[3] = {ax, ay, az};
  const double L[3] = {Lx, Ly, Lz};
  double k[3];
  for (int a = 0; a < 3; ++a) k[a] = 2.0 * M_PI * n[a] / L[a];
  const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  if (k2 == 0.0) {
    G[i] = 0.0;
    return;
  }
  const double inv4b2 = 1.0 / (4.0 * beta * beta);
  double u2[3][9];
  double km[3][9];
  for (int a = 0; a < 3; ++a) {
    for (int m = -alias; m <= alias; ++m) {
      double s = sinc_alias(n[a], g.K[a], m);
      double s2 = s * s, sp = 1.0;
      for (int t = 0; t < p; ++t) sp *= s2;
      u2[a][m + alias] = sp;
      km[a][m + alias] = 2.0 * M_PI * ((double)n[a] + (double)m * g.K[a]) / L[a];
    }
  }
  double num = 0.0, den = 0.0;
  for (int mx = 0; mx <= 2 * alias; ++mx)
    for (int my = 0; my <= 2 * alias; ++my)
      for (int mz = 0; mz <= 2 * alias; ++mz) {
        const double u = u2[0][mx] * u2[1][my] * u2[2][mz];
        den += u;
        if (u == 0.0) continue;
        const double kx = km[0][mx], ky = km[1][my], kz = km[2][mz];
        const double kk = kx * kx + ky * ky + kz * kz;
        const double phi = 4.0 * M_PI * exp(-kk * inv4b2) / kk;
        num += (k[0] * kx + k[1] * ky + k[2] * kz) * u * phi;
      }
  G[i] = num / (k2 * den * den);
}

// ----------------------------------------------------------------------------
// Backward of E with respect to positions: grad = -g * F.
// ----------------------------------------------------------------------------
template <typename T>
__global__ void k_scale_grad(const double* __restrict__ gE, const T* __restrict__ f, T* __restrict__ out, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  out[i] = (T)(-(*gE) * (double)f[i]);
}

}  // namespace dplr
