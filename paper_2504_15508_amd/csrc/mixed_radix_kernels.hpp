// PPPM-ik on meshes whose sizes are not all powers of two.
//
// The paper runs its precision study on small per-node grids such as
// 8x12x8, 10x15x10 and 12x18x12 (Results, accuracy of the precision
// variants), which the plane/pencil kernels cannot take: those assume
// power-of-two rows for their register transforms, bins and index masks.
// This path computes the same steps as the tuned one (spread, forward 3D
// transform, optimal-G ik multiply with FP64 energy/virial sums, three
// inverse 3D transforms, gather) on any mesh whose sizes factor into 2, 3
// and 5, with plain kernels sized for meshes of a few thousand to a few
// million points:
//  - spread: one thread per particle, 64-bit fixed-point global atomics
//    (integer sums, so the mesh is bitwise repeatable);
//  - transforms: full complex 3D transforms (the real-input symmetry is not
//    used), one LDS-resident row per block, self-sorting (Stockham) stages
//    of radix 4, 2, 3 and 5 with twiddles from sincospi;
//  - ik multiply: one thread per mesh point of the full spectrum, the energy
//    and virial summed in FP64 per block and reduced in a fixed tree;
//  - gather: one thread per particle, in the caller's order (no sort).
// Mesh layout: x fastest, index (z Ky + y) Kx + x, complex values of the
// plan's precision; the three field spectra follow one another.
#pragma once

#include "pppm_kernels.hpp"

namespace dplr {

// Fixed-point scale of the mixed-radix spread (both precisions): 2^40, so a
// mesh value must stay below 2^23 in charge units.
constexpr double kMixedFixedScale = 1099511627776.0;

// Stencil start s and offset d (weights M_P(d + P-1-t) at s + t) along one
// axis, in FP64 like the tuned path; non-finite inputs map to u = 0.
template <int P>
__device__ __forceinline__ int mixed_stencil(double r, double invh, int K, double& d) {
  const double Kd = (double)K;
  double v = r * invh;
  v = v - Kd * floor(v / Kd);
  if (v >= Kd) v -= Kd;
  if (!(v >= 0.0 && v < Kd)) v = 0.0;
  const double av = v - 0.5 * P;
  const double f = floor(av);
  d = av - f;
  int s = (int)f + 1;
  if (s < 0) s += K;
  if (s >= K) s -= K;
  return s;
}

// One thread per (particle, stencil plane tz): P^2 atomics each.
template <typename T, int P>
__global__ void __launch_bounds__(256) k_mixed_spread(const T* __restrict__ ion_pos, const T* __restrict__ ion_q,
                                                      const T* __restrict__ wc_pos, const T* __restrict__ wc_q,
                                                      int64_t n_ion, int64_t n, double ihx, double ihy, double ihz,
                                                      int Kx, int Ky, int Kz,
                                                      unsigned long long* __restrict__ mesh) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= n * P) return;
  const int64_t i = it / P;
  const int tz = (int)(it - i * P);
  const T* r = (i < n_ion) ? (ion_pos + 3 * i) : (wc_pos + 3 * (i - n_ion));
  const T q = (i < n_ion) ? ion_q[i] : wc_q[i - n_ion];
  double d[3];
  const int sx = mixed_stencil<P>((double)r[0], ihx, Kx, d[0]);
  const int sy = mixed_stencil<P>((double)r[1], ihy, Ky, d[1]);
  const int sz = mixed_stencil<P>((double)r[2], ihz, Kz, d[2]);
  T wx[P], wy[P], wz[P];
  bspline_weights<T, P>((T)d[0], wx);
  bspline_weights<T, P>((T)d[1], wy);
  bspline_weights<T, P>((T)d[2], wz);
  int gx[P];
#pragma unroll
  for (int t = 0; t < P; ++t) gx[t] = (sx + t) % Kx;
  T wzt = wz[0];
#pragma unroll
  for (int t = 1; t < P; ++t) wzt = (tz == t) ? wz[t] : wzt;
  const int gz = (sz + tz) % Kz;
  const T qz = q * wzt;
  for (int ty = 0; ty < P; ++ty) {
    const int gy = (sy + ty) % Ky;
    const T qyz = qz * wy[ty];
    unsigned long long* row = mesh + ((size_t)gz * Ky + gy) * Kx;
#pragma unroll
    for (int tx = 0; tx < P; ++tx) {
      const long long v = llrint((double)(qyz * wx[tx]) * kMixedFixedScale);
      atomicAdd(row + gx[tx], (unsigned long long)v);
    }
  }
}

// Per-particle stencil record, computed once per call: the offsets d (plan
// precision) and the charge in rec, the stencil starts packed as
// s_x | s_y << 10 | s_z << 20 in spk (mesh sizes <= 512).
template <typename T, int P>
__global__ void __launch_bounds__(256) k_mixed_prep(const T* __restrict__ ion_pos, const T* __restrict__ ion_q,
                                                    const T* __restrict__ wc_pos, const T* __restrict__ wc_q,
                                                    int64_t n_ion, int64_t n, double ihx, double ihy, double ihz,
                                                    int Kx, int Ky, int Kz, T4<T>* __restrict__ rec,
                                                    int* __restrict__ spk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T* r = (i < n_ion) ? (ion_pos + 3 * i) : (wc_pos + 3 * (i - n_ion));
  const T q = (i < n_ion) ? ion_q[i] : wc_q[i - n_ion];
  double d[3];
  const int sx = mixed_stencil<P>((double)r[0], ihx, Kx, d[0]);
  const int sy = mixed_stencil<P>((double)r[1], ihy, Ky, d[1]);
  const int sz = mixed_stencil<P>((double)r[2], ihz, Kz, d[2]);
  rec[i] = T4<T>{(T)d[0], (T)d[1], (T)d[2], q};
  spk[i] = sx | (sy << 10) | (sz << 20);
}

// Spread by z planes, for meshes whose xy plane of 64-bit accumulators fits
// in LDS: block z scans the packed stencil starts of every particle, queues
// (in LDS) those whose stencil covers plane z, and once 1024 are queued (or
// at the end) adds their P^2 plane terms with LDS integer atomics, so the
// weight arithmetic runs on full waves.  Integer sums are exact and order
// independent.  Grid (Kz, S) blocks of 1024 threads: block (z, s) takes the
// s-th of S consecutive particle ranges.  With S = 1 the plane is written as
// complex values (imaginary part 0) into the spectrum buffer; with S > 1 as
// 64-bit integers into partial[s][z][y][x], which k_mixed_combine adds.  LDS
// Kx Ky 64-bit words.
template <typename T, int P>
__global__ void __launch_bounds__(1024) k_mixed_spread_plane(const T4<T>* __restrict__ rec,
                                                             const int* __restrict__ spk, int64_t n, int Kx, int Ky,
                                                             int Kz, cpx<T>* __restrict__ spec,
                                                             long long* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned long long pl[];
  __shared__ int queue[2048];
  __shared__ int qn;
  const int z = blockIdx.x;
  const int nxy = Kx * Ky;
  const int S = gridDim.y;
  const int64_t chunk = (n + S - 1) / S;
  const int64_t lo = chunk * blockIdx.y, hi = min(n, lo + chunk);
  for (int e = threadIdx.x; e < nxy; e += blockDim.x) pl[e] = 0ull;
  if (threadIdx.x == 0) qn = 0;
  __syncthreads();
  for (int64_t base = lo; base < hi; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    if (i < hi) {
      int tz = z - (spk[i] >> 20);
      if (tz < 0) tz += Kz;
      if (tz < P) queue[atomicAdd(&qn, 1)] = (int)i;
    }
    __syncthreads();
    const int m = qn;  // < 2048: at most 1023 left over plus 1024 new
    __syncthreads();   // every thread has read qn before the next chunk adds to it
    if (m >= (int)blockDim.x || base + blockDim.x >= hi) {
      for (int k = threadIdx.x; k < m; k += blockDim.x) {
        const int j = queue[k];
        const T4<T> rc = rec[j];
        const int pk = spk[j];
        const int sx = pk & 1023, sy = (pk >> 10) & 1023;
        int tz = z - (pk >> 20);
        if (tz < 0) tz += Kz;
        T wx[P], wy[P], wz[P];
        bspline_weights<T, P>(rc.x, wx);
        bspline_weights<T, P>(rc.y, wy);
        bspline_weights<T, P>(rc.z, wz);
        T wzt = wz[0];
#pragma unroll
        for (int t = 1; t < P; ++t) wzt = (tz == t) ? wz[t] : wzt;
        const T qz = rc.w * wzt;
        int gx[P];
#pragma unroll
        for (int t = 0; t < P; ++t) gx[t] = (sx + t) % Kx;
        for (int ty = 0; ty < P; ++ty) {
          const int gy = (sy + ty) % Ky;
          const T qyz = qz * wy[ty];
          unsigned long long* row = pl + gy * Kx;
#pragma unroll
          for (int tx = 0; tx < P; ++tx) {
            const long long v = llrint((double)(qyz * wx[tx]) * kMixedFixedScale);
            atomicAdd(row + gx[tx], (unsigned long long)v);
          }
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) qn = 0;
      __syncthreads();
    }
  }
  __syncthreads();
  if (S == 1) {
    cpx<T>* out = spec + (int64_t)z * nxy;
    for (int e = threadIdx.x; e < nxy; e += blockDim.x)
      out[e] = cpx<T>{(T)((double)(long long)pl[e] * (1.0 / kMixedFixedScale)), (T)0};
  } else {
    long long* out = partial + ((int64_t)blockIdx.y * Kz + z) * nxy;
    for (int e = threadIdx.x; e < nxy; e += blockDim.x) out[e] = (long long)pl[e];
  }
}

// Sum of the S integer partial meshes of the split plane spread -> complex.
template <typename T>
__global__ void __launch_bounds__(256) k_mixed_combine(const long long* __restrict__ partial, int S, int64_t ntot,
                                                       cpx<T>* __restrict__ spec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  long long v = 0;
  for (int s2 = 0; s2 < S; ++s2) v += partial[(int64_t)s2 * ntot + i];
  spec[i] = cpx<T>{(T)((double)v * (1.0 / kMixedFixedScale)), (T)0};
}

// Fixed point -> complex mesh; clears the accumulators for the next call.
template <typename T>
__global__ void __launch_bounds__(256) k_mixed_unfix(long long* __restrict__ mesh, cpx<T>* __restrict__ out,
                                                     int64_t ntot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  const long long v = mesh[i];
  mesh[i] = 0;
  out[i] = cpx<T>{(T)((double)v * (1.0 / kMixedFixedScale)), (T)0};
}

__device__ __forceinline__ void sincospi_t(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_t(double x, double* s, double* c) { sincospi(x, s, c); }

// exp(sign 2 pi i a / b) for integers 0 <= a < b
template <typename T>
__device__ __forceinline__ cpx<T> unit_root(int a, int b, int sign) {
  T s, c;
  sincospi_t((T)(2 * a) / (T)b, &s, &c);
  return cpx<T>{c, sign > 0 ? s : -s};
}

// One self-sorting stage on C rows of N points held in LDS (row c at c N).
template <typename T, int R>
__device__ __forceinline__ void stockham_stage(const cpx<T>* __restrict__ a, cpx<T>* __restrict__ b, int N, int C,
                                               int p, int sign) {
  const int nb = N / R;
  cpx<T> w[R];
#pragma unroll
  for (int t = 0; t < R; ++t) w[t] = unit_root<T>(t, R, sign);
  for (int it = threadIdx.x; it < C * nb; it += blockDim.x) {
    const int c = it % C, i = it / C;
    const cpx<T>* ar = a + c * N;
    cpx<T>* br = b + c * N;
    const int k = i % p;
    cpx<T> u[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      u[q] = ar[i + q * nb];
      if (q > 0 && k > 0) u[q] = cmul(u[q], unit_root<T>((q * k) % (p * R), p * R, sign));
    }
    const int j = (i - k) * R + k;
#pragma unroll
    for (int s2 = 0; s2 < R; ++s2) {
      cpx<T> v = u[0];
#pragma unroll
      for (int q = 1; q < R; ++q) v = cadd(v, cmul(u[q], w[(q * s2) % R]));
      br[j + s2 * p] = v;
    }
  }
}

// In-place unnormalised DFT of every length-N row along one axis:
// X[k] = sum_n x[n] exp(sign 2 pi i n k / N).  Row r of component c starts
// at c * comp_stride + (r / stride) * stride * N + r % stride and its
// elements are stride apart (stride 1: x rows, Kx: y columns, Kx Ky: z
// columns).  Block b transforms the C consecutive rows b C .. b C + C - 1
// (C divides stride, so they lie side by side in memory and a load of one
// element of each is C contiguous values).  Grid (rows / C, components); LDS
// 2 C N complex values.  With packed != nullptr the real parts are written
// instead to packed[4 e + c] (e the mesh index of the element, c the
// component): the last inverse pass leaves the three fields interleaved for
// the gather.
// Self-sorting stages: with p points already transformed, butterfly i
// (0 <= i < N/R) takes x[i + q N/R], q < R, applies the twiddles
// exp(sign 2 pi i q k / (p R)) with k = i mod p, a length-R DFT, and stores
// to (i - k) R + k + s p, s < R.
template <typename T>
__global__ void __launch_bounds__(256) k_mixed_fft_axis(cpx<T>* __restrict__ data, int N, int64_t stride,
                                                        int64_t comp_stride, int sign, T* __restrict__ packed,
                                                        int C) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<T>* a = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* b = a + C * N;
  const int64_t r0 = (int64_t)blockIdx.x * C;
  // rows r0 .. r0 + C - 1 share r / stride, so row c starts at rbase + c
  const int64_t rbase = (r0 / stride) * stride * N + (r0 % stride);
  cpx<T>* base = data + (int64_t)blockIdx.y * comp_stride + rbase;
  for (int t = threadIdx.x; t < C * N; t += blockDim.x) {
    const int e = t / C, c = t - e * C;
    a[c * N + e] = base[(int64_t)e * stride + c];
  }
  __syncthreads();
  int p = 1, rem = N;
  while (rem > 1) {
    const int R = (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : (rem % 3 == 0) ? 3 : 5;
    switch (R) {
      case 4: stockham_stage<T, 4>(a, b, N, C, p, sign); break;
      case 2: stockham_stage<T, 2>(a, b, N, C, p, sign); break;
      case 3: stockham_stage<T, 3>(a, b, N, C, p, sign); break;
      default: stockham_stage<T, 5>(a, b, N, C, p, sign); break;
    }
    __syncthreads();
    cpx<T>* t = a;
    a = b;
    b = t;
    p *= R;
    rem /= R;
  }
  for (int t = threadIdx.x; t < C * N; t += blockDim.x) {
    const int e = t / C, c = t - e * C;
    const int64_t off = (int64_t)e * stride + c;
    if (packed) packed[4 * (rbase + off) + blockIdx.y] = a[c * N + e].x;
    else base[off] = a[c * N + e];
  }
}

// The same row transform taken as the paper's hardware-offloaded FFT forms it
// in its Mixed-Int32 configuration (Optimization section, int32 quantisation of
// the reduction chains): the N points of a row belong to `nodes` consecutive
// blocks of N / nodes points; each block's partial sum
//   P_b[k] = sum_{n in block b} x[n] exp(sign 2 pi i n k / N)
// is scaled by `scale`, rounded to the nearest integer and clamped to the
// int32 range (real and imaginary parts apart), the integers are summed over
// the blocks exactly and the sum is divided by `scale`.  Direct sums, O(N)
// per output.  Grid (rows, components); LDS N complex values; packed as in
// k_mixed_fft_axis.
template <typename T>
__global__ void __launch_bounds__(256) k_mixed_dft_q32(cpx<T>* __restrict__ data, int N, int64_t stride,
                                                       int64_t comp_stride, int sign, int nodes, double scale,
                                                       T* __restrict__ packed,
                                                       unsigned long long* __restrict__ clamped) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<T>* a = reinterpret_cast<cpx<T>*>(smem);
  const int64_t r = blockIdx.x;
  const int64_t rbase = (r / stride) * stride * N + (r % stride);
  cpx<T>* row = data + (int64_t)blockIdx.y * comp_stride + rbase;
  for (int e = threadIdx.x; e < N; e += blockDim.x) a[e] = row[(int64_t)e * stride];
  __syncthreads();
  const int seg = N / nodes;
  unsigned nclamp = 0;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    long long acc_re = 0, acc_im = 0;
    for (int bk = 0; bk < nodes; ++bk) {
      cpx<T> s = {(T)0, (T)0};
      for (int n = bk * seg; n < (bk + 1) * seg; ++n)
        s = cadd(s, cmul(a[n], unit_root<T>((int)(((int64_t)n * k) % N), N, sign)));
      // the partial value (in the plan's precision) scaled, rounded to the
      // nearest integer and clamped to int32 in FP64, so that the rounding is
      // to the integer nearest the partial value in FP32 plans too
      const double vr = rint((double)s.x * scale), vi = rint((double)s.y * scale);
      const double cr = fmin(fmax(vr, -2147483648.0), 2147483647.0);
      const double ci = fmin(fmax(vi, -2147483648.0), 2147483647.0);
      nclamp += (cr != vr) + (ci != vi);
      acc_re += (long long)cr;
      acc_im += (long long)ci;
    }
    const cpx<T> v = {(T)((double)acc_re / scale), (T)((double)acc_im / scale)};
    if (packed) packed[4 * (rbase + (int64_t)k * stride) + blockIdx.y] = v.x;
    else row[(int64_t)k * stride] = v;
  }
  // partial values that hit the int32 limits (saturated), counted for the caller
  if (clamped && nclamp) atomicAdd(clamped, (unsigned long long)nclamp);
}

// Energy/virial summands and the ik field spectra over the full spectrum:
//   E^_a(n) = -i fmul k'_a G(n) Q^(n), k'_a = 0 at the Nyquist index of an even K_a
//   (fmul = 1, or k_e / V when the inverse transforms are quantised);
//   per block: sum G |Q^|^2 and sum G |Q^|^2 [delta_ab - 2 (1 + k^2/(4 beta^2)) k_a k_b / k^2]
// in partials[block * 8 + c], c = E, xx, yy, zz, xy, xz, yz.
// G is the octant table [Kx/2+1][Ky/2+1][Kz/2+1] over |n_a|.
template <typename T>
__global__ void __launch_bounds__(256) k_mixed_poisson(const cpx<T>* __restrict__ Qh, cpx<T>* __restrict__ Ef,
                                                       const double* __restrict__ G, int Kx, int Ky, int Kz,
                                                       PoissonConsts pc, double fmul,
                                                       double* __restrict__ partials) {
  __shared__ double red[7][256];
  const int64_t ntot = (int64_t)Kx * Ky * Kz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  if (i < ntot) {
    const int ix = (int)(i % Kx);
    const int iy = (int)((i / Kx) % Ky);
    const int iz = (int)(i / ((int64_t)Kx * Ky));
    const int idx[3] = {ix, iy, iz};
    const int K[3] = {Kx, Ky, Kz};
    int an[3];
    double k[3], kd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int nn = (idx[a] <= K[a] / 2) ? idx[a] : idx[a] - K[a];
      an[a] = nn < 0 ? -nn : nn;
      k[a] = pc.two_pi_over_L[a] * (double)nn;
      kd[a] = ((K[a] & 1) == 0 && idx[a] == K[a] / 2) ? 0.0 : k[a];
    }
    const double g = G[((size_t)an[0] * (Ky / 2 + 1) + an[1]) * (Kz / 2 + 1) + an[2]];
    const cpx<T> qv = Qh[i];
    const double qx = (double)qv.x, qy = (double)qv.y;
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (k2 > 0.0) {
      const double e = g * (qx * qx + qy * qy);
      const double c = 2.0 * (1.0 + k2 * pc.inv_4beta2) / k2;
      acc[0] = e;
      acc[1] = e * (1.0 - c * k[0] * k[0]);
      acc[2] = e * (1.0 - c * k[1] * k[1]);
      acc[3] = e * (1.0 - c * k[2] * k[2]);
      acc[4] = -e * c * k[0] * k[1];
      acc[5] = -e * c * k[0] * k[2];
      acc[6] = -e * c * k[1] * k[2];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T f = (T)(fmul * (kd[a] * g));  // -i f (x + i y) = f y - i f x
      Ef[(int64_t)a * ntot + i] = cpx<T>{f * qv.y, -f * qv.x};
    }
  }
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 7; ++c) red[c][t] = acc[c];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int c = 0; c < 7; ++c) red[c][t] += red[c][t + h];
    }
    __syncthreads();
  }
  if (t < 7) partials[(size_t)blockIdx.x * 8 + t] = red[t][0];
}

// E = pre * sum of the block partials (and the virial likewise), fixed tree.
__global__ void __launch_bounds__(256) k_mixed_reduce(const double* __restrict__ partials, int nblk, double pre,
                                                      double* __restrict__ energy, double* __restrict__ virial) {
  __shared__ double red[7 * 256];
  reduce_partials(partials, nblk, pre, energy, virial, red);
}

// F_ja = (k_e q_j / V) sum_g W(u_j - g) E_a(g), caller's order, from the
// interleaved real fields (x, y, z, unused) the last inverse pass wrote.
// Block 0 also reduces the energy/virial partials (as k_mixed_reduce).  Block of
// 256 threads: 256 / P particles, one thread per (particle, stencil plane tz);
// the P plane sums of a particle are added in tz order (deterministic).
template <typename T, int P>
__global__ void __launch_bounds__(256) k_mixed_gather(const T* __restrict__ ion_pos, const T* __restrict__ ion_q,
                                                      const T* __restrict__ wc_pos, const T* __restrict__ wc_q,
                                                      int64_t n_ion, int64_t n, double ihx, double ihy, double ihz,
                                                      int Kx, int Ky, int Kz, const T4<T>* __restrict__ Ef,
                                                      T* __restrict__ ion_f, T* __restrict__ wc_f, T fscale,
                                                      int accumulate, const double* __restrict__ partials,
                                                      int nblk, double pre, double* __restrict__ energy,
                                                      double* __restrict__ virial) {
  __shared__ T part[256][3];
  if (blockIdx.x == 0) {
    // block 0 also finishes the energy and virial (the ik multiply's block
    // partials are complete: that kernel ran before this one on the stream)
    __shared__ double red[7 * 256];
    reduce_partials(partials, nblk, pre, energy, virial, red);
  }
  constexpr int PPB = 256 / P;
  const int jl = threadIdx.x / P, tz = threadIdx.x % P;
  const int64_t i = (int64_t)blockIdx.x * PPB + jl;
  const bool on = jl < PPB && i < n;
  T f0 = 0, f1 = 0, f2 = 0;
  if (on) {
  const T* r = (i < n_ion) ? (ion_pos + 3 * i) : (wc_pos + 3 * (i - n_ion));
  double d[3];
  const int sx = mixed_stencil<P>((double)r[0], ihx, Kx, d[0]);
  const int sy = mixed_stencil<P>((double)r[1], ihy, Ky, d[1]);
  const int sz = mixed_stencil<P>((double)r[2], ihz, Kz, d[2]);
  T wx[P], wy[P], wz[P];
  bspline_weights<T, P>((T)d[0], wx);
  bspline_weights<T, P>((T)d[1], wy);
  bspline_weights<T, P>((T)d[2], wz);
  int gx[P];
#pragma unroll
  for (int t = 0; t < P; ++t) gx[t] = (sx + t) % Kx;
  T wzt = wz[0];
#pragma unroll
  for (int t = 1; t < P; ++t) wzt = (tz == t) ? wz[t] : wzt;
  const int gz = (sz + tz) % Kz;
#pragma unroll
  for (int ty = 0; ty < P; ++ty) {
    const int gy = (sy + ty) % Ky;
    const T wyz = wzt * wy[ty];
    const int64_t rb = ((int64_t)gz * Ky + gy) * Kx;
#pragma unroll
    for (int tx = 0; tx < P; ++tx) {
      const T4<T> v = Ef[rb + gx[tx]];
      const T w = wyz * wx[tx];
      f0 += w * v.x;
      f1 += w * v.y;
      f2 += w * v.z;
    }
  }
  }
  part[threadIdx.x][0] = f0;
  part[threadIdx.x][1] = f1;
  part[threadIdx.x][2] = f2;
  __syncthreads();
  if (!on || tz != 0) return;
  T g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
  for (int t = 0; t < P; ++t) {
    g0 += part[threadIdx.x + t][0];
    g1 += part[threadIdx.x + t][1];
    g2 += part[threadIdx.x + t][2];
  }
  const T q = (i < n_ion) ? ion_q[i] : wc_q[i - n_ion];
  const T s = fscale * q;
  T* out = (i < n_ion) ? (ion_f + 3 * i) : (wc_f + 3 * (i - n_ion));
  const T v[3] = {s * g0, s * g1, s * g2};
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = accumulate ? out[a] + v[a] : v[a];
}

}  // namespace dplr
