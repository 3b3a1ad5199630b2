// PPPM-ik on meshes whose sizes are not all powers of two.
//
// The paper runs its precision study on small per-node grids such as
// 8x12x8, 10x15x10 and 12x18x12 (Results, accuracy of the precision
// variants), which the plane/pencil kernels cannot take: those assume
// power-of-two rows for their register transforms, bins and index masks.
// This path computes the same steps as the tuned one (spread, forward 3D
// transform, optimal-G ik multiply with FP64 energy/virial sums, inverse 3D
// transforms of the field, gather) on any mesh whose sizes factor into 2, 3
// and 5.  Two forms:
//  - fused (an xy plane of complex values fits in LDS, no int32 transforms):
//    three passes over the mesh, the layout of the power-of-two path.  The
//    plane spread (particles counting-sorted by split, stencil-start plane
//    and row group; 64-bit fixed-point LDS atomics, so the mesh is bitwise
//    repeatable) is followed by the x and y transforms in LDS; one pass per
//    group of (x, y) columns adds the split spectra and does the z transform,
//    the ik multiply and the inverse z transforms of two complex fields,
//    Ex^ + i Ey^ and Ez^ (the fields are real, so one complex inverse
//    transform carries two of them); one pass per (plane, field) does the
//    inverse y and x transforms.  The row transforms are in-place
//    self-sorting stages of radix 2, 3, 4, 5 and composites up to 12;
//  - per axis (larger planes, or the int32 transforms): full complex 3D
//    transforms with one pass per axis and component (Stockham stages of
//    radix 4, 2, 3, 5 between two LDS buffers, or the quantised direct sums),
//    the ik multiply as its own pass over the full spectrum, and the plane
//    spread (or global 64-bit atomics when even the integer plane does not
//    fit in LDS).
// Both gather with P lanes per particle (one per stencil column), in the
// sorted order when the spread sorted the particles.
// Mesh layout: x fastest, index (z Ky + y) Kx + x, complex values of the
// plan's precision.
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

// Spread by z planes, for meshes whose xy plane of 64-bit accumulators fits
// in LDS.  The particles are counting-sorted by (split, stencil-start plane)
// with the plane kernels' sort (k_bin_hist / k_bin_colscan / k_bin_place, one
// bin per split and plane), which leaves per particle the offsets d and the
// charge (rec) and the packed stencil starts s_x | s_y << 10 | s_z << 20
// (spk).  Block (z, s) walks only the particles of split s whose
// stencil-start plane is one of z-P+1 .. z (at most two contiguous ranges of
// the sorted records) and adds their P^2 terms on plane z with LDS integer
// atomics (scale 2^40: exact, order-independent sums).  With one split the
// plane is written as complex values (imaginary part 0) into the spectrum
// buffer; with S splits as 64-bit integers into partial[s][z][y][x], which
// k_mixed_combine adds.  LDS Kx Ky 64-bit words.
template <typename T, int P>
__global__ void __launch_bounds__(1024) k_mixed_spread_sorted(const T4<T>* __restrict__ rec,
                                                              const int* __restrict__ spk,
                                                              const int* __restrict__ bin_start, Geo g,
                                                              cpx<T>* __restrict__ spec,
                                                              long long* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned long long pl[];
  __shared__ Ranges R;
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  const int z = blockIdx.x, split = blockIdx.y;
  const int nxy = Kx * Ky;
  const RangeLoad rl = range_load(bin_start, g, split, z - (P - 1), P, 0, g.NQ);
  for (int e = threadIdx.x; e < nxy; e += blockDim.x) pl[e] = 0ull;
  ranges_finish(R, rl);  // contains barriers
  const int total = R.pre[R.n];
  for (int v = threadIdx.x; v < total; v += blockDim.x) {
    const int j = range_index2(R, v);
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
    for (int t = 0; t < P; ++t) {
      gx[t] = sx + t;
      if (gx[t] >= Kx) gx[t] -= Kx;
    }
#pragma unroll
    for (int ty = 0; ty < P; ++ty) {
      int gy = sy + ty;
      if (gy >= Ky) gy -= Ky;
      const T qyz = qz * wy[ty];
      unsigned long long* row = pl + gy * Kx;
#pragma unroll
      for (int tx = 0; tx < P; ++tx) {
        const long long v2 = llrint((double)(qyz * wx[tx]) * kMixedFixedScale);
        atomicAdd(row + gx[tx], (unsigned long long)v2);
      }
    }
  }
  __syncthreads();
  if (gridDim.y == 1) {
    cpx<T>* out = spec + (int64_t)z * nxy;
    for (int e = threadIdx.x; e < nxy; e += blockDim.x)
      out[e] = cpx<T>{(T)((double)(long long)pl[e] * (1.0 / kMixedFixedScale)), (T)0};
  } else {
    long long* out = partial + ((int64_t)split * Kz + z) * nxy;
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
// tw holds exp(sign 2 pi i m / N), m < N (the row's roots of unity, computed
// once per block), so the stage twiddle exp(sign 2 pi i q k / (p R)) is
// tw[q k N / (p R)].
template <typename T, int R>
__device__ __forceinline__ void stockham_stage(const cpx<T>* __restrict__ a, cpx<T>* __restrict__ b, int N, int C,
                                               int p, const cpx<T>* __restrict__ tw) {
  const int nb = N / R;
  const int tstep = N / (p * R);
  cpx<T> w[R];
#pragma unroll
  for (int t = 0; t < R; ++t) w[t] = tw[t * (N / R)];
  for (int it = threadIdx.x; it < C * nb; it += blockDim.x) {
    const int c = it % C, i = it / C;
    const cpx<T>* ar = a + c * N;
    cpx<T>* br = b + c * N;
    const int k = i % p;
    cpx<T> u[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      u[q] = ar[i + q * nb];
      if (q > 0 && k > 0) u[q] = cmul(u[q], tw[q * k * tstep]);
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
// (2 C + 1) N complex values (two row buffers and the root-of-unity table).  With packed != nullptr the real parts are written
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
  cpx<T>* tw = b + C * N;  // the N roots of unity of this row length
  for (int m = threadIdx.x; m < N; m += blockDim.x) tw[m] = unit_root<T>(m, N, sign);
  const int64_t r0 = (int64_t)blockIdx.x * C;
  // rows r0 .. r0 + C - 1: along y and z they share r / stride and lie side by
  // side (row c starts at rbase + c, element e at e stride + c); along x
  // (stride 1) they follow one another (element e of row c at c N + e).  In
  // both cases consecutive threads touch consecutive values.
  const int64_t rbase = (r0 / stride) * stride * N + (r0 % stride);
  cpx<T>* base = data + (int64_t)blockIdx.y * comp_stride + rbase;
  const bool xrows = stride == 1;
  auto off_of = [&](int t, int& c, int& e) -> int64_t {
    if (xrows) {
      c = t / N;
      e = t - c * N;
      return t;
    }
    e = t / C;
    c = t - e * C;
    return (int64_t)e * stride + c;
  };
  for (int t = threadIdx.x; t < C * N; t += blockDim.x) {
    int c, e;
    const int64_t off = off_of(t, c, e);
    a[c * N + e] = base[off];
  }
  __syncthreads();
  int p = 1, rem = N;
  while (rem > 1) {
    const int R = (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : (rem % 3 == 0) ? 3 : 5;
    switch (R) {
      case 4: stockham_stage<T, 4>(a, b, N, C, p, tw); break;
      case 2: stockham_stage<T, 2>(a, b, N, C, p, tw); break;
      case 3: stockham_stage<T, 3>(a, b, N, C, p, tw); break;
      default: stockham_stage<T, 5>(a, b, N, C, p, tw); break;
    }
    __syncthreads();
    cpx<T>* t = a;
    a = b;
    b = t;
    p *= R;
    rem /= R;
  }
  for (int t = threadIdx.x; t < C * N; t += blockDim.x) {
    int c, e;
    const int64_t off = off_of(t, c, e);
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

// ---------------------------------------------------------------------------
// Fused form, for plans whose xy plane of complex values fits in LDS: three
// passes over the mesh instead of eight (the layout of the power-of-two path):
//  - k_mixed_spread_xy: the plane spread, then the x and y transforms of the
//    plane in LDS; writes one spectrum plane per (plane, split);
//  - k_mixed_fftz_poisson: per group of C (x, y) columns, the sum of the
//    split spectra, the z transform, the ik multiply with the FP64 energy and
//    virial sums, and the inverse z transforms of two complex fields:
//    Ex^ + i Ey^ (whose inverse is Ex + i Ey, both fields being real) and Ez^;
//  - k_mixed_ifft_xy: per (plane, field), the inverse y and x transforms in
//    LDS; writes the real fields interleaved for the gather.
// ---------------------------------------------------------------------------

// Most points of a plane the fused kernels hold (128 KiB of complex values;
// the bound also keeps a stage's butterflies within the registers of a
// 1024-thread block).
template <typename T>
struct FusedPlane {
  static constexpr int kMaxPts = (128 * 1024) / (int)sizeof(cpx<T>);
};
constexpr int kFusedZMaxPts = 2048;  // C Kz bound of k_mixed_fftz_poisson (one field)
constexpr int kFusedZThreads = 512;

// floor(x / d) for 0 <= x, d < 2^23 from the float reciprocal inv = 1 / d:
// the estimate is off by at most one either way and is corrected.
__device__ __forceinline__ int qdiv(int x, int d, float inv) {
  int q = (int)((float)x * inv);
  const int r = x - q * d;
  if (r < 0) --q;
  else if (r >= d) ++q;
  return q;
}

// Radices of the in-place stages: 2, 3, 4 and 5 in closed form or from the
// root table, and the composites R = R1 R2 below, computed as R2 transforms
// of length R1, the twiddles w_R^(n2 k1), then R1 transforms of length R2
// (Cooley-Tukey with n = R2 n1 + n2, k = k1 + R1 k2).
template <int R> struct RadixSplit { static constexpr int R1 = 1, R2 = 1; };
template <> struct RadixSplit<16> { static constexpr int R1 = 4, R2 = 4; };
template <> struct RadixSplit<12> { static constexpr int R1 = 4, R2 = 3; };
template <> struct RadixSplit<10> { static constexpr int R1 = 5, R2 = 2; };
template <> struct RadixSplit<8> { static constexpr int R1 = 4, R2 = 2; };
template <> struct RadixSplit<6> { static constexpr int R1 = 3, R2 = 2; };

// Length-R DFT of u in place, X[s] = sum_q u[q] w^(q s) with w = exp(-+2 pi i / R)
// (INV: the + sign).  tw holds the N roots of unity of the transform's sign
// (R divides N), so w^m = tw[m N / R].
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_radix(cpx<T>* u, const cpx<T>* __restrict__ tw, int N) {
  if constexpr (R == 2) {
    const cpx<T> a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  } else if constexpr (R == 4) {
    dft4<T, INV>(u[0], u[1], u[2], u[3]);
  } else if constexpr (R == 3) {
    // w = -1/2 -+ i sqrt(3)/2:  X1, X2 = u0 - (u1 + u2)/2 -+ i sqrt(3)/2 (u1 - u2)
    const T h = (T)0.86602540378443864676;
    const cpx<T> sm = cadd(u[1], u[2]), df = csub(u[1], u[2]);
    const cpx<T> m = {u[0].x - (T)0.5 * sm.x, u[0].y - (T)0.5 * sm.y};
    const cpx<T> t = INV ? cpx<T>{-h * df.y, h * df.x} : cpx<T>{h * df.y, -h * df.x};
    u[0] = cadd(u[0], sm);
    u[1] = cadd(m, t);
    u[2] = csub(m, t);
  } else if constexpr (R == 5) {
    const int st = N / 5;
    cpx<T> w[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) w[t] = tw[t * st];
    cpx<T> v[5];
#pragma unroll
    for (int s2 = 0; s2 < 5; ++s2) {
      v[s2] = u[0];
#pragma unroll
      for (int q = 1; q < 5; ++q) v[s2] = cadd(v[s2], cmul(u[q], w[(q * s2) % 5]));
    }
#pragma unroll
    for (int s2 = 0; s2 < 5; ++s2) u[s2] = v[s2];
  } else {
    constexpr int R1 = RadixSplit<R>::R1, R2 = RadixSplit<R>::R2;
    static_assert(R1 * R2 == R, "radix without a split");
    const int st = N / R;
    cpx<T> y[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = u[R2 * n1 + n2];
      dft_radix<T, R1, INV>(y[n2], tw, N);
#pragma unroll
      for (int k1 = 1; k1 < R1; ++k1)
        if (n2 > 0) y[n2][k1] = cmul(y[n2][k1], tw[((n2 * k1) % R) * st]);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cpx<T> t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2][k1];
      dft_radix<T, R2, INV>(t, tw, N);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) u[k1 + R1 * k2] = t[k2];
    }
  }
}

// The butterflies (r, i) of one thread in a stage over nrows rows of nb
// butterflies: threadIdx.x, threadIdx.x + blockDim.x, ... of the flattened
// index (rfast: r + nrows i, otherwise i + nb r), stepped without divisions.
struct BflyWalk {
  int r, i, dr, di;
  __device__ __forceinline__ BflyWalk(int nrows, int nb, bool rfast) {
    const int t = threadIdx.x, B = blockDim.x;
    if (rfast) {
      const float inv = 1.0f / (float)nrows;
      i = qdiv(t, nrows, inv);
      r = t - i * nrows;
      di = qdiv(B, nrows, inv);
      dr = B - di * nrows;
    } else {
      const float inv = 1.0f / (float)nb;
      r = qdiv(t, nb, inv);
      i = t - r * nb;
      dr = qdiv(B, nb, inv);
      di = B - dr * nb;
    }
  }
  __device__ __forceinline__ void next(int nrows, int nb, bool rfast) {
    r += dr;
    i += di;
    if (rfast) {
      if (r >= nrows) { r -= nrows; ++i; }
    } else if (i >= nb) {
      i -= nb;
      ++r;
    }
  }
};

// One self-sorting stage, in place, over `nrows` rows of N points in LDS
// (point e of row r at buf[r rs + e es]).  The butterflies are those of
// stockham_stage; each thread first loads the inputs of its butterflies (at
// most MAXB of them) into registers, the block waits, and the outputs are
// written over the same buffer, so no second buffer is needed.  rfast:
// consecutive threads take consecutive rows (rows side by side in memory),
// otherwise consecutive butterflies of a row.  tw: the N roots of unity of
// the transform's sign.  Every thread of the block calls it; it ends with a
// barrier.
template <typename T, int R, int MAXB, bool INV>
__device__ __forceinline__ void stage_inplace(cpx<T>* buf, int N, int nrows, int rs, int es, bool rfast, int p,
                                              const cpx<T>* __restrict__ tw) {
  const int nb = N / R;
  const int tstep = nb / p;  // N / (p R)
  const int total = nrows * nb;
  const float invp = 1.0f / (float)p;
  cpx<T> u[MAXB][R];
  BflyWalk wk(nrows, nb, rfast);
#pragma unroll
  for (int j = 0; j < MAXB; ++j) {
    if ((int)threadIdx.x + j * (int)blockDim.x < total) {
      const int k = wk.i - qdiv(wk.i, p, invp) * p;
      const cpx<T>* row = buf + wk.r * rs;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        cpx<T> v = row[(wk.i + q * nb) * es];
        if (q > 0 && k > 0) v = cmul(v, tw[q * k * tstep]);
        u[j][q] = v;
      }
    }
    wk.next(nrows, nb, rfast);
  }
  __syncthreads();
  BflyWalk wo(nrows, nb, rfast);
#pragma unroll
  for (int j = 0; j < MAXB; ++j) {
    if ((int)threadIdx.x + j * (int)blockDim.x < total) {
      const int k = wo.i - qdiv(wo.i, p, invp) * p;
      const int jj = (wo.i - k) * R + k;
      cpx<T>* row = buf + wo.r * rs;
      dft_radix<T, R, INV>(u[j], tw, N);
#pragma unroll
      for (int s2 = 0; s2 < R; ++s2) row[(jj + s2 * p) * es] = u[j][s2];
    }
    wo.next(nrows, nb, rfast);
  }
  __syncthreads();
}

// In-place unnormalised DFT of every row, X[k] = sum_n x[n] exp(-+2 pi i n k
// / N) (INV: +), stages of radix 4, 2, 3, 5 in that order of preference; tw
// holds the N roots of unity of that sign.  MAXPTS bounds nrows N and BLOCK
// is the block size, so no thread has more than MAXPTS / (R BLOCK)
// butterflies in a stage.
#ifndef DPLR_MIXED_MAX_RADIX
#define DPLR_MIXED_MAX_RADIX 12
#endif
// Radix of the next stage for rem points still to split: the largest of 16,
// 12, 10, 8, 6, 5, 4, 3, 2 (at most DPLR_MIXED_MAX_RADIX: radix 16 needs more
// registers than a 1024-thread block has without spilling) that divides rem.
__device__ __forceinline__ int pick_radix(int rem) {
  constexpr int kR[9] = {16, 12, 10, 8, 6, 5, 4, 3, 2};
#pragma unroll
  for (int j = 0; j < 9; ++j)
    if (kR[j] <= DPLR_MIXED_MAX_RADIX && rem % kR[j] == 0) return kR[j];
  return rem;  // not reached for 2-3-5 sizes
}

template <typename T, int BLOCK, int MAXPTS, bool INV>
__device__ __forceinline__ void lds_dft_rows(cpx<T>* buf, int N, int nrows, int rs, int es, bool rfast,
                                             const cpx<T>* __restrict__ tw) {
  int p = 1, rem = N;
  while (rem > 1) {
    const int R = pick_radix(rem);
#define DPLR_STAGE(RR)                                                                              \
  case RR:                                                                                          \
    if constexpr (RR <= DPLR_MIXED_MAX_RADIX)                                                       \
      stage_inplace<T, RR, (MAXPTS / RR + BLOCK - 1) / BLOCK, INV>(buf, N, nrows, rs, es, rfast, p, tw); \
    break;
    switch (R) {
      DPLR_STAGE(16) DPLR_STAGE(12) DPLR_STAGE(10) DPLR_STAGE(8) DPLR_STAGE(6) DPLR_STAGE(5) DPLR_STAGE(4)
      DPLR_STAGE(3) DPLR_STAGE(2)
      default: break;
    }
#undef DPLR_STAGE
    p *= R;
    rem /= R;
  }
}

// Plane spread (as k_mixed_spread_sorted) followed by the forward x and y
// transforms of the plane in LDS.  Block (z, s) writes the spectrum of its
// partial plane to part[s][z][y][x] (complex); k_mixed_fftz_poisson adds the
// S partial spectra in split order.  FP32 plans take the fixed-point scale of
// the tuned spread, 2^(30 - e) for charges below 2^e (the largest charge from
// the sort's per-chunk maxima), so each term converts in single precision
// (FP64 plans: 2^40).  The integer plane becomes complex in place: every
// thread holds its values in registers across a barrier.  Block of 1024
// threads; LDS (Kx Ky + Kx + Ky) complex values.
template <typename T, int P>
__global__ void __launch_bounds__(1024) k_mixed_spread_xy(const T4<T>* __restrict__ rec,
                                                          const int* __restrict__ spk,
                                                          const int* __restrict__ bin_start, Geo g,
                                                          const unsigned* __restrict__ qmax_part, int nqpart,
                                                          cpx<T>* __restrict__ part) {
  constexpr int kMax = FusedPlane<T>::kMaxPts;
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* pl = reinterpret_cast<unsigned long long*>(smem);
  cpx<T>* cp = reinterpret_cast<cpx<T>*>(smem);
  __shared__ Ranges R;
  __shared__ unsigned qm_s;
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  const int z = blockIdx.x, split = blockIdx.y;
  const int nxy = Kx * Ky;
  cpx<T>* twx = cp + nxy;  // beyond the integer plane as well
  cpx<T>* twy = twx + Kx;
  const RangeLoad rl = range_load(bin_start, g, split, z - (P - 1), P, 0, g.NQ);
  unsigned qb = 0u;
  if constexpr (sizeof(T) == 4) {
    for (int i = threadIdx.x; i < nqpart; i += blockDim.x) qb = max(qb, qmax_part[i]);
  }
  if (threadIdx.x == 0) qm_s = 0u;
  for (int e = threadIdx.x; e < nxy; e += blockDim.x) pl[e] = 0ull;
  for (int m = threadIdx.x; m < Kx; m += blockDim.x) twx[m] = unit_root<T>(m, Kx, -1);
  for (int m = threadIdx.x; m < Ky; m += blockDim.x) twy[m] = unit_root<T>(m, Ky, -1);
  if constexpr (sizeof(T) == 4) {
    qb = wave_max_u32(qb);
    __syncthreads();  // qm_s initialised
    if ((threadIdx.x & 63) == 0 && qb) atomicMax(&qm_s, qb);
  }
  ranges_finish(R, rl);  // contains barriers (also publishes qm_s)
  T scale;
  if constexpr (sizeof(T) == 4) scale = fixed_scale_fp32(qm_s);
  else scale = (T)kMixedFixedScale;
  const int total = R.pre[R.n];
  for (int v = threadIdx.x; v < total; v += blockDim.x) {
    const int j = range_index2(R, v);
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
    const T qz = rc.w * scale * wzt;
    int gx[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
      gx[t] = sx + t;
      if (gx[t] >= Kx) gx[t] -= Kx;
    }
#pragma unroll
    for (int ty = 0; ty < P; ++ty) {
      int gy = sy + ty;
      if (gy >= Ky) gy -= Ky;
      const T qyz = qz * wy[ty];
      unsigned long long* row = pl + gy * Kx;
#pragma unroll
      for (int tx = 0; tx < P; ++tx) atomicAdd(row + gx[tx], (unsigned long long)to_fixed<T>(qyz * wx[tx]));
    }
  }
  __syncthreads();
  const double inv_scale = 1.0 / (double)scale;
  constexpr int KV = (kMax + 1023) / 1024;
  long long held[KV];
#pragma unroll
  for (int j = 0; j < KV; ++j) {
    const int e = threadIdx.x + j * 1024;
    held[j] = e < nxy ? (long long)pl[e] : 0;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < KV; ++j) {
    const int e = threadIdx.x + j * 1024;
    if (e < nxy) cp[e] = cpx<T>{(T)((double)held[j] * inv_scale), (T)0};
  }
  __syncthreads();
  lds_dft_rows<T, 1024, kMax, false>(cp, Kx, Ky, Kx, 1, false, twx);  // x rows
  lds_dft_rows<T, 1024, kMax, false>(cp, Ky, Kx, 1, Kx, true, twy);   // y columns
  cpx<T>* out = part + ((int64_t)split * Kz + z) * nxy;
  for (int e = threadIdx.x; e < nxy; e += blockDim.x) out[e] = cp[e];
}

// Block b: the C columns (x, y) = b C .. b C + C - 1 (flattened x + Kx y) of
// every z.  LDS: the C columns of the spectrum and C columns of the second
// field side by side (point e of column c at e 2C + c; Ez^ in c < C, Ex^ + i
// Ey^ in c >= C), then the Kz roots of unity.  Energy/virial summands and the
// field spectra as k_mixed_poisson; per block FP64 sums in partials[b 8 + c].
// Writes fxy = Ex + i Ey and fz = Ez (z transformed back, x and y not).
template <typename T>
__global__ void __launch_bounds__(kFusedZThreads) k_mixed_fftz_poisson(
    const cpx<T>* __restrict__ part, int S, cpx<T>* __restrict__ fxy, cpx<T>* __restrict__ fz,
    const double* __restrict__ G, int Kx, int Ky, int Kz, int C, PoissonConsts pc, double fmul,
    double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double wred[7][kFusedZThreads / 64];
  cpx<T>* a = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* tw = a + 2 * C * Kz;
  const int nxy = Kx * Ky;
  const int64_t ntot = (int64_t)nxy * Kz;
  const int col0 = blockIdx.x * C;
  const int C2 = 2 * C;
  const int lc = __ffs(C) - 1;  // C is a power of two
  for (int m = threadIdx.x; m < Kz; m += blockDim.x) tw[m] = unit_root<T>(m, Kz, -1);
  for (int t = threadIdx.x; t < C * Kz; t += blockDim.x) {
    const int e = t >> lc, c = t & (C - 1);
    const int64_t gi = col0 + c + (int64_t)e * nxy;
    cpx<T> v = part[gi];
    for (int s2 = 1; s2 < S; ++s2) v = cadd(v, part[(int64_t)s2 * ntot + gi]);
    a[e * C2 + c] = v;
  }
  __syncthreads();
  lds_dft_rows<T, kFusedZThreads, kFusedZMaxPts, false>(a, Kz, C, 1, C2, true, tw);
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const int K[3] = {Kx, Ky, Kz};
  // this thread's columns: c = t mod C is the same on every pass of the loop
  // below when C divides the block size
  for (int t = threadIdx.x; t < C * Kz; t += blockDim.x) {
    const int iz = t >> lc, c = t & (C - 1);
    const int col = col0 + c;
    const int iy = col / Kx;
    const int idx[3] = {col - iy * Kx, iy, iz};
    int an[3];
    double k[3], f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int nn = (idx[d] <= K[d] / 2) ? idx[d] : idx[d] - K[d];
      an[d] = nn < 0 ? -nn : nn;
      k[d] = pc.two_pi_over_L[d] * (double)nn;
      f[d] = ((K[d] & 1) == 0 && idx[d] == K[d] / 2) ? 0.0 : k[d];
    }
    const double gv = G[((size_t)an[0] * (Ky / 2 + 1) + an[1]) * (Kz / 2 + 1) + an[2]];
    const cpx<T> qv = a[iz * C2 + c];
    const double qx = (double)qv.x, qy = (double)qv.y;
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (k2 > 0.0) {
      const double e = gv * (qx * qx + qy * qy);
      const double cc = 2.0 * (1.0 + k2 * pc.inv_4beta2) / k2;
      acc[0] += e;
      acc[1] += e * (1.0 - cc * k[0] * k[0]);
      acc[2] += e * (1.0 - cc * k[1] * k[1]);
      acc[3] += e * (1.0 - cc * k[2] * k[2]);
      acc[4] -= e * cc * k[0] * k[1];
      acc[5] -= e * cc * k[0] * k[2];
      acc[6] -= e * cc * k[1] * k[2];
    }
    // E_a^ = -i f_a Q^ with f_a = fmul k'_a G:  E_z^ = (f_z qy, -f_z qx) and
    // E_x^ + i E_y^ = (f_x qy + f_y qx, f_y qy - f_x qx)
    const T fx = (T)(fmul * (f[0] * gv)), fy = (T)(fmul * (f[1] * gv)), fzz = (T)(fmul * (f[2] * gv));
    a[iz * C2 + c] = cpx<T>{fzz * qv.y, -fzz * qv.x};
    a[iz * C2 + C + c] = cpx<T>{fx * qv.y + fy * qv.x, fy * qv.y - fx * qv.x};
  }
  __syncthreads();
  for (int m = threadIdx.x; m < Kz; m += blockDim.x) tw[m] = unit_root<T>(m, Kz, +1);
  __syncthreads();
  lds_dft_rows<T, kFusedZThreads, 2 * kFusedZMaxPts, true>(a, Kz, C2, 1, C2, true, tw);
  for (int t = threadIdx.x; t < C2 * Kz; t += blockDim.x) {
    const int e = t >> (lc + 1), c = t & (C2 - 1);
    const int64_t gi = col0 + (c < C ? c : c - C) + (int64_t)e * nxy;
    (c < C ? fz : fxy)[gi] = a[t];
  }
  // block sums: a fixed xor tree within each wave, then the waves in order
  const int th = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    double v = acc[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((th & 63) == 0) wred[c][th >> 6] = v;
  }
  __syncthreads();
  if (th < 7) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kFusedZThreads / 64; ++w) v += wred[th][w];
    partials[(size_t)blockIdx.x * 8 + th] = v;
  }
}

// Block (z, f): the inverse y and x transforms of plane z of field f (0: Ex +
// i Ey, 1: Ez) in LDS; writes packed[4 e + 0..1] = (Ex, Ey) or packed[4 e + 2]
// = Ez for mesh index e.  Block of 1024 threads; LDS (Kx Ky + Kx + Ky)
// complex values.
template <typename T>
__global__ void __launch_bounds__(1024) k_mixed_ifft_xy(const cpx<T>* __restrict__ fxy,
                                                        const cpx<T>* __restrict__ fz, int Kx, int Ky,
                                                        T* __restrict__ packed) {
  constexpr int kMax = FusedPlane<T>::kMaxPts;
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<T>* cp = reinterpret_cast<cpx<T>*>(smem);
  const int nxy = Kx * Ky;
  cpx<T>* twx = cp + nxy;
  cpx<T>* twy = twx + Kx;
  const int z = blockIdx.x, f = blockIdx.y;
  const int64_t base = (int64_t)z * nxy;
  const cpx<T>* src = (f == 0 ? fxy : fz) + base;
  for (int e = threadIdx.x; e < nxy; e += blockDim.x) cp[e] = src[e];
  for (int m = threadIdx.x; m < Kx; m += blockDim.x) twx[m] = unit_root<T>(m, Kx, +1);
  for (int m = threadIdx.x; m < Ky; m += blockDim.x) twy[m] = unit_root<T>(m, Ky, +1);
  __syncthreads();
  lds_dft_rows<T, 1024, kMax, true>(cp, Ky, Kx, 1, Kx, true, twy);   // y columns
  lds_dft_rows<T, 1024, kMax, true>(cp, Kx, Ky, Kx, 1, false, twx);  // x rows
  if (f == 0) {
    for (int e = threadIdx.x; e < nxy; e += blockDim.x)
      *reinterpret_cast<cpx<T>*>(packed + 4 * (base + e)) = cp[e];
  } else {
    for (int e = threadIdx.x; e < nxy; e += blockDim.x) packed[4 * (base + e) + 2] = cp[e].x;
  }
}

// Chunk of particles for this block of a gather whose grid is a multiple of
// the XCD count: the blocks b, b + 8, ... that the hardware deals to one XCD
// take consecutive chunks, so each XCD's L2 holds one stretch of the field
// instead of all eight sharing every line.  Chunks at or beyond nchunks are
// empty.
#ifndef DPLR_MIXED_GATHER_XCD
#define DPLR_MIXED_GATHER_XCD 1
#endif
__device__ __forceinline__ int xcd_chunk(int nchunks) {
  if (!DPLR_MIXED_GATHER_XCD) return (int)blockIdx.x;
  const int per_xcd = (int)gridDim.x / kNumXcd;
  return ((int)blockIdx.x % kNumXcd) * per_xcd + (int)blockIdx.x / kNumXcd;
}

// F_ja = (k_e q_j / V) sum_g W(u_j - g) E_a(g) from the interleaved real
// fields (x, y, z, unused) of the last inverse pass.  A wave serves 64 / P
// particles with P lanes each; lane tx reads the stencil column x = s_x + tx
// on all P^2 (y, z) rows, so the P lanes of a particle read P consecutive
// field values per load, and the column sums are added across the lanes
// (in lane order: deterministic).  All loads of a batch of z planes are
// issued before any is used.  Block 0 also reduces the energy/virial
// partials (the ik multiply's blocks ran before this kernel on the stream).
template <typename T, int P>
__device__ __forceinline__ void mixed_gather_column(const T4<T>* __restrict__ Ef, int Kx, int Ky, int Kz, int sx,
                                                    int sy, int sz, T dy, T dz, int tx, T (&part)[3]) {
  T wy[P], wz[P];
  bspline_weights<T, P>(dy, wy);
  bspline_weights<T, P>(dz, wz);
  int gx = sx + tx;
  if (gx >= Kx) gx -= Kx;
  constexpr int TZB = (P <= 5) ? P : ((P <= 6) ? 3 : 2);
#pragma unroll
  for (int tz0 = 0; tz0 < P; tz0 += TZB) {
    T4<T> r[TZB][P];
#pragma unroll
    for (int dzb = 0; dzb < TZB; ++dzb) {
      if (tz0 + dzb < P) {
        int gz = sz + tz0 + dzb;
        if (gz >= Kz) gz -= Kz;
        const T4<T>* fz = Ef + (int64_t)gz * Ky * Kx + gx;
#pragma unroll
        for (int ty = 0; ty < P; ++ty) {
          int gy = sy + ty;
          if (gy >= Ky) gy -= Ky;
          r[dzb][ty] = fz[gy * Kx];
        }
      }
    }
#pragma unroll
    for (int dzb = 0; dzb < TZB; ++dzb) {
      if (tz0 + dzb < P) {
#pragma unroll
        for (int ty = 0; ty < P; ++ty) {
          const T w = wz[tz0 + dzb] * wy[ty];
          part[0] += w * r[dzb][ty].x;
          part[1] += w * r[dzb][ty].y;
          part[2] += w * r[dzb][ty].z;
        }
      }
    }
  }
}

// Lane-group reduction and store of the force of one particle.
template <typename T, int P>
__device__ __forceinline__ void mixed_gather_store(const T (&part)[3], T qw, int grp, int tx, bool on, int64_t src,
                                                   int64_t n_ion, T* __restrict__ ion_f, T* __restrict__ wc_f,
                                                   int accumulate) {
  const int gbase = grp * P;
  T tot[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T mine = qw * part[a];
    T sum = (T)0;
#pragma unroll
    for (int q = 0; q < P; ++q) sum += __shfl(mine, gbase + q, 64);
    tot[a] = sum;
  }
  if (on && tx == 0) {
    T* out = (src < n_ion) ? (ion_f + 3 * src) : (wc_f + 3 * (src - n_ion));
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = accumulate ? out[a] + tot[a] : tot[a];
  }
}

// Particles per block of the mixed gathers (4 waves of 64 / P).
template <int P>
constexpr int mixed_gather_per_block() { return 4 * (64 / P); }

// From the sorted records of the plane spread: particle v of the sorted
// order, force to the caller's index perm[v].
template <typename T, int P>
__global__ void __launch_bounds__(256) k_mixed_gather_sorted(const T4<T>* __restrict__ rec,
                                                             const int* __restrict__ spk,
                                                             const int* __restrict__ perm, int64_t n_ion, int64_t n,
                                                             int Kx, int Ky, int Kz, const T4<T>* __restrict__ Ef,
                                                             T* __restrict__ ion_f, T* __restrict__ wc_f, T fscale,
                                                             int accumulate, const double* __restrict__ partials,
                                                             int nblk, double pre, double* __restrict__ energy,
                                                             double* __restrict__ virial, int nchunks) {
  if (blockIdx.x == 0) {
    __shared__ double red[7 * 256];
    reduce_partials(partials, nblk, pre, energy, virial, red);
  }
  constexpr int GPW = 64 / P;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / P, tx = lane - grp * P;
  const int chunk = xcd_chunk(nchunks);
  const int64_t v = (int64_t)chunk * mixed_gather_per_block<P>() + wave * GPW + grp;
  const bool on = grp < GPW && chunk < nchunks && v < n;
  T part[3] = {(T)0, (T)0, (T)0};
  T qw = (T)0;
  int64_t src = 0;
  if (on) {
    const T4<T> rc = rec[v];
    const int pk = spk[v];
    src = perm[v];
    T wxt, dxt;
    bspline_weight_at<T, P>(rc.x, tx, wxt, dxt);
    mixed_gather_column<T, P>(Ef, Kx, Ky, Kz, pk & 1023, (pk >> 10) & 1023, pk >> 20, rc.y, rc.z, tx, part);
    qw = fscale * rc.w * wxt;
  }
  mixed_gather_store<T, P>(part, qw, grp, tx, on, src, n_ion, ion_f, wc_f, accumulate);
}

// In the caller's order (stencils computed here, as in the spread).
template <typename T, int P>
__global__ void __launch_bounds__(256) k_mixed_gather(const T* __restrict__ ion_pos, const T* __restrict__ ion_q,
                                                      const T* __restrict__ wc_pos, const T* __restrict__ wc_q,
                                                      int64_t n_ion, int64_t n, double ihx, double ihy, double ihz,
                                                      int Kx, int Ky, int Kz, const T4<T>* __restrict__ Ef,
                                                      T* __restrict__ ion_f, T* __restrict__ wc_f, T fscale,
                                                      int accumulate, const double* __restrict__ partials,
                                                      int nblk, double pre, double* __restrict__ energy,
                                                      double* __restrict__ virial, int nchunks) {
  if (blockIdx.x == 0) {
    __shared__ double red[7 * 256];
    reduce_partials(partials, nblk, pre, energy, virial, red);
  }
  constexpr int GPW = 64 / P;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / P, tx = lane - grp * P;
  const int chunk = xcd_chunk(nchunks);
  const int64_t i = (int64_t)chunk * mixed_gather_per_block<P>() + wave * GPW + grp;
  const bool on = grp < GPW && chunk < nchunks && i < n;
  T part[3] = {(T)0, (T)0, (T)0};
  T qw = (T)0;
  if (on) {
    const T* r = (i < n_ion) ? (ion_pos + 3 * i) : (wc_pos + 3 * (i - n_ion));
    double d[3];
    const int sx = mixed_stencil<P>((double)r[0], ihx, Kx, d[0]);
    const int sy = mixed_stencil<P>((double)r[1], ihy, Ky, d[1]);
    const int sz = mixed_stencil<P>((double)r[2], ihz, Kz, d[2]);
    T wxt, dxt;
    bspline_weight_at<T, P>((T)d[0], tx, wxt, dxt);
    mixed_gather_column<T, P>(Ef, Kx, Ky, Kz, sx, sy, sz, (T)d[1], (T)d[2], tx, part);
    const T q = (i < n_ion) ? ion_q[i] : wc_q[i - n_ion];
    qw = fscale * q * wxt;
  }
  mixed_gather_store<T, P>(part, qw, grp, tx, on, i, n_ion, ion_f, wc_f, accumulate);
}

}  // namespace dplr
