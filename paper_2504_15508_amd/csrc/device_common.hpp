// Device building blocks of the PPPM kernels (gfx950): complex arithmetic,
// LDS-resident FFT stages and order-p B-spline assignment weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dplr {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) {
  return INV ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Small DFTs in registers.  Forward uses exp(-2 pi i nk/R) (the sign of the
// DFT definition in the paper's FFT section); INV uses the conjugate.
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__device__ __forceinline__ void dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  cpx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mi<T, INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cpx<T>* a) {
  // radix-2 split into two length-4 DFTs of the even and odd samples
  cpx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cpx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  const T r = (T)0.70710678118654752440;
  // o1 *= w8^1, o2 *= w8^2, o3 *= w8^3  (w8 = exp(-+2 pi i / 8))
  cpx<T> w1 = INV ? cpx<T>{(o1.x - o1.y) * r, (o1.x + o1.y) * r} : cpx<T>{(o1.x + o1.y) * r, (o1.y - o1.x) * r};
  cpx<T> w2 = mul_mi<T, INV>(o2);
  cpx<T> w3 = INV ? cpx<T>{(-o3.x - o3.y) * r, (o3.x - o3.y) * r} : cpx<T>{(o3.y - o3.x) * r, (-o3.x - o3.y) * r};
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, w1);
  a[5] = csub(e1, w1);
  a[2] = cadd(e2, w2);
  a[6] = csub(e2, w2);
  a[3] = cadd(e3, w3);
  a[7] = csub(e3, w3);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(cpx<T>* v) {
  if constexpr (R == 4) {
    dft4<T, INV>(v[0], v[1], v[2], v[3]);
  } else {
    dft8<T, INV>(v);
  }
}

// ---------------------------------------------------------------------------
// Batched 1D FFTs of length N on data held in LDS, in place.
//
// Self-sorting (Stockham) formulation: stage with sub-transform length Ns
// takes, for butterfly j, the R inputs j + r*N/R, multiplies input r by
// exp(-2 pi i r (j mod Ns) / (Ns R)), applies an R-point DFT and writes
// output r to (j div Ns) Ns R + (j mod Ns) + r Ns.  Every thread loads all its
// butterflies' inputs into registers, the block synchronises, then it writes,
// so one LDS buffer suffices.
//
// Element e of row `row` lives at buf[row * rstride + e * estride].
// rows_fast selects whether consecutive threads walk rows (column transforms,
// estride > 1) or butterflies within a row (row transforms) - both keep
// consecutive lanes on consecutive LDS words.
// tw holds exp(-2 pi i k / twN), k < twN, with N dividing twN.
// EPT bounds the elements per thread: nrows * N <= EPT * blockDim.x.
// ---------------------------------------------------------------------------
// Row transforms (estride == 1) keep one padding element after every 16, so
// the stride-R writes of the early stages do not pile onto a few LDS banks:
// element e of a row lives at e + e / 16 (lds_pad).  Column transforms
// (estride > 1) are laid out unpadded: their lanes already walk consecutive
// words.
__device__ __forceinline__ int lds_pad(int e) { return e + (e >> 4); }
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 4); }

// 24-bit integer products (full rate on CDNA; 32-bit products issue at a
// quarter of the rate).  Every LDS index and mesh index fits.
__device__ __forceinline__ int imul(int a, int b) { return (int)__umul24((unsigned)a, (unsigned)b); }

template <typename T, int R, bool INV, int EPT, bool PAD>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, int nrows, float inv_nrows, int N, int rstride, int estride,
                                          bool rows_fast, int Ns, const cpx<T>* tw, int twN) {
  constexpr int BPT = (EPT + R - 1) / R;
  const int nb = N / R;
  const int lnb = 31 - __clz(nb);  // nb is a power of two
  const int total = imul(nrows, nb);
  // (butterfly b) -> (row, j); with rows fastest, j = floor(b / nrows) is formed
  // as (b + 1/2) / nrows in FP32, exact for b < 2^20
  auto split = [&](int b, int& row, int& j) {
    if (rows_fast) {
      j = (int)(((float)b + 0.5f) * inv_nrows);
      row = b - imul(j, nrows);
    } else {
      j = b & (nb - 1);
      row = b >> lnb;
    }
  };
  cpx<T> v[BPT][R];
#pragma unroll
  for (int c = 0; c < BPT; ++c) {
    const int b = threadIdx.x + c * blockDim.x;
    if (b < total) {
      int row, j;
      split(b, row, j);
      const cpx<T>* base = buf + imul(row, rstride);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = j + r * nb;
        v[c][r] = base[PAD ? lds_pad(e) : imul(e, estride)];
      }
    }
  }
  __syncthreads();
  const int twstep = twN / (Ns * R);
#pragma unroll
  for (int c = 0; c < BPT; ++c) {
    const int b = threadIdx.x + c * blockDim.x;
    if (b < total) {
      int row, j;
      split(b, row, j);
      const int k = j & (Ns - 1);
      if (Ns > 1) {
        const int kt = imul(k, twstep);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[r * kt];
          if (INV) w.y = -w.y;
          v[c][r] = cmul(v[c][r], w);
        }
      }
      dft_small<T, R, INV>(v[c]);
      cpx<T>* base = buf + imul(row, rstride);
      const int o = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = o + r * Ns;
        base[PAD ? lds_pad(e) : imul(e, estride)] = v[c][r];
      }
    }
  }
  __syncthreads();
}

// Full transform: radix-8 stages while that leaves a length of 4 or more
// (or exactly 1), radix-4 for the rest.  N is a power of two >= 4.
template <typename T, bool INV, int EPT, bool PAD = false>
__device__ __forceinline__ void fft_rows(cpx<T>* buf, int nrows, int N, int rstride, int estride, bool rows_fast,
                                         const cpx<T>* tw, int twN) {
  const float inv_nrows = 1.0f / (float)nrows;
  int lg = 31 - __clz(N);
  int Ns = 1;
  while (lg > 0) {
    if (lg >= 3 && lg - 3 != 1) {
      fft_stage<T, 8, INV, EPT, PAD>(buf, nrows, inv_nrows, N, rstride, estride, rows_fast, Ns, tw, twN);
      Ns *= 8;
      lg -= 3;
    } else {
      fft_stage<T, 4, INV, EPT, PAD>(buf, nrows, inv_nrows, N, rstride, estride, rows_fast, Ns, tw, twN);
      Ns *= 4;
      lg -= 2;
    }
  }
}

// ---------------------------------------------------------------------------
// B-spline assignment.  For mesh coordinate u (in mesh units) the stencil is
// the P points g = s .. s+P-1 with s = floor(u - P/2) + 1, and the weight of
// point s+t is M_P(u - (s+t) + P/2) = M_P(d + P-1-t), d = u - P/2 - floor(u - P/2).
// The values M_P(d + i), i = 0..P-1, are built order by order with the
// B-spline recursion M_k(x) = [x M_{k-1}(x) + (k-x) M_{k-1}(x-1)] / (k-1).
// ---------------------------------------------------------------------------
template <typename T, int P>
__device__ __forceinline__ void bspline_weights(T d, T* w) {
  T m[P];
  m[0] = (T)1;
#pragma unroll
  for (int i = 1; i < P; ++i) m[i] = (T)0;
#pragma unroll
  for (int k = 2; k <= P; ++k) {
    const T inv = (T)1 / (T)(k - 1);
#pragma unroll
    for (int i = k - 1; i >= 0; --i) {
      const T a = (i <= k - 2) ? m[i] : (T)0;
      const T b = (i >= 1) ? m[i - 1] : (T)0;
      m[i] = ((d + (T)i) * a + ((T)k - d - (T)i) * b) * inv;
    }
  }
#pragma unroll
  for (int t = 0; t < P; ++t) w[t] = m[P - 1 - t];
}

}  // namespace dplr
