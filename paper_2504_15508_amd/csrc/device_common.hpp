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

// LDS row padding: one spare element after every 16 (see the Stockham passes below).
__device__ __forceinline__ int lds_pad(int e) { return e + (e >> 4); }
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 4); }

// 16-point DFT in registers as 4 x 4 (n = a + 4b, k = c + 4d):
// X[c + 4d] = sum_a W4^{ad} W16^{ac} sum_b x[a + 4b] W4^{bc}.  In place,
// natural order in and out.
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cpx<T>* x) {
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, r2 = (T)0.70710678118654752440;
  cpx<T> t[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    cpx<T> b0 = x[a], b1 = x[a + 4], b2 = x[a + 8], b3 = x[a + 12];
    dft4<T, INV>(b0, b1, b2, b3);
    t[a][0] = b0; t[a][1] = b1; t[a][2] = b2; t[a][3] = b3;
  }
  // twiddles W16^{ac} (a, c = 1..3); W16 = exp(-+ 2 pi i / 16)
  const T sg = INV ? (T)1 : (T)-1;
  const cpx<T> w1{c1, sg * s1}, w2{r2, sg * r2}, w3{s1, sg * c1};
  const cpx<T> w4{(T)0, sg}, w6{-r2, sg * r2}, w9{-c1, -sg * s1};
  t[1][1] = cmul(t[1][1], w1); t[1][2] = cmul(t[1][2], w2); t[1][3] = cmul(t[1][3], w3);
  t[2][1] = cmul(t[2][1], w2); t[2][2] = cmul(t[2][2], w4); t[2][3] = cmul(t[2][3], w6);
  t[3][1] = cmul(t[3][1], w3); t[3][2] = cmul(t[3][2], w6); t[3][3] = cmul(t[3][3], w9);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cpx<T> d0 = t[0][c], d1 = t[1][c], d2 = t[2][c], d3 = t[3][c];
    dft4<T, INV>(d0, d1, d2, d3);
    x[c] = d0; x[c + 4] = d1; x[c + 8] = d2; x[c + 12] = d3;
  }
}

// L-point DFT in registers, L in {1, 2, 4, 8, 16}, natural order.
template <typename T, int L, bool INV>
__device__ __forceinline__ void dft_l(cpx<T>* v) {
  if constexpr (L == 2) {
    const cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (L == 4) {
    dft4<T, INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (L == 8) {
    dft8<T, INV>(v);
  } else if constexpr (L == 16) {
    dft16<T, INV>(v);
  }
}

// ---------------------------------------------------------------------------
// Batched in-place FFTs of length N = 16 L (L in {1, 2, 4, 8, 16}) on rows held
// in LDS, computed in registers: L threads per row, 16 values per thread, one
// exchange through the row itself.  With n = l + L n1 and k = k1 + 16 k2,
//   X[k1 + 16 k2] = sum_l W_L^{l k2} W_N^{l k1} sum_n1 x[l + L n1] W_16^{n1 k1}:
// thread l transforms x[l + L n1] over n1 (16 points), multiplies by
// W_N^{l k1} and writes to slot k1 L + l; thread m then reads slots
// 16 m .. 16 m + 15 (k1 = m J + j, J = 16 / L, all l) and transforms over l
// (L points), writing X in natural order.  The inverse runs the steps
// backwards with conjugate twiddles.  Element e of row r lives at
// buf[r * rstride + (PAD ? lds_pad(e) : e * estride)]; rows_fast selects
// whether consecutive threads walk rows (column layouts) or the L threads of
// one row.  Every thread of the block must call it (it synchronises).
// ---------------------------------------------------------------------------
// The first read phase takes its inputs from load(r, e) and the last write
// phase hands its outputs to store(r, e, value), so a caller can fuse a
// conversion or rearrangement into the transform's own passes; the exchange
// in between goes through buf.  Every read made by load happens before the
// first barrier, so buf may alias what load reads.
template <typename T, int L, bool INV, bool PAD, typename LoadF, typename StoreF>
__device__ __forceinline__ void fft_rows_reg_io(cpx<T>* buf, int nrows, int rstride, int estride, bool rows_fast,
                                                const cpx<T>* tw, int twN, LoadF load, StoreF store) {
  constexpr int N = 16 * L, J = 16 / L;
  const int t = threadIdx.x;
  const bool act = t < nrows * L;
  int r = 0, l = 0;
  if (act) {
    if (rows_fast) { l = t / nrows; r = t - l * nrows; }
    else { r = t / L; l = t - r * L; }
  }
  cpx<T>* row = buf + r * rstride;
  auto at = [&](int e) -> cpx<T>& { return row[PAD ? lds_pad(e) : e * estride]; };
  const int step = twN / N;
  cpx<T> v[16];
  if constexpr (!INV) {
    if (act) {
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) v[n1] = load(r, l + L * n1);
    }
    __syncthreads();
    if (act) {
      dft16<T, false>(v);
#pragma unroll
      for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[((l * k1) & (N - 1)) * step]);
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) at(k1 * L + l) = v[k1];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = at(16 * l + e);  // (k1 = l J + e / L, l' = e % L)
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        dft_l<T, L, false>(v + j * L);
#pragma unroll
        for (int k2 = 0; k2 < L; ++k2) store(r, l * J + j + 16 * k2, v[j * L + k2]);
      }
    }
    __syncthreads();
  } else {
    if (act) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
#pragma unroll
        for (int k2 = 0; k2 < L; ++k2) v[j * L + k2] = load(r, l * J + j + 16 * k2);
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        dft_l<T, L, true>(v + j * L);
        const int k1 = l * J + j;
#pragma unroll
        for (int m = 1; m < L; ++m) {
          cpx<T> w = tw[((m * k1) & (N - 1)) * step];
          w.y = -w.y;
          v[j * L + m] = cmul(v[j * L + m], w);
        }
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) at(16 * l + e) = v[e];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) v[k1] = at(k1 * L + l);
    }
    __syncthreads();
    if (act) {
      dft16<T, true>(v);
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) store(r, l + L * n1, v[n1]);
    }
    __syncthreads();
  }
}

template <typename T, int L, bool INV, bool PAD>
__device__ __forceinline__ void fft_rows_reg(cpx<T>* buf, int nrows, int rstride, int estride, bool rows_fast,
                                             const cpx<T>* tw, int twN) {
  auto elem = [=](int r, int e) -> cpx<T>& { return buf[r * rstride + (PAD ? lds_pad(e) : e * estride)]; };
  fft_rows_reg_io<T, L, INV, PAD>(
      buf, nrows, rstride, estride, rows_fast, tw, twN, [&](int r, int e) { return elem(r, e); },
      [&](int r, int e, const cpx<T>& x) { elem(r, e) = x; });
}

// Column transforms (element e of column c at buf[e * estride + c], consecutive
// threads on consecutive columns) with fused input and output: applicable for
// FP32 columns of N = 16 L <= 256 points when the block has ncols * L
// threads; false (nothing done) otherwise.
template <typename T, bool INV, typename LoadF, typename StoreF>
__device__ __forceinline__ bool fft_cols_io(cpx<T>* buf, int ncols, int N, int estride, const cpx<T>* tw, int twN,
                                            LoadF load, StoreF store) {
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    const int L = N / 16;
    if (N < 16 || N > 256 || ncols * L > (int)blockDim.x) return false;
    switch (L) {
      case 1: fft_rows_reg_io<T, 1, INV, false>(buf, ncols, 1, estride, true, tw, twN, load, store); return true;
      case 2: fft_rows_reg_io<T, 2, INV, false>(buf, ncols, 1, estride, true, tw, twN, load, store); return true;
      case 4: fft_rows_reg_io<T, 4, INV, false>(buf, ncols, 1, estride, true, tw, twN, load, store); return true;
      case 8: fft_rows_reg_io<T, 8, INV, false>(buf, ncols, 1, estride, true, tw, twN, load, store); return true;
      case 16: fft_rows_reg_io<T, 16, INV, false>(buf, ncols, 1, estride, true, tw, twN, load, store); return true;
    }
    return false;
  }
}

// Row transforms (PAD layout, exchange through buf) with fused input and
// output: applicable for FP32 rows of N = 16 L <= 256 points when the block
// has nrows * L threads; false (nothing done) otherwise.
template <typename T, bool INV, typename LoadF, typename StoreF>
__device__ __forceinline__ bool fft_rows_io(cpx<T>* buf, int nrows, int N, int rstride, const cpx<T>* tw, int twN,
                                            LoadF load, StoreF store) {
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    const int L = N / 16;
    if (N < 16 || N > 256 || nrows * L > (int)blockDim.x) return false;
    switch (L) {
      case 1: fft_rows_reg_io<T, 1, INV, true>(buf, nrows, rstride, 1, false, tw, twN, load, store); return true;
      case 2: fft_rows_reg_io<T, 2, INV, true>(buf, nrows, rstride, 1, false, tw, twN, load, store); return true;
      case 4: fft_rows_reg_io<T, 4, INV, true>(buf, nrows, rstride, 1, false, tw, twN, load, store); return true;
      case 8: fft_rows_reg_io<T, 8, INV, true>(buf, nrows, rstride, 1, false, tw, twN, load, store); return true;
      case 16: fft_rows_reg_io<T, 16, INV, true>(buf, nrows, rstride, 1, false, tw, twN, load, store); return true;
    }
    return false;
  }
}

// Register FFTs for N = 16 L with L <= 16 when the block has enough threads
// (FP32 only: the FP64 registers would spill); false when not applicable.
template <typename T, bool INV, bool PAD>
__device__ __forceinline__ bool fft_rows_try_reg(cpx<T>* buf, int nrows, int N, int rstride, int estride,
                                                 bool rows_fast, const cpx<T>* tw, int twN) {
  if constexpr (sizeof(T) != 4) return false;
  const int L = N / 16;
  if (N < 16 || N > 256 || nrows * L > (int)blockDim.x) return false;
  switch (L) {
    case 1: fft_rows_reg<T, 1, INV, PAD>(buf, nrows, rstride, estride, rows_fast, tw, twN); return true;
    case 2: fft_rows_reg<T, 2, INV, PAD>(buf, nrows, rstride, estride, rows_fast, tw, twN); return true;
    case 4: fft_rows_reg<T, 4, INV, PAD>(buf, nrows, rstride, estride, rows_fast, tw, twN); return true;
    case 8: fft_rows_reg<T, 8, INV, PAD>(buf, nrows, rstride, estride, rows_fast, tw, twN); return true;
    case 16: fft_rows_reg<T, 16, INV, PAD>(buf, nrows, rstride, estride, rows_fast, tw, twN); return true;
  }
  return false;
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
  if (fft_rows_try_reg<T, INV, PAD>(buf, nrows, N, rstride, estride, rows_fast, tw, twN)) return;
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
// On [0, 1) each M_P(d + i), i = 0..P-1, is a polynomial of degree P-1 in d.
// Its coefficients follow from the B-spline recursion
// M_k(x) = [x M_{k-1}(x) + (k-x) M_{k-1}(x-1)] / (k-1), applied to coefficient
// arrays at compile time; a weight is then P-1 fused multiply-adds (Horner)
// instead of the O(P^2) recursion per coordinate.
// ---------------------------------------------------------------------------
template <int P>
struct BsplineCoeffs {
  double c[P][P];  // c[i][j]: coefficient of d^j in M_P(d + i), 0 <= d < 1
  constexpr BsplineCoeffs() : c{} {
    double m[P][P] = {};  // M_k(d + i) for the current order k
    m[0][0] = 1.0;        // M_1(d) = 1
    for (int k = 2; k <= P; ++k) {
      double nm[P][P] = {};
      for (int i = 0; i < k; ++i) {
        for (int j = 0; j < P; ++j) {
          double v = 0.0;
          if (i <= k - 2) {  // (d + i) M_{k-1}(d + i)
            v += i * m[i][j];
            if (j > 0) v += m[i][j - 1];
          }
          if (i >= 1) {  // (k - i - d) M_{k-1}(d + i - 1)
            v += (k - i) * m[i - 1][j];
            if (j > 0) v -= m[i - 1][j - 1];
          }
          nm[i][j] = v / (k - 1);
        }
      }
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) m[i][j] = nm[i][j];
    }
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) c[i][j] = m[i][j];
  }
};

template <typename T, int P>
__device__ __forceinline__ void bspline_weights(T d, T* w) {
  constexpr BsplineCoeffs<P> C{};
#pragma unroll
  for (int t = 0; t < P; ++t) {
    const int i = P - 1 - t;
    T v = (T)C.c[i][P - 1];
#pragma unroll
    for (int j = P - 2; j >= 0; --j) v = v * d + (T)C.c[i][j];
    w[t] = v;
  }
}

// Derivatives dw[t] = M'_P(d + P-1-t) of the weights above with respect to the
// mesh coordinate (the derivative of each polynomial, also by Horner).
template <typename T, int P>
__device__ __forceinline__ void bspline_dweights(T d, T* dw) {
  constexpr BsplineCoeffs<P> C{};
#pragma unroll
  for (int t = 0; t < P; ++t) {
    const int i = P - 1 - t;
    T v = (T)((P - 1) * C.c[i][P - 1]);
#pragma unroll
    for (int j = P - 2; j >= 1; --j) v = v * d + (T)(j * C.c[i][j]);
    dw[t] = v;
  }
}

// Weight w[t] and derivative dw[t] of one stencil point t (runtime, 0..P-1):
// the polynomial's coefficients are selected first, then evaluated by Horner.
template <typename T, int P>
__device__ __forceinline__ void bspline_weight_at(T d, int t, T& w, T& dw) {
  constexpr BsplineCoeffs<P> C{};
  T c[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    T v = (T)C.c[P - 1][j];
#pragma unroll
    for (int k = 1; k < P; ++k) v = (t == k) ? (T)C.c[P - 1 - k][j] : v;
    c[j] = v;
  }
  T a = c[P - 1], b = (T)(P - 1) * c[P - 1];
#pragma unroll
  for (int j = P - 2; j >= 0; --j) {
    a = a * d + c[j];
    if (j >= 1) b = b * d + (T)j * c[j];
  }
  w = a;
  dw = b;
}

}  // namespace dplr
