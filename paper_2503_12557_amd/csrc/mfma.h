// Matrix-core (MFMA) products for the workgroup-level contractions: real
// FP32 / FP64 16x16x4 tiles, a complex product as four real ones, operand
// addresses from two-level index maps so that tensor contractions whose row,
// column or contracted index is a pair of tensor legs run as one product.
#pragma once

#include "common.h"

namespace pm {

typedef float mf32x4 __attribute__((ext_vector_type(4)));
typedef double mf64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 mbf16x8 __attribute__((ext_vector_type(8)));

// bfloat16 of x, rounded to nearest even (inf / nan kept)
__device__ __forceinline__ __bf16 to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  const unsigned short h = (unsigned short)(u >> 16);
  return __builtin_bit_cast(__bf16, h);
}

// One 16x16x4 matrix-core product per real type. Operand layout (both
// types): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]. Output
// register v of lane l holds D[row(l, v)][l % 16].
template <typename R> struct Mfma;
template <> struct Mfma<float> {
  typedef mf32x4 acc;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
  typedef mf64x4 acc;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <typename T>
__device__ __forceinline__ void split(T x, typename RealOf<T>::type& re,
                                      typename RealOf<T>::type& im) {
  if constexpr (IsCplx<T>::value) {
    re = x.re;
    im = x.im;
  } else {
    re = x;
    im = 0;
  }
}
template <typename T>
__device__ __forceinline__ T join(typename RealOf<T>::type re, typename RealOf<T>::type im) {
  if constexpr (IsCplx<T>::value) return T(re, im);
  else return re;
}

// Offset of index x of a two-level index: (x / d) * hi + (x % d) * lo
// (indices below 2^16, d <= 2^16; a single stride s is {1, s, 0}).
struct IMap {
  FastDiv d;
  int hi, lo;
  __device__ IMap(int s) : d(1), hi(s), lo(0) {}
  __device__ IMap(int d_, int hi_, int lo_) : d(d_), hi(hi_), lo(lo_) {}
  __device__ __forceinline__ int operator()(int x) const {
    const int q = d.div(x);
    return q * hi + (x - q * d.d) * lo;
  }
};

// ---------------------------------------------------------------------------
// C (m x n) = op(A) op(B) (+ C if acc) with A[i][kk] at A[ai(i) + ak(kk)],
// B[kk][j] at B[bk(kk) + bj(j)] and C[i][j] at C[ci(i) + cj(j)]; CA / CB
// conjugate that operand. Waves take 32 x 32 output blocks (2 x 2 MFMA
// tiles). herm (square C with ci(i) = i * ldc, cj = 1): only the blocks on
// and below the diagonal are formed and conj(C[i][j]) is also written to
// C[j][i] below it. Operands may be in global memory or LDS; out-of-range
// rows, columns and k read as zero. The caller synchronises before reading
// C. BF (real FP32 operands only): the operands are rounded to bfloat16 and
// multiplied by v_mfma_f32_16x16x32_bf16 (lane l holds A[l % 16][8 (l / 16)
// + t] and B[8 (l / 16) + t][l % 16], t < 8) with FP32 accumulation. G3
// (complex operands): three real products per complex one, P1 = Re A Re B,
// P2 = Im A Im B, P3 = (Re A + Im A)(Re B + Im B), Re C = P1 - P2, Im C =
// P3 - P1 - P2 (a quarter fewer matrix-core cycles; the imaginary part's
// error bound grows from u (|Re A||Im B| + |Im A||Re B|) to about
// u (|Re A| + |Im A|)(|Re B| + |Im B|)).
// ---------------------------------------------------------------------------
template <typename T, bool CA, bool CB, bool BF = false, bool G3 = false>
__device__ void mgemm_map(int m, int n, int k, const T* __restrict__ A, IMap ai, IMap ak,
                          const T* __restrict__ B, IMap bk, IMap bj, T* __restrict__ C, IMap ci,
                          IMap cj, bool herm, bool acc) {
  typedef typename RealOf<T>::type R;
  typedef Mfma<R> F;
  typedef typename F::acc V;
  constexpr bool CX = IsCplx<T>::value;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = PEPS_NT >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nbi = (m + 31) >> 5, nbj = (n + 31) >> 5;
  const int njobs = herm ? nbi * (nbi + 1) / 2 : nbi * nbj;
  const R sa = CA ? R(-1) : R(1), sb = CB ? R(-1) : R(1);
  for (int job = wv; job < njobs; job += nw) {
    int bi, bjb;
    if (herm) {
      bi = 0;
      while ((bi + 1) * (bi + 2) / 2 <= job) ++bi;
      bjb = job - bi * (bi + 1) / 2;
    } else {
      bi = job / nbj;
      bjb = job - bi * nbj;
    }
    const int i0 = bi * 32, j0 = bjb * 32;
    // complex: cr / ci_ the real and imaginary sums, or P1 / P2 with P3 in
    // cp (G3)
    V cr[2][2], ci_[2][2], cp[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cr[a][b][v] = 0;
          ci_[a][b][v] = 0;
          cp[a][b][v] = 0;
        }
    if (acc) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = i0 + 16 * a + F::row(lane, v), j = j0 + 16 * b + li;
            if (i < m && j < n) {
              R re, im;
              split(C[ci(i) + cj(j)], re, im);
              cr[a][b][v] = re;
              if constexpr (CX && G3)
                cp[a][b][v] = re + im;
              else
                ci_[a][b][v] = im;
            }
          }
    }
    const bool ia0 = i0 + li < m, ia1 = i0 + 16 + li < m;
    const bool jb0 = j0 + li < n, jb1 = j0 + 16 + li < n;
    const T* pa0 = A + (ia0 ? ai(i0 + li) : 0);
    const T* pa1 = A + (ia1 ? ai(i0 + 16 + li) : 0);
    const T* pb0 = B + (jb0 ? bj(j0 + li) : 0);
    const T* pb1 = B + (jb1 ? bj(j0 + 16 + li) : 0);
    if constexpr (BF) {
      static_assert(!CX, "bfloat16 products take real operands");
      for (int k0 = 0; k0 < k; k0 += 32) {
        mbf16x8 av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int kk = k0 + 8 * lk + t;
          const bool kin = kk < k;
          const int oa = kin ? ak(kk) : 0, ob = kin ? bk(kk) : 0;
          av[0][t] = to_bf16((kin && ia0) ? (float)pa0[oa] : 0.f);
          av[1][t] = to_bf16((kin && ia1) ? (float)pa1[oa] : 0.f);
          bv[0][t] = to_bf16((kin && jb0) ? (float)pb0[ob] : 0.f);
          bv[1][t] = to_bf16((kin && jb1) ? (float)pb1[ob] : 0.f);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            cr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], cr[a][b], 0, 0, 0);
      }
    } else {
    // k-steps of 4 loaded ahead of their products: four for real operands,
    // two for complex ones (register budget)
    constexpr int KS = CX ? 2 : 4;
    for (int k0 = 0; k0 < k; k0 += 4 * KS) {
      R ar[KS][2], aim[KS][2], br[KS][2], bim[KS][2];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int kk = k0 + 4 * s + lk;
        const bool kin = kk < k;
        const int oa = kin ? ak(kk) : 0, ob = kin ? bk(kk) : 0;
        T x0 = (kin && ia0) ? pa0[oa] : T(0);
        T x1 = (kin && ia1) ? pa1[oa] : T(0);
        T y0 = (kin && jb0) ? pb0[ob] : T(0);
        T y1 = (kin && jb1) ? pb1[ob] : T(0);
        split(x0, ar[s][0], aim[s][0]);
        split(x1, ar[s][1], aim[s][1]);
        split(y0, br[s][0], bim[s][0]);
        split(y1, br[s][1], bim[s][1]);
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            cr[a][b] = F::mac(ar[s][a], br[s][b], cr[a][b]);
            if constexpr (CX && G3) {
              const R ai2 = sa * aim[s][a], bi2 = sb * bim[s][b];
              ci_[a][b] = F::mac(ai2, bi2, ci_[a][b]);
              cp[a][b] = F::mac(ar[s][a] + ai2, br[s][b] + bi2, cp[a][b]);
            } else if constexpr (CX) {
              // (ar + i sa ai)(br + i sb bi)
              const R ai2 = sa * aim[s][a], bi2 = sb * bim[s][b];
              cr[a][b] = F::mac(-ai2, bi2, cr[a][b]);
              ci_[a][b] = F::mac(ar[s][a], bi2, ci_[a][b]);
              ci_[a][b] = F::mac(ai2, br[s][b], ci_[a][b]);
            }
          }
      }
    }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + 16 * a + F::row(lane, v), j = j0 + 16 * b + li;
          if (i < m && j < n) {
            T val;
            if constexpr (CX && G3) {
              const R p1 = cr[a][b][v], p2 = ci_[a][b][v];
              val = join<T>(p1 - p2, cp[a][b][v] - p1 - p2);
            } else {
              val = join<T>(cr[a][b][v], ci_[a][b][v]);
            }
            C[ci(i) + cj(j)] = val;
            if (herm && bi != bjb) C[ci(j) + cj(i)] = conjx(val);
          }
        }
  }
}

// Strided form: A[i*sai + kk*sak], B[kk*sbk + j*sbj], C[i*ldc + j].
template <typename T, bool CA, bool CB, bool BF = false, bool G3 = false>
__device__ __forceinline__ void mgemm(int m, int n, int k, const T* __restrict__ A, int sai,
                                      int sak, const T* __restrict__ B, int sbk, int sbj,
                                      T* __restrict__ C, int ldc, bool herm, bool acc) {
  mgemm_map<T, CA, CB, BF, G3>(m, n, k, A, IMap(sai), IMap(sak), B, IMap(sbk), IMap(sbj), C, IMap(ldc),
                       IMap(1), herm, acc);
}

}  // namespace pm
