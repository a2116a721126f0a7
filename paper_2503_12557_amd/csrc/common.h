// Shared device-side definitions: precision modes, block reductions,
// workgroup-level small linear algebra on LDS (Householder QR, one-sided
// Jacobi, strided GEMM) and the lattice tables the kernels read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define PEPS_BLOCK_MAX 512
// threads of the running block (launches use 256 or 512)
#define PEPS_NT ((int)blockDim.x)

namespace pm {

// ---------------------------------------------------------------------------
// Precision modes. T is the arithmetic type of contractions, QR and SVD.
// In BF16 mode every contraction operand is rounded to bfloat16 (round to
// nearest even) and the products are accumulated in FP32.
// ---------------------------------------------------------------------------
enum Mode { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16 = 2, MODE_C128 = 3, MODE_C64 = 4 };

// Threads per environment / sampler workgroup: the 8-byte and 16-byte
// element modes hold more LDS per workgroup (one per CU), so they run eight
// waves; FP32 and BF16 fit two workgroups per CU and run four waves each.
__host__ __device__ constexpr int env_threads(int mode) {
  return (mode == MODE_F32 || mode == MODE_BF16) ? 256 : 512;
}

// ---------------------------------------------------------------------------
// Complex scalar for the complex-tensor modes. Contractions of the network
// never conjugate (the amplitude is holomorphic in the tensors); the
// orthogonalisations (Householder, Jacobi) and the minSR Gram use conjx.
// ---------------------------------------------------------------------------
template <typename R>
struct cplx {
  R re, im;
  cplx() = default;
  template <typename U>
  __host__ __device__ constexpr cplx(U r) : re(R(r)), im(0) {}
  __host__ __device__ constexpr cplx(R r, R i) : re(r), im(i) {}
  __host__ __device__ cplx& operator+=(const cplx& b) {
    re += b.re;
    im += b.im;
    return *this;
  }
  __host__ __device__ cplx& operator-=(const cplx& b) {
    re -= b.re;
    im -= b.im;
    return *this;
  }
  __host__ __device__ cplx& operator*=(const cplx& b) {
    const R r = re * b.re - im * b.im;
    im = re * b.im + im * b.re;
    re = r;
    return *this;
  }
  __host__ __device__ cplx& operator*=(R s) {
    re *= s;
    im *= s;
    return *this;
  }
};
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) {
  return cplx<R>(a.re + b.re, a.im + b.im);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) {
  return cplx<R>(a.re - b.re, a.im - b.im);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator-(cplx<R> a) {
  return cplx<R>(-a.re, -a.im);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return cplx<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(cplx<R> a, R s) {
  return cplx<R>(a.re * s, a.im * s);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) {
  return cplx<R>(a.re * s, a.im * s);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator/(cplx<R> a, R s) {
  return cplx<R>(a.re / s, a.im / s);
}
template <typename R>
__host__ __device__ __forceinline__ bool operator==(cplx<R> a, cplx<R> b) {
  return a.re == b.re && a.im == b.im;
}
template <typename R>
__host__ __device__ __forceinline__ bool operator!=(cplx<R> a, cplx<R> b) {
  return !(a == b);
}

template <typename T> struct RealOf { typedef T type; };
template <typename R> struct RealOf<cplx<R>> { typedef R type; };
template <typename T> struct IsCplx { static constexpr bool value = false; };
template <typename R> struct IsCplx<cplx<R>> { static constexpr bool value = true; };

__host__ __device__ __forceinline__ float conjx(float x) { return x; }
__host__ __device__ __forceinline__ double conjx(double x) { return x; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> conjx(cplx<R> x) { return cplx<R>(x.re, -x.im); }
__host__ __device__ __forceinline__ float abs2x(float x) { return x * x; }
__host__ __device__ __forceinline__ double abs2x(double x) { return x * x; }
template <typename R>
__host__ __device__ __forceinline__ R abs2x(cplx<R> x) { return x.re * x.re + x.im * x.im; }
__device__ __forceinline__ float absx(float x) { return fabsf(x); }
__device__ __forceinline__ double absx(double x) { return fabs(x); }
template <typename R>
__device__ __forceinline__ R absx(cplx<R> x) { return sqrt(x.re * x.re + x.im * x.im); }
__host__ __device__ __forceinline__ float realx(float x) { return x; }
__host__ __device__ __forceinline__ double realx(double x) { return x; }
template <typename R>
__host__ __device__ __forceinline__ R realx(cplx<R> x) { return x.re; }
__host__ __device__ __forceinline__ float imagx(float) { return 0.f; }
__host__ __device__ __forceinline__ double imagx(double) { return 0.0; }
template <typename R>
__host__ __device__ __forceinline__ R imagx(cplx<R> x) { return x.im; }
__device__ __forceinline__ bool finitex(float x) { return isfinite(x); }
__device__ __forceinline__ bool finitex(double x) { return isfinite(x); }
template <typename R>
__device__ __forceinline__ bool finitex(cplx<R> x) { return isfinite(x.re) && isfinite(x.im); }
// 1 / x
__device__ __forceinline__ float recipx(float x) { return 1.f / x; }
__device__ __forceinline__ double recipx(double x) { return 1.0 / x; }
template <typename R>
__device__ __forceinline__ cplx<R> recipx(cplx<R> x) {
  // Smith's scaling: no overflow of |x|^2 for large entries
  if (fabs(x.re) >= fabs(x.im)) {
    const R r = x.im / x.re, den = x.re + x.im * r;
    return cplx<R>(R(1) / den, -r / den);
  }
  const R r = x.re / x.im, den = x.re * r + x.im;
  return cplx<R>(r / den, R(-1) / den);
}
// (nr + i ni) / (dr + i di) in FP64 by Smith's algorithm; for di = 0 it
// reduces exactly to the two real divisions.
__device__ __forceinline__ void cdiv(double nr, double ni, double dr, double di, double& qr,
                                     double& qi) {
  if (fabs(di) <= fabs(dr)) {
    const double r = di / dr, den = dr + di * r;
    qr = (nr + ni * r) / den;
    qi = (ni - nr * r) / den;
  } else {
    const double r = dr / di, den = dr * r + di;
    qr = (nr * r + ni) / den;
    qi = (ni * r - nr) / den;
  }
}

__device__ __forceinline__ float shfl_xor_x(float v, int o) { return __shfl_xor(v, o, 64); }
__device__ __forceinline__ double shfl_xor_x(double v, int o) { return __shfl_xor(v, o, 64); }
template <typename R>
__device__ __forceinline__ cplx<R> shfl_xor_x(cplx<R> v, int o) {
  return cplx<R>(__shfl_xor(v.re, o, 64), __shfl_xor(v.im, o, 64));
}

// bytes per element of the compute type of a mode
__host__ __device__ constexpr size_t mode_elem_bytes(int mode) {
  return mode == MODE_C128 ? 16 : (mode == MODE_F64 || mode == MODE_C64) ? 8 : 4;
}

// Data-parallel-primitive (DPP) lane moves inside a row of 16 lanes:
// 0xB1 = quad_perm [1,0,3,2] (lane ^ 1), 0x4E = quad_perm [2,3,0,1]
// (lane ^ 2), 0x141 = half-row mirror (lane i <- 7 - i in each group of 8),
// 0x140 = row mirror (lane i <- 15 - i). Summing a value with its partner
// under these four in turn reduces groups of 2, 4, 8 and 16 lanes.
template <int CTRL>
__device__ __forceinline__ float dppx(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dppx(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, typename R>
__device__ __forceinline__ cplx<R> dppx(cplx<R> v) {
  return cplx<R>(dppx<CTRL>(v.re), dppx<CTRL>(v.im));
}

template <int M> struct ModeT;
template <> struct ModeT<MODE_F64> { typedef double T; };
template <> struct ModeT<MODE_F32> { typedef float T; };
template <> struct ModeT<MODE_BF16> { typedef float T; };
template <> struct ModeT<MODE_C128> { typedef cplx<double> T; };
template <> struct ModeT<MODE_C64> { typedef cplx<float> T; };

__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  return __uint_as_float(u);
}

template <int M> __device__ __forceinline__ typename ModeT<M>::T opnd(typename ModeT<M>::T x) {
  if constexpr (M == MODE_BF16) return bf16_round(x);
  else return x;
}

// Exact n / d for 0 <= n < 2^16 and 1 <= d <= 2^16 by a multiply-high with
// m = floor(2^32 / d) + 1: n m / 2^32 = n / d + n (1 - frac(2^32/d)) / 2^32,
// and the added term is below 2^-16 <= 1/d, so the floor is unchanged. The
// element loops decode their coordinates with it instead of runtime division.
struct FastDiv {
  uint32_t m;
  int d;
  __device__ explicit FastDiv(int d_)
      : m(d_ <= 1 ? 0u : 0xffffffffu / (uint32_t)d_ + 1u), d(d_) {}
  __device__ __forceinline__ int div(int n) const {
    return d <= 1 ? n : (int)__umulhi((uint32_t)n, m);
  }
};
// q <- q / d, returns q mod d
__device__ __forceinline__ int divmod(int& q, const FastDiv& f) {
  const int nq = f.div(q);
  const int r = q - nq * f.d;
  q = nq;
  return r;
}

// Physical index of a site; masked so a malformed sample byte cannot index
// outside the parameter block (samples with values > 1 are flagged).
__device__ __forceinline__ int pbit(uint8_t v) { return v & 1; }

template <typename T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };
template <> struct Eps<float> { static constexpr float v = 1.1920929e-7f; };
template <typename R> struct Eps<cplx<R>> { static constexpr R v = Eps<R>::v; };

// ---------------------------------------------------------------------------
// Lattice tables (host-computed, device-resident int array).
//   site_param_off[N] : offset of T[x,y][p=0] in theta
//   site_block[N]     : Dl*Dr*Du*Dd
//   site_legs[4N]     : Dl, Dr, Du, Dd
//   site_compact[N]   : offset of the site in a compact O row
//   compact_site[Nc]  : site of every compact O column
//   env_dims[slot][y][3] : (bl, k, br) of every environment tensor
// Environment slot s = x for the top environment E^u[x] (x = 0..Lx-2) and
// s = Lx-1 + (x-1) for the bottom environment E^l[x] (x = 1..Lx-1).
// ---------------------------------------------------------------------------
struct Lattice {
  int Lx, Ly, D, chi, N;
  int n_params, n_compact;
  int bmax;          // max(chi, D): largest boundary-MPS bond
  int site_box;      // bmax * D * bmax elements per environment tensor
  int n_slots;       // 2 * (Lx - 1)
  int off_param, off_block, off_legs, off_compact, off_env, off_csite;  // into tab
  // maximal truncated weight of a boundary-MPS truncation (0: keep chi)
  double trunc_w;
};

__device__ __forceinline__ int slot_top(const Lattice& L, int x) { return x; }
__device__ __forceinline__ int slot_bottom(const Lattice& L, int x) { return L.Lx - 1 + (x - 1); }

// ---------------------------------------------------------------------------
// Reductions over the 256-thread block. `red` is LDS scratch of >= 8 values.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dppx<0xB1>(v);
  v += dppx<0x4E>(v);
  v += dppx<0x141>(v);
  v += dppx<0x140>(v);
  v += shfl_xor_x(v, 16);
  v += shfl_xor_x(v, 32);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  T w = dppx<0xB1>(v);
  v = w > v ? w : v;
  w = dppx<0x4E>(v);
  v = w > v ? w : v;
  w = dppx<0x141>(v);
  v = w > v ? w : v;
  w = dppx<0x140>(v);
  v = w > v ? w : v;
  w = __shfl_xor(v, 16, 64);
  v = w > v ? w : v;
  w = __shfl_xor(v, 32, 64);
  v = w > v ? w : v;
  return v;
}

template <typename T>
__device__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < PEPS_NT / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

template <typename T>
__device__ T block_max(T v, T* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int i = 1; i < PEPS_NT / 64; ++i) s = red[i] > s ? red[i] : s;
  __syncthreads();
  return s;
}

// Largest modulus of t[0..cnt) (row stride ld for rows of width w) over the block.
template <typename T>
__device__ typename RealOf<T>::type block_absmax(const T* t, int rows, int w, int ld, T* red) {
  typedef typename RealOf<T>::type R;
  R mx = 0;
  for (int i = threadIdx.x; i < rows * w; i += PEPS_NT) {
    const int r = i / w, c = i - r * w;
    const R a = absx(t[r * ld + c]);
    mx = a > mx ? a : mx;
  }
  return block_max(mx, reinterpret_cast<R*>(red));
}

// Exponent e with mx * 2^-e in [0.5, 1); 0 when mx is zero or not finite.
__device__ __forceinline__ int pow2_exponent(double mx) {
  if (!(mx > 0.0) || !isfinite(mx)) return 0;
  int e;
  frexp(mx, &e);
  return e;
}

// t *= 2^-e (exact: a power of two changes no mantissa).
template <typename T>
__device__ void scale_pow2(T* t, int cnt, int e) {
  typedef typename RealOf<T>::type R;
  if (e == 0) return;
  const R f = (R)ldexp(1.0, -e);
  for (int i = threadIdx.x; i < cnt; i += PEPS_NT) t[i] *= f;
}

// Sum over groups of G consecutive lanes (G a power of two, G <= 64).
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
  if (G >= 2) v += dppx<0xB1>(v);
  if (G >= 4) v += dppx<0x4E>(v);
  if (G >= 8) v += dppx<0x141>(v);
  if (G >= 16) v += dppx<0x140>(v);
  if (G >= 32) v += shfl_xor_x(v, 16);
  if (G >= 64) v += shfl_xor_x(v, 32);
  return v;
}

// 16-byte vectors of FP32 (the caller guarantees alignment)
__device__ __forceinline__ float4 ld4(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
template <int M>
__device__ __forceinline__ float4 op4(float4 v) {
  return make_float4(opnd<M>(v.x), opnd<M>(v.y), opnd<M>(v.z), opnd<M>(v.w));
}
__device__ __forceinline__ void fma4(float4& acc, float w, float4 v) {
  acc.x = fmaf(w, v.x, acc.x);
  acc.y = fmaf(w, v.y, acc.y);
  acc.z = fmaf(w, v.z, acc.z);
  acc.w = fmaf(w, v.w, acc.w);
}

// The GEMM below for FP32 when B's and C's rows are contiguous, 16-byte
// aligned and n is a multiple of 4: each thread keeps four columns of two
// rows and reads B as 16-byte vectors. Every sum runs over k in order, as
// in the general form, so the results are the same.
template <int M>
__device__ void gemm_f4(int m, int n, int k, const float* A, int sai, int sak, const float* B,
                        int sbk, float* C, int sci, bool acc) {
  const int nq = n >> 2;
  int lj = 0;
  while ((1 << lj) < nq && lj < 6) ++lj;
  const int LJ = 1 << lj;
  const int tx = threadIdx.x & (LJ - 1), ty = threadIdx.x >> lj;
  const int rp = PEPS_NT >> lj;
  for (int i = ty; i < m; i += 2 * rp) {
    const int i2 = i + rp;
    const bool two = i2 < m;
    const float* a1 = A + i * sai;
    const float* a2 = A + (two ? i2 : i) * sai;
    for (int jq = tx; jq < nq; jq += LJ) {
      const float* bp = B + 4 * jq;
      float4 s1 = make_float4(0.f, 0.f, 0.f, 0.f), s2 = s1;
#pragma unroll 4
      for (int kk = 0; kk < k; ++kk) {
        const float4 bv = op4<M>(ld4(bp + kk * sbk));
        fma4(s1, opnd<M>(a1[kk * sak]), bv);
        fma4(s2, opnd<M>(a2[kk * sak]), bv);
      }
      float* c1 = C + i * sci + 4 * jq;
      if (acc) {
        const float4 o = ld4(c1);
        s1 = make_float4(o.x + s1.x, o.y + s1.y, o.z + s1.z, o.w + s1.w);
      }
      st4(c1, s1);
      if (two) {
        float* c2 = C + i2 * sci + 4 * jq;
        if (acc) {
          const float4 o = ld4(c2);
          s2 = make_float4(o.x + s2.x, o.y + s2.y, o.z + s2.z, o.w + s2.w);
        }
        st4(c2, s2);
      }
    }
  }
}

// The GEMM below for FP32 when both A's rows and B's columns are
// contiguous in k (C = A B^T of row-major A and B), 16-byte aligned, k a
// multiple of 4: A and B are read as 16-byte vectors; every sum still runs
// over k in order, so the results are the same.
template <int M>
__device__ void gemm_nt_f4(int m, int n, int k, const float* A, int sai, const float* B, int sbj,
                           float* C, int sci, int scj, bool acc) {
  int lj = 0;
  while ((1 << lj) < n && lj < 6) ++lj;
  const int LJ = 1 << lj;
  const int tx = threadIdx.x & (LJ - 1), ty = threadIdx.x >> lj;
  const int rp = PEPS_NT >> lj;
  for (int i = ty; i < m; i += 2 * rp) {
    const int i2 = i + rp;
    const bool two = i2 < m;
    const float* a1 = A + i * sai;
    const float* a2 = A + (two ? i2 : i) * sai;
    for (int j = tx; j < n; j += LJ) {
      const float* bp = B + j * sbj;
      float s1 = 0.f, s2 = 0.f;
#pragma unroll 2
      for (int kk = 0; kk < k; kk += 4) {
        const float4 b4 = op4<M>(ld4(bp + kk));
        const float4 x = op4<M>(ld4(a1 + kk));
        const float4 y = op4<M>(ld4(a2 + kk));
        s1 = fmaf(x.x, b4.x, s1);
        s1 = fmaf(x.y, b4.y, s1);
        s1 = fmaf(x.z, b4.z, s1);
        s1 = fmaf(x.w, b4.w, s1);
        s2 = fmaf(y.x, b4.x, s2);
        s2 = fmaf(y.y, b4.y, s2);
        s2 = fmaf(y.z, b4.z, s2);
        s2 = fmaf(y.w, b4.w, s2);
      }
      float* c1 = C + i * sci + j * scj;
      *c1 = acc ? *c1 + s1 : s1;
      if (two) {
        float* c2 = C + i2 * sci + j * scj;
        *c2 = acc ? *c2 + s2 : s2;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Strided GEMM over the block: C[i,j] (+)= sum_k A[i*sai + k*sak] * B[k*sbk + j*sbj]
// written to C[i*sci + j*scj]. Operands may live in LDS or global memory.
// Lanes run over j (a power of two >= n, at most 64), the rest of the block
// over i, two rows per thread so each B element is read once for both.
// The caller synchronises before reading C. CB conjugates the B operand.
// ---------------------------------------------------------------------------
template <int M, bool CB = false, typename T>
__device__ void gemm(int m, int n, int k, const T* A, int sai, int sak, const T* B, int sbk,
                     int sbj, T* C, int sci, int scj, bool acc) {
  if constexpr (std::is_same<T, float>::value && !CB) {
    if (sbj == 1 && scj == 1 && (n & 3) == 0 && (sbk & 3) == 0 && (sci & 3) == 0 &&
        ((reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(C)) & 15) == 0) {
      gemm_f4<M>(m, n, k, A, sai, sak, B, sbk, C, sci, acc);
      return;
    }
    if (sak == 1 && sbk == 1 && (k & 3) == 0 && (sai & 3) == 0 && (sbj & 3) == 0 &&
        ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0) {
      gemm_nt_f4<M>(m, n, k, A, sai, B, sbj, C, sci, scj, acc);
      return;
    }
  }
  int lj = 0;
  while ((1 << lj) < n && lj < 6) ++lj;
  const int LJ = 1 << lj;
  const int tx = threadIdx.x & (LJ - 1), ty = threadIdx.x >> lj;
  const int rp = PEPS_NT >> lj;
  for (int i = ty; i < m; i += 2 * rp) {
    const int i2 = i + rp;
    const bool two = i2 < m;
    const T* a1 = A + i * sai;
    const T* a2 = A + (two ? i2 : i) * sai;
    for (int j = tx; j < n; j += LJ) {
      const T* bp = B + j * sbj;
      T s1 = 0, s2 = 0;
#pragma unroll 4
      for (int kk = 0; kk < k; ++kk) {
        T bv = opnd<M>(bp[kk * sbk]);
        if constexpr (CB) bv = conjx(bv);
        s1 += opnd<M>(a1[kk * sak]) * bv;
        s2 += opnd<M>(a2[kk * sak]) * bv;
      }
      T* c1 = C + i * sci + j * scj;
      *c1 = acc ? *c1 + s1 : s1;
      if (two) {
        T* c2 = C + i2 * sci + j * scj;
        *c2 = acc ? *c2 + s2 : s2;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Householder QR keeping only R, for a stacked LDS matrix A (m x n, row
// stride lda, n <= 256) whose first kr rows are already upper triangular
// (zero below the diagonal) and whose remaining rows are dense. Reflector j
// only touches row j and the dense rows, so the triangular block is never
// swept. On exit rows 0..min(m,n)-1 hold R and every entry below the
// diagonal is zero. Column c belongs to wave (c mod waves); inside the wave four
// lanes share a column and split its rows, so the reflector's dot products
// reduce over four lanes without touching LDS, and each column costs one
// barrier: the wave that owns column j+1 also sums its squares for the next
// reflector. nrm: LDS scratch of >= 2 elements. For complex T the reflectors
// are unitary, H = I - tau v v^H, and R has a complex diagonal.
// ---------------------------------------------------------------------------
template <typename T>
__device__ void house_qr_stacked(T* A, int kr, int m, int n, int lda,
                                 typename RealOf<T>::type* nrm) {
  typedef typename RealOf<T>::type R;
  const int NW = PEPS_NT / 64;  // waves in the block
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int sub = lane & 3, cl = lane >> 2;  // row subset, column slot in the wave
  const int kmax = m < n ? m : n;
  if (kmax <= 0) return;
  // squares of column 0 below its diagonal (rows >= max(kr, 1))
  if (wv == 0) {
    const int r0 = kr > 1 ? kr : 1;
    R sq = 0;
    for (int i = r0 + lane; i < m; i += 64) sq += abs2x(A[i * lda]);
    sq = wave_sum(sq);
    if (lane == 0) nrm[0] = sq;
  }
  __syncthreads();
  for (int j = 0; j < kmax; ++j) {
    const int r0 = kr > j + 1 ? kr : j + 1;
    const R s = nrm[j & 1];
    const int r0n = kr > j + 2 ? kr : j + 2;  // rows of the next reflector
    if (s == R(0)) {
      // nothing to eliminate in column j; the next column's squares are
      // still needed
      if (j + 1 < kmax && ((j + 1) % NW) == wv) {
        R sq = 0;
        for (int i = r0n + lane; i < m; i += 64) sq += abs2x(A[i * lda + j + 1]);
        sq = wave_sum(sq);
        if (lane == 0) nrm[(j + 1) & 1] = sq;
      }
      __syncthreads();
      continue;
    }
    const T ajj = A[j * lda + j];
    T alpha, v0;
    R tau;
    if constexpr (IsCplx<T>::value) {
      // H = I - tau v v^H with v = (ajj - alpha, column below); alpha takes
      // the opposite phase of ajj so v0 suffers no cancellation
      const R aa = absx(ajj);
      const R nr = sqrt(aa * aa + s);
      alpha = aa > R(0) ? ajj * (-nr / aa) : T(-nr);
      v0 = ajj - alpha;
      tau = R(2) / (abs2x(v0) + s);
    } else {
      const T nr = sqrt(ajj * ajj + s);
      alpha = ajj > T(0) ? -nr : nr;
      v0 = ajj - alpha;
      tau = T(2) / (v0 * v0 + s);
    }
    // columns c > j owned by this lane: c = NW * (16 q + cl) + wv
    for (int q = 0; q < 256 / (16 * NW); ++q) {
      const int c = NW * (16 * q + cl) + wv;
      const bool own = c > j && c < n;  // uniform across the four lanes of c
      T d = 0;
      T rowj = 0;
      if (own) {
        rowj = A[j * lda + c];
        for (int i = r0 + sub; i < m; i += 4) d += conjx(A[i * lda + j]) * A[i * lda + c];
      }
      d += dppx<0xB1>(d);
      d += dppx<0x4E>(d);
      R sqn = 0;
      if (own) {
        const T w = tau * (conjx(v0) * rowj + d);
        if (sub == 0) A[j * lda + c] = rowj - v0 * w;
        for (int i = r0 + sub; i < m; i += 4) {
          const T nv = A[i * lda + c] - A[i * lda + j] * w;
          A[i * lda + c] = nv;
          if (i >= r0n) sqn += abs2x(nv);
        }
      }
      if (c == j + 1 && j + 1 < kmax) {  // this column feeds the next reflector
        sqn += dppx<0xB1>(sqn);
        sqn += dppx<0x4E>(sqn);
        if (sub == 0) nrm[(j + 1) & 1] = sqn;
      }
    }
    __syncthreads();
    // column j is final: R_jj = alpha, zeros below (nobody reads it again)
    if (tid == 0) A[j * lda + j] = alpha;
    for (int i = r0 + tid; i < m; i += PEPS_NT) A[i * lda + j] = T(0);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi on the m rows of the LDS matrix X (m x n, row
// stride ldx, m <= n): rotates pairs of rows until every pair is orthogonal
// to relative tolerance tol. Pairs follow the circle (round-robin) schedule,
// m-1 rounds of m/2 disjoint pairs per sweep; each pair is held by G lanes,
// each lane keeping its NC elements of both rows in registers between the
// dot products and the rotation. sflag: LDS int; nrm: 2m reals of LDS.
// Returns the number of sweeps used, or -1 if max_sweeps was reached.
// ---------------------------------------------------------------------------
// NC contiguous elements through 16-byte LDS accesses (caller checks alignment)
template <typename T, int NC>
__device__ __forceinline__ void load16(const T* src, T* dst) {
  constexpr int W = sizeof(T) >= 16 ? 1 : 16 / (int)sizeof(T);
#pragma unroll
  for (int t = 0; t + W <= NC; t += W) {
    const float4 v = *reinterpret_cast<const float4*>(src + t);
    __builtin_memcpy(dst + t, &v, 16);
  }
}
template <typename T, int NC>
__device__ __forceinline__ void store16(T* dst, const T* src) {
  constexpr int W = sizeof(T) >= 16 ? 1 : 16 / (int)sizeof(T);
#pragma unroll
  for (int t = 0; t + W <= NC; t += W) {
    float4 v;
    __builtin_memcpy(&v, src + t, 16);
    *reinterpret_cast<float4*>(dst + t) = v;
  }
}

template <typename T, int NC>
__device__ int jacobi_rows_nc(T* X, int m, int n, int ldx, typename RealOf<T>::type tol,
                              int max_sweeps, int* sflag, int G, typename RealOf<T>::type* nrm) {
  typedef typename RealOf<T>::type R;
  const int tid = threadIdx.x;
  const int mp = m + (m & 1);
  const int npairs = mp >> 1;
  const int pr = tid / G, lane = tid - (tid / G) * G;
  const int per_pass = PEPS_NT / G;
  // lane owns the contiguous elements [lane*NC, lane*NC + NC) of both rows
  const int e0 = lane * NC;
  const bool full = e0 + NC <= n;
  // 16-byte accesses when every owned run is 16-byte aligned
  const bool vec = (NC * sizeof(T)) % 16 == 0 && (ldx * sizeof(T)) % 16 == 0 &&
                   (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // squared row norms, refreshed every sweep and then carried through the
    // rotations: a' = a - t |c|, b' = b + t |c|
    for (int i = tid; i < m; i += PEPS_NT) {
      R q2 = 0;
      for (int e = 0; e < n; ++e) q2 += abs2x(X[i * ldx + e]);
      nrm[i] = q2;
    }
    if (tid == 0) sflag[0] = 0;
    __syncthreads();
    for (int r = 0; r < mp - 1; ++r) {
      for (int pb = 0; pb < npairs; pb += per_pass) {
        const int pi = pb + pr;
        int p = -1, q = -1;
        if (pi < npairs) {
          if (pi == 0) {
            p = mp - 1;
            q = r;
          } else {
            p = r + pi;
            if (p >= mp - 1) p -= mp - 1;
            q = r - pi;
            if (q < 0) q += mp - 1;
          }
        }
        const bool act = (pi < npairs) && p < m && q < m;
        T xp[NC], xq[NC];
        T* rp = X + p * ldx + e0;
        T* rq = X + q * ldx + e0;
        if (act && full && vec) {
          load16<T, NC>(rp, xp);
          load16<T, NC>(rq, xq);
        } else if (act && full) {
#pragma unroll
          for (int t = 0; t < NC; ++t) {
            xp[t] = rp[t];
            xq[t] = rq[t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < NC; ++t) {
            const bool ok = act && e0 + t < n;
            xp[t] = ok ? rp[t] : T(0);
            xq[t] = ok ? rq[t] : T(0);
          }
        }
        T c = 0;
#pragma unroll
        for (int t = 0; t < NC; ++t) c += conjx(xp[t]) * xq[t];
        c = group_sum(c, G);
        const R a = act ? nrm[p] : R(0), b = act ? nrm[q] : R(0);
        // |c| (real: the signed value, whose sign the rotation absorbs)
        R cm;
        if constexpr (IsCplx<T>::value) cm = absx(c);
        else cm = c;
        if (act && cm != R(0) && cm * cm > tol * tol * (a * b)) {
          R zeta, az, t, cs;
          if constexpr (std::is_same<T, float>::value) {
            // FP32: hardware reciprocal and reciprocal square root (1 ulp);
            // the rotation only needs to be orthogonal to rounding
            zeta = (b - a) * (0.5f * __builtin_amdgcn_rcpf(cm));
            az = fabsf(zeta);
            if (az > 1.f / Eps<float>::v) t = 0.5f * __builtin_amdgcn_rcpf(zeta);
            else
              t = copysignf(__builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(1.f + zeta * zeta)),
                            zeta);
            cs = __builtin_amdgcn_rsqf(1.f + t * t);
          } else {
            zeta = (b - a) / (R(2) * cm);
            az = fabs(zeta);
            if (az > R(1) / Eps<R>::v) t = R(0.5) / zeta;
            else t = (zeta >= R(0) ? R(1) : R(-1)) / (az + sqrt(R(1) + zeta * zeta));
            cs = R(1) / sqrt(R(1) + t * t);
          }
          const R sn = cs * t;
          // complex: rotate (p, e* q) with e = c/|c|, which makes <p, e* q> real
          T sq, cq;
          if constexpr (IsCplx<T>::value) {
            const T ec = conjx(c) * (R(1) / cm);
            sq = ec * sn;
            cq = ec * cs;
          } else {
            sq = sn;
            cq = cs;
          }
          if (full) {
            T yp[NC], yq[NC];
#pragma unroll
            for (int u = 0; u < NC; ++u) {
              yp[u] = cs * xp[u] - sq * xq[u];
              yq[u] = sn * xp[u] + cq * xq[u];
            }
            if (vec) {
              store16<T, NC>(rp, yp);
              store16<T, NC>(rq, yq);
            } else {
#pragma unroll
              for (int u = 0; u < NC; ++u) {
                rp[u] = yp[u];
                rq[u] = yq[u];
              }
            }
          } else {
#pragma unroll
            for (int u = 0; u < NC; ++u)
              if (e0 + u < n) {
                rp[u] = cs * xp[u] - sq * xq[u];
                rq[u] = sn * xp[u] + cq * xq[u];
              }
          }
          if (lane == 0) {
            sflag[0] = 1;
            nrm[p] = a - t * cm;
            nrm[q] = b + t * cm;
          }
        }
      }
      __syncthreads();
    }
    const int f = sflag[0];
    __syncthreads();
    if (f == 0) return sweep + 1;
  }
  return -1;
}

// Real rows, m a power of two (4 <= m <= 64): the same one-sided Jacobi with
// the pairs of a sweep in recursive block order. For b = m/2, m/4, ..., 1 the
// rows fall into blocks of 2b; during b rounds the first half of each block
// (resident rows, held in the registers of one group for the whole phase)
// meets every row of the second half (travelling rows, read from LDS each
// round). A sweep is again m-1 rounds of m/2 disjoint pairs covering every
// pair once, but only the travelling row goes through LDS.
// Rotations are applied in scaled form (fast plane rotations, Gentleman;
// with the scales kept apart as in Anda and Park): row i is stored as
// X_i = d_i Y_i, and the rotation [c -s; s c] of rows p, q with t = s/c
// becomes Y_p -= (t d_q / d_p) Y_q, Y_q += (t d_p / d_q) Y_p, d_{p,q} *= c:
// one multiply-add per element instead of two. c >= 2^-1/2 and a row meets
// m-1 <= 63 partners per sweep, so a scale stays above 2^-32; the scales are
// folded back into the rows at the start of every sweep and on exit.
// t comes from t = sgn(b - a) 2 g / (|b - a| + sqrt((b - a)^2 + 4 g^2))
// (a, b the squared norms, g the inner product). nrm holds 2m reals: the
// squared norms of X, then the scales d.
template <typename T, int NC>
__device__ __noinline__ int jacobi_rows_blk(T* X, int m, int n, int ldx, T tol, int max_sweeps,
                                            int* sflag, int G, T* nrm) {
  static_assert(!IsCplx<T>::value, "scaled rotations are for real rows");
  T* dd = nrm + m;
  const int tid = threadIdx.x;
  const int npairs = m >> 1;
  const int pi = tid / G, lane = tid - (tid / G) * G;
  const bool grp = pi < npairs;
  const int e0 = lane * NC;
  const bool full = e0 + NC <= n;
  const bool vec = (NC * sizeof(T)) % 16 == 0 && (ldx * sizeof(T)) % 16 == 0 &&
                   (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  auto ld = [&](int row, T (&y)[NC]) __attribute__((always_inline)) {
    const T* src = X + row * ldx + e0;
    if (full && vec) {
      load16<T, NC>(src, y);
    } else {
#pragma unroll
      for (int u = 0; u < NC; ++u) y[u] = e0 + u < n ? src[u] : T(0);
    }
  };
  auto st = [&](int row, const T (&y)[NC]) __attribute__((always_inline)) {
    T* dst = X + row * ldx + e0;
    if (full && vec) {
      store16<T, NC>(dst, y);
    } else {
#pragma unroll
      for (int u = 0; u < NC; ++u)
        if (e0 + u < n) dst[u] = y[u];
    }
  };
  // fold the scales into the rows (X_i = d_i Y_i), refresh the squared norms
  auto fold = [&]() __attribute__((always_inline)) {
    if (grp) {
      for (int h = 0; h < 2; ++h) {
        const int row = 2 * pi + h;
        T y[NC];
        ld(row, y);
        const T d = dd[row];
        T q2 = 0;
#pragma unroll
        for (int u = 0; u < NC; ++u) {
          y[u] *= d;
          q2 += y[u] * y[u];
        }
        st(row, y);
        q2 = group_sum(q2, G);
        if (lane == 0) {
          nrm[row] = q2;
          dd[row] = T(1);
        }
      }
    }
    __syncthreads();
  };
  for (int i = tid; i < m; i += PEPS_NT) dd[i] = T(1);
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    fold();
    if (tid == 0) sflag[0] = 0;
    __syncthreads();
    for (int b = npairs; b >= 1; b >>= 1) {
      const int i = pi & (b - 1);
      const int base = 2 * (pi - i);  // first row of this group's block
      const int rr = base + i;        // resident row
      T yr[NC];
      T dr = 1, ar = 0;
      if (grp) {
        ld(rr, yr);
        dr = dd[rr];
        ar = nrm[rr];
      }
      bool moved = false;
      for (int k = 0; k < b; ++k) {
        const int q = base + b + ((i + k) & (b - 1));
        T yq[NC];
        T c = 0, dq = 1, bq = 0;
        if (grp) {
          ld(q, yq);
          dq = dd[q];
          bq = nrm[q];
#pragma unroll
          for (int u = 0; u < NC; ++u) c += yr[u] * yq[u];
        }
        c = group_sum(c, G) * (dr * dq);
        if (grp && c != T(0) && c * c > tol * tol * (ar * bq)) {
          const T dlt = bq - ar;
          T t, cs, idr, idq;
          if constexpr (std::is_same<T, float>::value) {
            // hardware reciprocal, square root and reciprocal square root
            // (1 ulp): the rotation only needs to be orthogonal to rounding
            const float h = __builtin_amdgcn_sqrtf(fmaf(dlt, dlt, 4.f * c * c));
            t = (dlt >= 0.f ? 2.f * c : -2.f * c) * __builtin_amdgcn_rcpf(fabsf(dlt) + h);
            cs = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));
            idr = __builtin_amdgcn_rcpf(dr);
            idq = __builtin_amdgcn_rcpf(dq);
          } else {
            const T h = sqrt(dlt * dlt + T(4) * c * c);
            t = (dlt >= T(0) ? T(2) * c : T(-2) * c) / (fabs(dlt) + h);
            cs = T(1) / sqrt(T(1) + t * t);
            idr = T(1) / dr;
            idq = T(1) / dq;
          }
          const T t1 = t * dq * idr, t2 = t * dr * idq;
#pragma unroll
          for (int u = 0; u < NC; ++u) {
            const T yp = yr[u];
            yr[u] = yp - t1 * yq[u];
            yq[u] = yq[u] + t2 * yp;
          }
          st(q, yq);
          dr *= cs;
          ar -= t * c;
          moved = true;
          if (lane == 0) {
            sflag[0] = 1;
            dd[q] = dq * cs;
            nrm[q] = bq + t * c;
          }
        }
        __syncthreads();
      }
      if (moved) {
        st(rr, yr);
        if (lane == 0) {
          dd[rr] = dr;
          nrm[rr] = ar;
        }
      }
      __syncthreads();
    }
    const int f = sflag[0];
    __syncthreads();
    if (f == 0) return sweep + 1;
  }
  fold();
  return -1;
}

// The block-order scaled Jacobi above with its shape fixed at compile time:
// MR FP32 rows of NR elements in LDS (row stride ldx a multiple of 4,
// 16-byte aligned), 256 threads, G = min(64, 512 / MR, NR) lanes per pair
// holding NC = NR / G elements each. Addressing is 32-bit LDS offsets with
// vector accesses, the phases and rounds have fixed trip counts, and the
// lane groups reduce with fixed DPP steps; the arithmetic and its order are
// those of jacobi_rows_blk, so the results are identical.
typedef float jf4 __attribute__((ext_vector_type(4)));
typedef float jf2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) float lds_float;
typedef __attribute__((address_space(3))) jf4 lds_jf4;
typedef __attribute__((address_space(3))) jf2 lds_jf2;
typedef __attribute__((address_space(3))) int lds_int;

template <int G>
__device__ __forceinline__ float gsum_fixed(float v) {
  if constexpr (G >= 2) v += dppx<0xB1>(v);
  if constexpr (G >= 4) v += dppx<0x4E>(v);
  if constexpr (G >= 8) v += dppx<0x141>(v);
  if constexpr (G >= 16) v += dppx<0x140>(v);
  if constexpr (G >= 32) v += shfl_xor_x(v, 16);
  if constexpr (G >= 64) v += shfl_xor_x(v, 32);
  return v;
}

template <int NC>
__device__ __forceinline__ void ld_fixed(const lds_float* src, float (&y)[NC]) {
  if constexpr (NC % 4 == 0) {
#pragma unroll
    for (int v = 0; v < NC / 4; ++v) {
      const jf4 t = ((const lds_jf4*)src)[v];
      y[4 * v] = t.x;
      y[4 * v + 1] = t.y;
      y[4 * v + 2] = t.z;
      y[4 * v + 3] = t.w;
    }
  } else if constexpr (NC == 2) {
    const jf2 t = *(const lds_jf2*)src;
    y[0] = t.x;
    y[1] = t.y;
  } else {
#pragma unroll
    for (int u = 0; u < NC; ++u) y[u] = src[u];
  }
}
template <int NC>
__device__ __forceinline__ void st_fixed(lds_float* dst, const float (&y)[NC]) {
  if constexpr (NC % 4 == 0) {
#pragma unroll
    for (int v = 0; v < NC / 4; ++v) {
      jf4 t;
      t.x = y[4 * v];
      t.y = y[4 * v + 1];
      t.z = y[4 * v + 2];
      t.w = y[4 * v + 3];
      ((lds_jf4*)dst)[v] = t;
    }
  } else if constexpr (NC == 2) {
    jf2 t;
    t.x = y[0];
    t.y = y[1];
    *(lds_jf2*)dst = t;
  } else {
#pragma unroll
    for (int u = 0; u < NC; ++u) dst[u] = y[u];
  }
}

template <int MR, int NR>
__device__ __noinline__ int jacobi_fixed_lds(float* Xg, int ldx, float tol, int max_sweeps,
                                             int* sflag_g, float* nrm_g) {
  constexpr int NP = MR / 2;
  constexpr int G0 = 512 / MR < 64 ? 512 / MR : 64;
  constexpr int G = NR < G0 ? NR : G0;
  constexpr int NC = NR / G;
  static_assert(G * NC == NR && G * NP <= 256 && (MR & (MR - 1)) == 0, "shape");
  lds_float* X = (lds_float*)Xg;
  lds_int* sflag = (lds_int*)sflag_g;
  lds_float* nrm = (lds_float*)nrm_g;
  lds_float* dd = nrm + MR;
  const int tid = threadIdx.x;
  const int pi = tid / G, lane = tid % G;
  const bool grp = pi < NP;
  const int e0 = lane * NC;
  auto fold = [&]() __attribute__((always_inline)) {
    if (grp) {
      for (int h = 0; h < 2; ++h) {
        const int row = 2 * pi + h;
        float y[NC];
        ld_fixed<NC>(X + row * ldx + e0, y);
        const float d = dd[row];
        float q2 = 0.f;
#pragma unroll
        for (int u = 0; u < NC; ++u) {
          y[u] *= d;
          q2 += y[u] * y[u];
        }
        st_fixed<NC>(X + row * ldx + e0, y);
        q2 = gsum_fixed<G>(q2);
        if (lane == 0) {
          nrm[row] = q2;
          dd[row] = 1.f;
        }
      }
    }
    __syncthreads();
  };
  if (tid < MR) dd[tid] = 1.f;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    fold();
    if (tid == 0) sflag[0] = 0;
    __syncthreads();
#pragma unroll
    for (int b = NP; b >= 1; b >>= 1) {
      const int i = pi & (b - 1);
      const int base = 2 * (pi - i);
      const int rr = base + i;
      float yr[NC];
      float dr = 1.f, ar = 0.f;
      if (grp) {
        ld_fixed<NC>(X + rr * ldx + e0, yr);
        dr = dd[rr];
        ar = nrm[rr];
      }
      bool moved = false;
      for (int k = 0; k < b; ++k) {
        const int q = base + b + ((i + k) & (b - 1));
        float yq[NC];
        float c = 0.f, dq = 1.f, bq = 0.f;
        if (grp) {
          ld_fixed<NC>(X + q * ldx + e0, yq);
          dq = dd[q];
          bq = nrm[q];
#pragma unroll
          for (int u = 0; u < NC; ++u) c += yr[u] * yq[u];
        }
        c = gsum_fixed<G>(c) * (dr * dq);
        if (grp && c != 0.f && c * c > tol * tol * (ar * bq)) {
          const float dlt = bq - ar;
          const float h = __builtin_amdgcn_sqrtf(fmaf(dlt, dlt, 4.f * c * c));
          const float t = (dlt >= 0.f ? 2.f * c : -2.f * c) * __builtin_amdgcn_rcpf(fabsf(dlt) + h);
          const float cs = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));
          const float idr = __builtin_amdgcn_rcpf(dr);
          const float idq = __builtin_amdgcn_rcpf(dq);
          const float t1 = t * dq * idr, t2 = t * dr * idq;
#pragma unroll
          for (int u = 0; u < NC; ++u) {
            const float yp = yr[u];
            yr[u] = yp - t1 * yq[u];
            yq[u] = yq[u] + t2 * yp;
          }
          st_fixed<NC>(X + q * ldx + e0, yq);
          dr *= cs;
          ar -= t * c;
          moved = true;
          if (lane == 0) {
            sflag[0] = 1;
            dd[q] = dq * cs;
            nrm[q] = bq + t * c;
          }
        }
        __syncthreads();
      }
      if (moved) {
        st_fixed<NC>(X + rr * ldx + e0, yr);
        if (lane == 0) {
          dd[rr] = dr;
          nrm[rr] = ar;
        }
      }
      __syncthreads();
    }
    const int f = sflag[0];
    __syncthreads();
    if (f == 0) return sweep + 1;
  }
  fold();
  return -1;
}

// The same for the other shapes on that path (m a power of two, 4 <= m <=
// 64): G lanes per pair and NC elements per lane fixed at compile time,
// rows in LDS (16-byte aligned, ldx a multiple of 4), runtime m and n with
// the lanes past n masked. Same arithmetic and order as jacobi_rows_blk.
template <int NC, int G>
__device__ __noinline__ int jacobi_blk_lds(float* Xg, int m, int n, int ldx, float tol,
                                           int max_sweeps, int* sflag_g, float* nrm_g) {
  lds_float* X = (lds_float*)Xg;
  lds_int* sflag = (lds_int*)sflag_g;
  lds_float* nrm = (lds_float*)nrm_g;
  lds_float* dd = nrm + m;
  const int tid = threadIdx.x;
  const int npairs = m >> 1;
  const int pi = tid / G, lane = tid % G;
  const bool grp = pi < npairs;
  const int e0 = lane * NC;
  const bool full = e0 + NC <= n;
  auto ld = [&](int row, float (&y)[NC]) __attribute__((always_inline)) {
    const lds_float* src = X + row * ldx + e0;
    if (full) {
#pragma unroll
      for (int u = 0; u < NC; ++u) y[u] = src[u];
    } else {
#pragma unroll
      for (int u = 0; u < NC; ++u) y[u] = e0 + u < n ? src[u] : 0.f;
    }
  };
  auto st = [&](int row, const float (&y)[NC]) __attribute__((always_inline)) {
    lds_float* dst = X + row * ldx + e0;
    if (full) {
#pragma unroll
      for (int u = 0; u < NC; ++u) dst[u] = y[u];
    } else {
#pragma unroll
      for (int u = 0; u < NC; ++u)
        if (e0 + u < n) dst[u] = y[u];
    }
  };
  auto fold = [&]() __attribute__((always_inline)) {
    if (grp) {
      for (int h = 0; h < 2; ++h) {
        const int row = 2 * pi + h;
        float y[NC];
        ld(row, y);
        const float d = dd[row];
        float q2 = 0.f;
#pragma unroll
        for (int u = 0; u < NC; ++u) {
          y[u] *= d;
          q2 += y[u] * y[u];
        }
        st(row, y);
        q2 = gsum_fixed<G>(q2);
        if (lane == 0) {
          nrm[row] = q2;
          dd[row] = 1.f;
        }
      }
    }
    __syncthreads();
  };
  for (int i = tid; i < m; i += PEPS_NT) dd[i] = 1.f;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    fold();
    if (tid == 0) sflag[0] = 0;
    __syncthreads();
    for (int b = npairs; b >= 1; b >>= 1) {
      const int i = pi & (b - 1);
      const int base = 2 * (pi - i);
      const int rr = base + i;
      float yr[NC];
      float dr = 1.f, ar = 0.f;
      if (grp) {
        ld(rr, yr);
        dr = dd[rr];
        ar = nrm[rr];
      }
      bool moved = false;
      for (int k = 0; k < b; ++k) {
        const int q = base + b + ((i + k) & (b - 1));
        float yq[NC];
        float c = 0.f, dq = 1.f, bq = 0.f;
        if (grp) {
          ld(q, yq);
          dq = dd[q];
          bq = nrm[q];
#pragma unroll
          for (int u = 0; u < NC; ++u) c += yr[u] * yq[u];
        }
        c = gsum_fixed<G>(c) * (dr * dq);
        if (grp && c != 0.f && c * c > tol * tol * (ar * bq)) {
          const float dlt = bq - ar;
          const float h = __builtin_amdgcn_sqrtf(fmaf(dlt, dlt, 4.f * c * c));
          const float t = (dlt >= 0.f ? 2.f * c : -2.f * c) * __builtin_amdgcn_rcpf(fabsf(dlt) + h);
          const float cs = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));
          const float idr = __builtin_amdgcn_rcpf(dr);
          const float idq = __builtin_amdgcn_rcpf(dq);
          const float t1 = t * dq * idr, t2 = t * dr * idq;
#pragma unroll
          for (int u = 0; u < NC; ++u) {
            const float yp = yr[u];
            yr[u] = yp - t1 * yq[u];
            yq[u] = yq[u] + t2 * yp;
          }
          st(q, yq);
          dr *= cs;
          ar -= t * c;
          moved = true;
          if (lane == 0) {
            sflag[0] = 1;
            dd[q] = dq * cs;
            nrm[q] = bq + t * c;
          }
        }
        __syncthreads();
      }
      if (moved) {
        st(rr, yr);
        if (lane == 0) {
          dd[rr] = dr;
          nrm[rr] = ar;
        }
      }
      __syncthreads();
    }
    const int f = sflag[0];
    __syncthreads();
    if (f == 0) return sweep + 1;
  }
  fold();
  return -1;
}

// The same sweep for rows too long to hold in registers (nc > 32): each lane
// strides over the row twice, once for the dot product and once to rotate.
template <typename T>
__device__ int jacobi_rows_long(T* X, int m, int n, int ldx, typename RealOf<T>::type tol,
                                int max_sweeps, int* sflag, int G,
                                typename RealOf<T>::type* nrm) {
  typedef typename RealOf<T>::type R;
  const int tid = threadIdx.x;
  const int mp = m + (m & 1);
  const int npairs = mp >> 1;
  const int pr = tid / G, lane = tid - (tid / G) * G;
  const int per_pass = PEPS_NT / G;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int i = tid; i < m; i += PEPS_NT) {
      R q2 = 0;
      for (int e = 0; e < n; ++e) q2 += abs2x(X[i * ldx + e]);
      nrm[i] = q2;
    }
    if (tid == 0) sflag[0] = 0;
    __syncthreads();
    for (int r = 0; r < mp - 1; ++r) {
      for (int pb = 0; pb < npairs; pb += per_pass) {
        const int pi = pb + pr;
        int p = -1, q = -1;
        if (pi < npairs) {
          if (pi == 0) {
            p = mp - 1;
            q = r;
          } else {
            p = r + pi;
            if (p >= mp - 1) p -= mp - 1;
            q = r - pi;
            if (q < 0) q += mp - 1;
          }
        }
        const bool act = (pi < npairs) && p < m && q < m;
        T* rp = X + (act ? p : 0) * ldx;
        T* rq = X + (act ? q : 0) * ldx;
        T c = 0;
        if (act)
          for (int e = lane; e < n; e += G) c += conjx(rp[e]) * rq[e];
        c = group_sum(c, G);
        const R a = act ? nrm[p] : R(0), b = act ? nrm[q] : R(0);
        R cm;
        if constexpr (IsCplx<T>::value) cm = absx(c);
        else cm = c;
        if (act && cm != R(0) && fabs(cm) > tol * sqrt(a * b)) {
          const R zeta = (b - a) / (R(2) * cm);
          const R az = fabs(zeta);
          R t;
          if (az > R(1) / Eps<R>::v) t = R(0.5) / zeta;
          else t = (zeta >= R(0) ? R(1) : R(-1)) / (az + sqrt(R(1) + zeta * zeta));
          const R cs = R(1) / sqrt(R(1) + t * t);
          const R sn = cs * t;
          T sq, cq;
          if constexpr (IsCplx<T>::value) {
            const T ec = conjx(c) * (R(1) / cm);
            sq = ec * sn;
            cq = ec * cs;
          } else {
            sq = sn;
            cq = cs;
          }
          for (int e = lane; e < n; e += G) {
            const T xp = rp[e], xq = rq[e];
            rp[e] = cs * xp - sq * xq;
            rq[e] = sn * xp + cq * xq;
          }
          if (lane == 0) {
            sflag[0] = 1;
            nrm[p] = a - t * cm;
            nrm[q] = b + t * cm;
          }
        }
      }
      __syncthreads();
    }
    const int f = sflag[0];
    __syncthreads();
    if (f == 0) return sweep + 1;
  }
  return -1;
}

template <typename T>
__device__ int jacobi_rows(T* X, int m, int n, int ldx, typename RealOf<T>::type tol,
                           int max_sweeps, int* sflag, typename RealOf<T>::type* nrm) {
  if (m < 2) return 0;
  const int npairs = (m + (m & 1)) >> 1;
  int G = 64;
  while (G > 1 && G * npairs > PEPS_NT) G >>= 1;
  const int nc = (n + G - 1) / G;
  // FP32 rows (FP32 and BF16 modes) take the block order with scaled
  // rotations; in FP64 its two extra divisions per rotation cost more than
  // the LDS traffic it saves
  if constexpr (std::is_same<T, float>::value) {
    if (m == 64 && n == 64 && PEPS_NT == 256 && (ldx & 3) == 0 &&
        (reinterpret_cast<uintptr_t>(X) & 15) == 0 &&
        __builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)X))
      return jacobi_fixed_lds<64, 64>(X, ldx, tol, max_sweeps, sflag, nrm);
    if (m >= 4 && m <= 64 && (m & (m - 1)) == 0 && PEPS_NT == 256 && (ldx & 3) == 0 &&
        (reinterpret_cast<uintptr_t>(X) & 15) == 0 &&
        __builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)X)) {
      if (m == 16 && n == 64) return jacobi_fixed_lds<16, 64>(X, ldx, tol, max_sweeps, sflag, nrm);
      if (m == 16 && n == 16) return jacobi_fixed_lds<16, 16>(X, ldx, tol, max_sweeps, sflag, nrm);
      if (m == 4 && n == 64) return jacobi_fixed_lds<4, 64>(X, ldx, tol, max_sweeps, sflag, nrm);
      if (m == 4 && n == 4) return jacobi_fixed_lds<4, 4>(X, ldx, tol, max_sweeps, sflag, nrm);
      if (m == 32 && n == 64) return jacobi_fixed_lds<32, 64>(X, ldx, tol, max_sweeps, sflag, nrm);
      if (G == 64 && nc == 1)
        return jacobi_blk_lds<1, 64>(X, m, n, ldx, tol, max_sweeps, sflag, nrm);
      if (G == 32 && nc == 1)
        return jacobi_blk_lds<1, 32>(X, m, n, ldx, tol, max_sweeps, sflag, nrm);
      if (G == 32 && nc == 2)
        return jacobi_blk_lds<2, 32>(X, m, n, ldx, tol, max_sweeps, sflag, nrm);
      if (G == 16 && nc <= 4)
        return jacobi_blk_lds<4, 16>(X, m, n, ldx, tol, max_sweeps, sflag, nrm);
      if (G == 8 && nc <= 8)
        return jacobi_blk_lds<8, 8>(X, m, n, ldx, tol, max_sweeps, sflag, nrm);
    }
    if (m >= 4 && m <= 64 && (m & (m - 1)) == 0) {
      if (nc <= 4) return jacobi_rows_blk<T, 4>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
      if (nc <= 8) return jacobi_rows_blk<T, 8>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
    }
  }
  if (nc <= 1) return jacobi_rows_nc<T, 1>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
  if (nc <= 2) return jacobi_rows_nc<T, 2>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
  if (nc <= 4) return jacobi_rows_nc<T, 4>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
  if (nc <= 8) return jacobi_rows_nc<T, 8>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
  if (nc <= 16) return jacobi_rows_nc<T, 16>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
  // FP32 rows: the 32-element form would set the register budget (and so
  // the occupancy) of every kernel that can call it
  if constexpr (!std::is_same<T, float>::value) {
    if (nc <= 32) return jacobi_rows_nc<T, 32>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
  }
  return jacobi_rows_long<T>(X, m, n, ldx, tol, max_sweeps, sflag, G, nrm);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) from its published definition.
// ---------------------------------------------------------------------------
struct u4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u4 philox(u4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    u4 o;
    o.x = hi1 ^ c.y ^ k0;
    o.y = lo1;
    o.z = hi0 ^ c.w ^ k1;
    o.w = lo0;
    c = o;
  }
  return c;
}

__device__ __forceinline__ double philox_uniform(uint32_t x0, uint32_t x1) {
  const uint64_t v = ((uint64_t)x1 << 32) | x0;
  return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace pm
