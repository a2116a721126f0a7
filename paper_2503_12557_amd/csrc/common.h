// Shared device-side definitions: precision modes, block reductions,
// workgroup-level small linear algebra on LDS (Householder QR, one-sided
// Jacobi, strided GEMM) and the lattice tables the kernels read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PEPS_BLOCK 256

namespace pm {

// ---------------------------------------------------------------------------
// Precision modes. T is the arithmetic type of contractions, QR and SVD.
// In BF16 mode every contraction operand is rounded to bfloat16 (round to
// nearest even) and the products are accumulated in FP32.
// ---------------------------------------------------------------------------
enum Mode { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16 = 2 };

template <int M> struct ModeT;
template <> struct ModeT<MODE_F64> { typedef double T; };
template <> struct ModeT<MODE_F32> { typedef float T; };
template <> struct ModeT<MODE_BF16> { typedef float T; };

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

// Physical index of a site; masked so a malformed sample byte cannot index
// outside the parameter block (samples with values > 1 are flagged).
__device__ __forceinline__ int pbit(uint8_t v) { return v & 1; }

template <typename T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };
template <> struct Eps<float> { static constexpr float v = 1.1920929e-7f; };

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
};

__device__ __forceinline__ int slot_top(const Lattice& L, int x) { return x; }
__device__ __forceinline__ int slot_bottom(const Lattice& L, int x) { return L.Lx - 1 + (x - 1); }

// ---------------------------------------------------------------------------
// Reductions over the 256-thread block. `red` is LDS scratch of >= 8 values.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
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
  for (int i = 0; i < PEPS_BLOCK / 64; ++i) s += red[i];
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
  for (int i = 1; i < PEPS_BLOCK / 64; ++i) s = red[i] > s ? red[i] : s;
  __syncthreads();
  return s;
}

// Sum over groups of G consecutive lanes (G a power of two, G <= 64).
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
  for (int o = G >> 1; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Strided GEMM over the block: C[i,j] (+)= sum_k A[i*sai + k*sak] * B[k*sbk + j*sbj]
// written to C[i*sci + j*scj]. Operands may live in LDS or global memory.
// The caller synchronises before reading C.
// ---------------------------------------------------------------------------
template <int M, typename T>
__device__ void gemm(int m, int n, int k, const T* A, int sai, int sak, const T* B, int sbk,
                     int sbj, T* C, int sci, int scj, bool acc) {
  const int tot = m * n;
  for (int idx = threadIdx.x; idx < tot; idx += PEPS_BLOCK) {
    const int i = idx / n, j = idx - (idx / n) * n;
    T s = 0;
    const T* a = A + i * sai;
    const T* b = B + j * sbj;
    for (int kk = 0; kk < k; ++kk) s += opnd<M>(a[kk * sak]) * opnd<M>(b[kk * sbk]);
    T* c = C + i * sci + j * scj;
    *c = acc ? *c + s : s;
  }
}

// ---------------------------------------------------------------------------
// Householder QR of the LDS matrix A (m x n, row stride lda), keeping only R:
// on exit rows 0..min(m,n)-1 hold R (upper trapezoidal) and the rest of
// column j below the diagonal is zero. v: LDS scratch of m, w: of n,
// red: reduction scratch.
// ---------------------------------------------------------------------------
template <typename T>
__device__ void house_qr_r(T* A, int m, int n, int lda, T* v, T* w, T* red) {
  const int tid = threadIdx.x;
  const int kmax = m < n ? m : n;
  for (int j = 0; j < kmax; ++j) {
    T s = 0;
    for (int i = j + 1 + tid; i < m; i += PEPS_BLOCK) {
      const T a = A[i * lda + j];
      s += a * a;
    }
    s = block_sum(s, red);
    if (s == T(0)) continue;  // block-uniform
    const T ajj = A[j * lda + j];
    const T nrm = sqrt(ajj * ajj + s);
    const T alpha = ajj > T(0) ? -nrm : nrm;
    const T v0 = ajj - alpha;
    const T tau = T(2) / (v0 * v0 + s);
    for (int i = j + tid; i < m; i += PEPS_BLOCK) v[i] = (i == j) ? v0 : A[i * lda + j];
    __syncthreads();
    const int nc = n - j - 1;
    if (nc > 0) {
      int G = 64;
      while (G > 1 && G * nc > PEPS_BLOCK) G >>= 1;
      const int ncol_par = PEPS_BLOCK / G;
      const int g = tid / G, lane = tid - (tid / G) * G;
      for (int c0 = 0; c0 < nc; c0 += ncol_par) {
        const int c = j + 1 + c0 + g;
        T p = 0;
        if (c0 + g < nc)
          for (int i = j + lane; i < m; i += G) p += v[i] * A[i * lda + c];
        p = group_sum(p, G);
        if (lane == 0 && c0 + g < nc) w[c] = tau * p;
      }
      __syncthreads();
      const int nr = m - j;
      const int tot = nr * nc;
      for (int idx = tid; idx < tot; idx += PEPS_BLOCK) {
        const int i = j + idx / nc, c = j + 1 + idx - (idx / nc) * nc;
        A[i * lda + c] -= v[i] * w[c];
      }
    }
    __syncthreads();
    if (tid == 0) A[j * lda + j] = alpha;
    for (int i = j + 1 + tid; i < m; i += PEPS_BLOCK) A[i * lda + j] = T(0);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi on the m rows of the LDS matrix X (m x n, row
// stride ldx, m <= n, m <= 2*PEPS_BLOCK): rotates pairs of rows until every
// pair is orthogonal to relative tolerance tol. Pairs follow the circle
// (round-robin) schedule, m-1 rounds of m/2 disjoint pairs per sweep.
// Returns the number of sweeps used, or -1 if max_sweeps was reached.
// ---------------------------------------------------------------------------
template <typename T>
__device__ int jacobi_rows(T* X, int m, int n, int ldx, T tol, int max_sweeps, int* sflag) {
  const int tid = threadIdx.x;
  const int mp = m + (m & 1);
  const int npairs = mp >> 1;
  if (m < 2) return 0;
  int G = 64;
  while (G > 1 && G * npairs > PEPS_BLOCK) G >>= 1;
  const int pr = tid / G, lane = tid - (tid / G) * G;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int r = 0; r < mp - 1; ++r) {
      for (int pb = 0; pb < npairs; pb += PEPS_BLOCK / G) {
        const int pi = pb + pr;
        int p = -1, q = -1;
        if (pi < npairs) {
          if (pi == 0) {
            p = mp - 1;
            q = r;
          } else {
            p = (r + pi) % (mp - 1);
            q = (r - pi + (mp - 1)) % (mp - 1);
          }
        }
        const bool act = (pi < npairs) && p < m && q < m;
        T a = 0, b = 0, c = 0;
        if (act) {
          for (int e = lane; e < n; e += G) {
            const T xp = X[p * ldx + e], xq = X[q * ldx + e];
            a += xp * xp;
            b += xq * xq;
            c += xp * xq;
          }
        }
        a = group_sum(a, G);
        b = group_sum(b, G);
        c = group_sum(c, G);
        if (act && c != T(0) && fabs(c) > tol * sqrt(a * b)) {
          const T zeta = (b - a) / (T(2) * c);
          const T az = fabs(zeta);
          T t;
          if (az > T(1) / Eps<T>::v) t = T(0.5) / zeta;
          else t = (zeta >= T(0) ? T(1) : T(-1)) / (az + sqrt(T(1) + zeta * zeta));
          const T cs = T(1) / sqrt(T(1) + t * t);
          const T sn = cs * t;
          for (int e = lane; e < n; e += G) {
            const T xp = X[p * ldx + e], xq = X[q * ldx + e];
            X[p * ldx + e] = cs * xp - sn * xq;
            X[q * ldx + e] = sn * xp + cs * xq;
          }
          if (lane == 0) *sflag = 1;
        }
      }
      __syncthreads();
    }
    const int f = *sflag;
    __syncthreads();
    if (f == 0) return sweep + 1;
  }
  return -1;
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
