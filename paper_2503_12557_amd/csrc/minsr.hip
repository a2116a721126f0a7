// minSR step (Sec. "Reformulation of the imaginary-time Schroedinger
// equation for sampling techniques", Eqs. tdvp and tdvp_fast) in FP64:
//   m      = column means of O over the batch (zeros where p != s_xy),
//   a_s    = sum_k O_sk m_k,  |m|^2,
//   G      = O O^T computed from the compact rows with the physical-index
//            mask (only samples with equal s_xy share the parameters of
//            site (x, y)),
//   T      = (G - a 1^T - 1 a^T + |m|^2) / n + eps I   (= Obar Obar^T + eps I),
//   T      = L L^T by a blocked right-looking Cholesky,
//   y      = T^-1 ebar,  dtheta = Obar^T y.
// Complex parameters (complex modes) take the same steps with the Hermitian
// forms: a_s = sum_k O_sk conj(m_k), G = O O^H, T = L L^H and
// dtheta = Obar^H y; the scalar type S is double or cplx<double>.
#include "common.h"
#include "kernels.h"

namespace pm {

// FP64 scalar of the solve for an O element type
template <typename TO> struct SolveT { typedef double type; };
template <typename R> struct SolveT<cplx<R>> { typedef cplx<double> type; };

__device__ __forceinline__ double to_s(float v) { return (double)v; }
__device__ __forceinline__ double to_s(double v) { return v; }
template <typename R>
__device__ __forceinline__ cplx<double> to_s(cplx<R> v) {
  return cplx<double>((double)v.re, (double)v.im);
}

// dtheta / mean entries are (re, im) pairs for complex parameters
__device__ __forceinline__ void put(double* out, size_t k, double v) { out[k] = v; }
__device__ __forceinline__ void put(double* out, size_t k, cplx<double> v) {
  out[2 * k] = v.re;
  out[2 * k + 1] = v.im;
}

// m_k for every parameter k; one thread per compact index.
template <typename TO>
__global__ void k_colmean(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
                          const uint8_t* __restrict__ samples, int n,
                          typename SolveT<TO>::type* __restrict__ mean) {
  typedef typename SolveT<TO>::type S;
  const int jc = blockIdx.x * blockDim.x + threadIdx.x;
  if (jc >= L.n_compact) return;
  const int site = tab[L.off_csite + jc];
  const int j = jc - tab[L.off_compact + site];
  S acc0 = 0.0, acc1 = 0.0;
  for (int s = 0; s < n; ++s) {
    const S v = to_s(O[(size_t)s * L.n_compact + jc]);
    if (pbit(samples[(size_t)s * L.N + site])) acc1 += v;
    else acc0 += v;
  }
  const int off = tab[L.off_param + site], blk = tab[L.off_block + site];
  mean[off + j] = acc0 / (double)n;
  mean[off + blk + j] = acc1 / (double)n;
}

// a_s = sum_k O_sk conj(m_k) (block per sample); slot n holds |m|^2 (block n).
template <typename TO>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_proj_mean(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
            const uint8_t* __restrict__ samples, int n,
            const typename SolveT<TO>::type* __restrict__ mean,
            typename SolveT<TO>::type* __restrict__ a) {
  typedef typename SolveT<TO>::type S;
  __shared__ S red[8];
  const int s = blockIdx.x;
  S acc = 0.0;
  if (s < n) {
    for (int jc = threadIdx.x; jc < L.n_compact; jc += PEPS_NT) {
      const int site = tab[L.off_csite + jc];
      const int j = jc - tab[L.off_compact + site];
      const int p = pbit(samples[(size_t)s * L.N + site]);
      acc += to_s(O[(size_t)s * L.n_compact + jc]) *
             conjx(mean[tab[L.off_param + site] + p * tab[L.off_block + site] + j]);
    }
  } else {
    for (int k = threadIdx.x; k < L.n_params; k += PEPS_NT) acc += S(abs2x(mean[k]));
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) a[s] = acc;
}

// E statistics: ws[0] = mean Re E, ws[8] = mean Im E (complex parameters
// only; real ones use Re E), ws[1] = mean |E - <E>|^2.
template <bool CPLX>
__global__ void k_estats(const double* __restrict__ eloc, int n, double* __restrict__ ws,
                         int* __restrict__ bad) {
  __shared__ double red[8];
  double s = 0.0, si = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) {
    const double v = eloc[2 * i];
    if (!isfinite(v) || !isfinite(eloc[2 * i + 1])) atomicOr(bad, 1);
    s += v;
    if (CPLX) si += eloc[2 * i + 1];
  }
  s = block_sum(s, red);
  const double mu = s / n;
  double mi = 0.0;
  if (CPLX) mi = block_sum(si, red) / n;
  double q = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) {
    const double v = eloc[2 * i] - mu;
    q += v * v;
    if (CPLX) {
      const double w = eloc[2 * i + 1] - mi;
      q += w * w;
    }
  }
  q = block_sum(q, red);
  if (threadIdx.x == 0) {
    ws[0] = mu;
    ws[1] = q / n;
    ws[8] = mi;
  }
}

// Masked Gram G[s,s'] = sum_k O_sk conj(O_s'k) over compact columns, 64 x 64
// tiles of the lower triangle, 4 x 4 outputs per thread; written with the
// centring and eps already applied:
// T = (G - a_s - conj(a_s') + |m|^2)/n + eps delta.
#define GT 64
#define GK 16
template <typename TO>
__global__ void __launch_bounds__(256)
k_gram(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
       const uint8_t* __restrict__ samples, int n, const typename SolveT<TO>::type* __restrict__ a,
       double eps, typename SolveT<TO>::type* __restrict__ Tm) {
  typedef typename SolveT<TO>::type S;
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  __shared__ S As[GK][GT + 1], Bs[GK][GT + 1];
  __shared__ uint8_t Pa[GK][GT], Pb[GK][GT];
  const int tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;
  S acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  const int s0 = bi * GT, t0 = bj * GT;
  for (int k0 = 0; k0 < L.n_compact; k0 += GK) {
    for (int e = tid; e < GK * GT; e += 256) {
      const int kk = e / GT, r = e - kk * GT;  // r fastest: samples
      const int jc = k0 + kk;
      const int sa = s0 + r, sb = t0 + r;
      S va = 0.0, vb = 0.0;
      uint8_t pa = 0, pb = 0;
      if (jc < L.n_compact) {
        const int site = tab[L.off_csite + jc];
        if (sa < n) {
          va = to_s(O[(size_t)sa * L.n_compact + jc]);
          pa = pbit(samples[(size_t)sa * L.N + site]);
        }
        if (sb < n) {
          vb = conjx(to_s(O[(size_t)sb * L.n_compact + jc]));
          pb = pbit(samples[(size_t)sb * L.N + site]);
        }
      }
      As[kk][r] = va;
      Bs[kk][r] = vb;
      Pa[kk][r] = pa;
      Pb[kk][r] = pb;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < GK; ++kk) {
      S av[4], bv[4];
      uint8_t ap[4], bp[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        av[i] = As[kk][tr * 4 + i];
        ap[i] = Pa[kk][tr * 4 + i];
        bv[i] = Bs[kk][tc * 4 + i];
        bp[i] = Pb[kk][tc * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if constexpr (IsCplx<S>::value) {
            if (ap[i] == bp[j]) acc[i][j] += av[i] * bv[j];
          } else {
            acc[i][j] += (ap[i] == bp[j]) ? av[i] * bv[j] : 0.0;
          }
    }
    __syncthreads();
  }
  const S m2 = a[n];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = s0 + tr * 4 + i, t = t0 + tc * 4 + j;
      if (s < n && t < n && t <= s) {
        S v = (acc[i][j] - a[s] - conjx(a[t]) + m2) / (double)n;
        if (s == t) {
          v += S(eps);
          if constexpr (IsCplx<S>::value) v.im = 0.0;  // Hermitian diagonal
        }
        Tm[(size_t)s * n + t] = v;
        Tm[(size_t)t * n + s] = conjx(v);
      }
    }
}

// trace of T (before eps) into ws[2]
template <typename S>
__global__ void k_trace(const S* __restrict__ Tm, int n, double eps, double* __restrict__ ws) {
  __shared__ double red[8];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) s += realx(Tm[(size_t)i * n + i]) - eps;
  s = block_sum(s, red);
  if (threadIdx.x == 0) ws[2] = s;
}

// ---- blocked Cholesky T = L L^H, lower, in place on the full matrix ----
#define CB 64
// factor the diagonal block kb (one block of 256 threads, in LDS)
template <typename S>
__global__ void __launch_bounds__(256) k_chol_diag(S* __restrict__ A, int n, int kb,
                                                   double* __restrict__ ws) {
  __shared__ S Sd[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = (n - k0) < CB ? (n - k0) : CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    Sd[i][j] = A[(size_t)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    __shared__ double piv;
    if (tid == 0) {
      double d = realx(Sd[j][j]);
      if (!(d > 0.0)) {
        ws[4] = 1.0;  // not positive definite
        d = 1e-300;
      }
      piv = sqrt(d);
      if (piv < ws[5]) ws[5] = piv;
      Sd[j][j] = S(piv);
    }
    __syncthreads();
    const double ip = 1.0 / piv;
    for (int i = j + 1 + tid; i < nb; i += 256) {
      if constexpr (IsCplx<S>::value) Sd[i][j] = Sd[i][j] * ip;
      else Sd[i][j] /= piv;
    }
    __syncthreads();
    const int rem = nb - j - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int i = j + 1 + e / rem, c = j + 1 + e % rem;
      if (c <= i) Sd[i][c] -= Sd[i][j] * conjx(Sd[c][j]);
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    A[(size_t)(k0 + i) * n + k0 + j] = (j <= i) ? Sd[i][j] : S(0.0);
  }
}

// rows below the diagonal block: X L_kk^H = A_ik  (one thread per row)
template <typename S>
__global__ void __launch_bounds__(256) k_chol_trsm(S* __restrict__ A, int n, int kb) {
  __shared__ S Lk[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = (n - k0) < CB ? (n - k0) : CB;
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    Lk[i][j] = conjx(A[(size_t)(k0 + i) * n + k0 + j]);
  }
  __syncthreads();
  const int row = k0 + nb + blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  S x[CB];
  S* a = A + (size_t)row * n + k0;
#pragma unroll
  for (int j = 0; j < CB; ++j) x[j] = (j < nb) ? a[j] : S(0.0);
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    if (j < nb) {
      S v = x[j];
#pragma unroll
      for (int i = 0; i < CB; ++i)
        if (i < j) v -= x[i] * Lk[j][i];
      if constexpr (IsCplx<S>::value) x[j] = v * (1.0 / realx(Lk[j][j]));
      else x[j] = v / Lk[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < CB; ++j)
    if (j < nb) a[j] = x[j];
}

// trailing update A_ij -= L_ik conj(L_jk) for the lower triangle, 64 x 64 tiles
template <typename S>
__global__ void __launch_bounds__(256) k_chol_syrk(S* __restrict__ A, int n, int kb) {
  const int k0 = kb * CB;
  const int base = k0 + CB;
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  const int i0 = base + bi * GT, j0 = base + bj * GT;
  __shared__ S As[CB][GT + 1], Bs[CB][GT + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * GT; e += 256) {
    const int r = e / CB, kk = e - r * CB;
    As[kk][r] = (i0 + r < n) ? A[(size_t)(i0 + r) * n + k0 + kk] : S(0.0);
    Bs[kk][r] = (j0 + r < n) ? conjx(A[(size_t)(j0 + r) * n + k0 + kk]) : S(0.0);
  }
  __syncthreads();
  const int tr = tid / 16, tc = tid % 16;
  S acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int kk = 0; kk < CB; ++kk) {
    S av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      av[i] = As[kk][tr * 4 + i];
      bv[i] = Bs[kk][tc * 4 + i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = i0 + tr * 4 + i, c = j0 + tc * 4 + j;
      if (r < n && c < n && c <= r) A[(size_t)r * n + c] -= acc[i][j];
    }
}

// y = L^-H L^-1 ebar in one block: ebar = (E - <E>)/sqrt(n) (Re E for real
// parameters)
template <typename S>
__global__ void __launch_bounds__(256) k_chol_solve(const S* __restrict__ Lm, int n,
                                                    const double* __restrict__ eloc,
                                                    const double* __restrict__ ws,
                                                    S* __restrict__ y) {
  const int tid = threadIdx.x;
  const double isn = 1.0 / sqrt((double)n);
  for (int i = tid; i < n; i += 256) {
    if constexpr (IsCplx<S>::value)
      y[i] = S((eloc[2 * i] - ws[0]) * isn, (eloc[2 * i + 1] - ws[8]) * isn);
    else
      y[i] = (eloc[2 * i] - ws[0]) * isn;
  }
  __syncthreads();
  // forward: L z = ebar
  for (int j = 0; j < n; ++j) {
    __shared__ S yj;
    if (tid == 0) {
      if constexpr (IsCplx<S>::value) yj = y[j] * (1.0 / realx(Lm[(size_t)j * n + j]));
      else yj = y[j] / Lm[(size_t)j * n + j];
      y[j] = yj;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += 256) y[i] -= Lm[(size_t)i * n + j] * yj;
    __syncthreads();
  }
  // backward: L^H y = z
  for (int j = n - 1; j >= 0; --j) {
    __shared__ S yj;
    if (tid == 0) {
      if constexpr (IsCplx<S>::value) yj = y[j] * (1.0 / realx(Lm[(size_t)j * n + j]));
      else yj = y[j] / Lm[(size_t)j * n + j];
      y[j] = yj;
    }
    __syncthreads();
    for (int i = tid; i < j; i += 256) y[i] -= conjx(Lm[(size_t)j * n + i]) * yj;
    __syncthreads();
  }
}

// dtheta_k = (sum_s conj(O_sk) y_s - conj(m_k) sum_s y_s)/sqrt(n);
// certificate failure -> NaN
template <typename TO>
__global__ void k_dtheta(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
                         const uint8_t* __restrict__ samples, int n,
                         const typename SolveT<TO>::type* __restrict__ y,
                         const typename SolveT<TO>::type* __restrict__ mean,
                         const typename SolveT<TO>::type* __restrict__ sy_p,
                         const double* __restrict__ ws, double* __restrict__ dth) {
  typedef typename SolveT<TO>::type S;
  const int jc = blockIdx.x * blockDim.x + threadIdx.x;
  if (jc >= L.n_compact) return;
  const int site = tab[L.off_csite + jc];
  const int j = jc - tab[L.off_compact + site];
  const int off = tab[L.off_param + site], blk = tab[L.off_block + site];
  const bool fail = ws[6] != 0.0;
  S acc0 = 0.0, acc1 = 0.0;
  for (int s = 0; s < n; ++s) {
    const S v = conjx(to_s(O[(size_t)s * L.n_compact + jc])) * y[s];
    if (pbit(samples[(size_t)s * L.N + site])) acc1 += v;
    else acc0 += v;
  }
  const S sy = *sy_p;
  const double isn = 1.0 / sqrt((double)n);
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  const S d0 = (acc0 - conjx(mean[off + j]) * sy) * isn;
  const S d1 = (acc1 - conjx(mean[off + blk + j]) * sy) * isn;
  put(dth, off + j, fail ? S(nan) : d0);
  put(dth, off + blk + j, fail ? S(nan) : d1);
}

template <typename S>
__global__ void k_sum_y(const S* __restrict__ y, int n, S* __restrict__ out) {
  __shared__ S red[8];
  S s = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) s += y[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

// certificate: no eigenvalue of T + eps I is dropped if trace(T) + eps <= eps / rcond
// (a non-finite local energy, flagged by k_estats, fails it too: diag[3] = 2)
__global__ void k_certify(int n, double eps, double rcond, double* __restrict__ ws,
                          const int* __restrict__ bad, double* __restrict__ diag) {
  if (threadIdx.x != 0) return;
  const double bound = ws[2] + eps;
  const bool ok = (eps > 0.0) && (bound * rcond <= eps);
  ws[6] = ok ? 0.0 : 1.0;
  if (ws[4] != 0.0) ws[6] = 1.0;
  if (*bad) ws[6] = 1.0;
  diag[0] = bound;
  diag[1] = eps;
  diag[2] = 0.0;
  diag[3] = *bad ? 2.0 : ws[6];
  diag[4] = ws[0];
  diag[5] = ws[1];
  diag[6] = (double)n;
  diag[7] = ws[5];
}

// fresh state of a call: a kernel rather than a memset, so the whole step
// can be recorded into a graph and the workspace can be shared memory
__global__ void k_init_ws(double* ws, int* bad) {
  if (threadIdx.x == 0) {
    ws[4] = 0.0;
    ws[5] = 1e300;
    ws[6] = 0.0;
    *bad = 0;
  }
}

template <typename TO>
static hipError_t minsr_impl(const Lattice& L, const int* tab, const TO* O, const uint8_t* samples,
                             int n, const double* eloc, double eps, double rcond, double* dtheta,
                             double* diag, void* mean_v, void* Tm_v, void* vec_v,
                             hipStream_t st) {
  typedef typename SolveT<TO>::type S;
  S* mean = (S*)mean_v;
  S* Tm = (S*)Tm_v;
  // vec layout: a[n+1] | y[n] | sum y | ws[16] (FP64) | bad (int)
  S* a = (S*)vec_v;
  S* y = a + n + 1;
  S* sy = y + n;
  double* ws = (double*)(sy + 1);
  int* bad = (int*)(ws + 16);
  hipLaunchKernelGGL(k_init_ws, dim3(1), dim3(64), 0, st, ws, bad);
  const int cb = (L.n_compact + 255) / 256;
  hipLaunchKernelGGL(k_colmean<TO>, dim3(cb), dim3(256), 0, st, L, tab, O, samples, n, mean);
  hipLaunchKernelGGL(k_proj_mean<TO>, dim3(n + 1), dim3(256), 0, st, L, tab, O, samples, n,
                     (const S*)mean, a);
  hipLaunchKernelGGL(k_estats<IsCplx<S>::value>, dim3(1), dim3(256), 0, st, eloc, n, ws, bad);
  const int nt = (n + GT - 1) / GT;
  hipLaunchKernelGGL(k_gram<TO>, dim3(nt, nt), dim3(256), 0, st, L, tab, O, samples, n,
                     (const S*)a, eps, Tm);
  hipLaunchKernelGGL(k_trace<S>, dim3(1), dim3(256), 0, st, (const S*)Tm, n, eps, ws);
  const int nkb = (n + CB - 1) / CB;
  for (int kb = 0; kb < nkb; ++kb) {
    hipLaunchKernelGGL(k_chol_diag<S>, dim3(1), dim3(256), 0, st, Tm, n, kb, ws);
    const int rest = n - (kb + 1) * CB;
    if (rest > 0) {
      hipLaunchKernelGGL(k_chol_trsm<S>, dim3((rest + 255) / 256), dim3(256), 0, st, Tm, n, kb);
      const int nr = (rest + GT - 1) / GT;
      hipLaunchKernelGGL(k_chol_syrk<S>, dim3(nr, nr), dim3(256), 0, st, Tm, n, kb);
    }
  }
  hipLaunchKernelGGL(k_certify, dim3(1), dim3(64), 0, st, n, eps, rcond, ws, (const int*)bad,
                     diag);
  hipLaunchKernelGGL(k_chol_solve<S>, dim3(1), dim3(256), 0, st, (const S*)Tm, n, eloc,
                     (const double*)ws, y);
  hipLaunchKernelGGL(k_sum_y<S>, dim3(1), dim3(256), 0, st, (const S*)y, n, sy);
  hipLaunchKernelGGL(k_dtheta<TO>, dim3(cb), dim3(256), 0, st, L, tab, O, samples, n,
                     (const S*)y, (const S*)mean, (const S*)sy, (const double*)ws, dtheta);
  return hipGetLastError();
}

// bytes of the minSR workspaces: mean [N_p], T [n][n], vec
void minsr_ws_bytes(const Lattice& L, int mode, int n, size_t* mean, size_t* T, size_t* vec) {
  const size_t es = (mode == MODE_C128 || mode == MODE_C64) ? 16 : 8;
  *mean = (size_t)L.n_params * es;
  *T = (size_t)n * n * es;
  *vec = ((size_t)2 * n + 2) * es + 16 * sizeof(double) + 16;
}

// grad_k = sum_s g_s O_sk with O expanded from the compact rows (zero where
// p != s_xy): the vector-Jacobian product of ln Psi over a batch.
template <typename TO>
__global__ void k_vjp(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
                      const uint8_t* __restrict__ samples, int n, const double* __restrict__ g,
                      double* __restrict__ out) {
  const int jc = blockIdx.x * blockDim.x + threadIdx.x;
  if (jc >= L.n_compact) return;
  const int site = tab[L.off_csite + jc];
  const int j = jc - tab[L.off_compact + site];
  const int off = tab[L.off_param + site], blk = tab[L.off_block + site];
  double acc0 = 0.0, acc1 = 0.0;
  for (int s = 0; s < n; ++s) {
    const double v = (double)O[(size_t)s * L.n_compact + jc] * g[s];
    if (pbit(samples[(size_t)s * L.N + site])) acc1 += v;
    else acc0 += v;
  }
  out[off + j] = acc0;
  out[off + blk + j] = acc1;
}

hipError_t launch_vjp(const Lattice& L, const int* tab, int mode, const void* O,
                      const uint8_t* samples, int n, const double* g, double* out,
                      hipStream_t st) {
  const int cb = (L.n_compact + 255) / 256;
  if (mode == MODE_F64)
    hipLaunchKernelGGL(k_vjp<double>, dim3(cb), dim3(256), 0, st, L, tab, (const double*)O,
                       samples, n, g, out);
  else
    hipLaunchKernelGGL(k_vjp<float>, dim3(cb), dim3(256), 0, st, L, tab, (const float*)O,
                       samples, n, g, out);
  return hipGetLastError();
}

// Parameter update of the optimisation loop (Eq. tdvp): theta moves by
// -tau dtheta, element by element over the real (or interleaved complex)
// FP64 parameters; a step whose certificate failed leaves theta unchanged.
__global__ void k_theta_update(double* __restrict__ theta, const double* __restrict__ dtheta,
                               const double* __restrict__ diag, double tau, size_t m) {
  if (diag[3] != 0.0) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (size_t)gridDim.x * blockDim.x)
    theta[i] = fma(-tau, dtheta[i], theta[i]);
}

hipError_t launch_theta_update(double* theta, const double* dtheta, const double* diag,
                               double tau, size_t m, hipStream_t st) {
  const size_t blocks = (m + 255) / 256 < 1024 ? (m + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_theta_update, dim3(blocks > 0 ? (unsigned)blocks : 1u), dim3(256), 0, st,
                     theta, dtheta, diag, tau, m);
  return hipGetLastError();
}

hipError_t launch_minsr(const Lattice& L, const int* tab, int mode, const void* O,
                        const uint8_t* samples, int n, const double* eloc, double eps,
                        double rcond, double* dtheta, double* diag, void* ws_mean, void* ws_T,
                        void* ws_vec, hipStream_t st) {
  switch (mode) {
    case MODE_F64:
      return minsr_impl<double>(L, tab, (const double*)O, samples, n, eloc, eps, rcond, dtheta,
                                diag, ws_mean, ws_T, ws_vec, st);
    case MODE_C128:
      return minsr_impl<cplx<double>>(L, tab, (const cplx<double>*)O, samples, n, eloc, eps,
                                      rcond, dtheta, diag, ws_mean, ws_T, ws_vec, st);
    case MODE_C64:
      return minsr_impl<cplx<float>>(L, tab, (const cplx<float>*)O, samples, n, eloc, eps, rcond,
                                     dtheta, diag, ws_mean, ws_T, ws_vec, st);
    default:
      return minsr_impl<float>(L, tab, (const float*)O, samples, n, eloc, eps, rcond, dtheta,
                               diag, ws_mean, ws_T, ws_vec, st);
  }
}

}  // namespace pm
