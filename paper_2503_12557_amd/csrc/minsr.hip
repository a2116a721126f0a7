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
#include "common.h"
#include "kernels.h"

namespace pm {

// m_k for every parameter k; one thread per compact index.
template <typename TO>
__global__ void k_colmean(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
                          const uint8_t* __restrict__ samples, int n, double* __restrict__ mean) {
  const int jc = blockIdx.x * blockDim.x + threadIdx.x;
  if (jc >= L.n_compact) return;
  const int site = tab[L.off_csite + jc];
  const int j = jc - tab[L.off_compact + site];
  double acc0 = 0.0, acc1 = 0.0;
  for (int s = 0; s < n; ++s) {
    const double v = (double)O[(size_t)s * L.n_compact + jc];
    if (pbit(samples[(size_t)s * L.N + site])) acc1 += v;
    else acc0 += v;
  }
  const int off = tab[L.off_param + site], blk = tab[L.off_block + site];
  mean[off + j] = acc0 / n;
  mean[off + blk + j] = acc1 / n;
}

// a_s = sum_k O_sk m_k (block per sample); slot n holds |m|^2 (block n).
template <typename TO>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_proj_mean(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
            const uint8_t* __restrict__ samples, int n, const double* __restrict__ mean,
            double* __restrict__ a) {
  __shared__ double red[8];
  const int s = blockIdx.x;
  double acc = 0.0;
  if (s < n) {
    for (int jc = threadIdx.x; jc < L.n_compact; jc += PEPS_NT) {
      const int site = tab[L.off_csite + jc];
      const int j = jc - tab[L.off_compact + site];
      const int p = pbit(samples[(size_t)s * L.N + site]);
      acc += (double)O[(size_t)s * L.n_compact + jc] *
             mean[tab[L.off_param + site] + p * tab[L.off_block + site] + j];
    }
  } else {
    for (int k = threadIdx.x; k < L.n_params; k += PEPS_NT) acc += mean[k] * mean[k];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) a[s] = acc;
}

// E statistics: ws[0] = mean Re E, ws[1] = sum (Re E - mean)^2 / n.
__global__ void k_estats(const double* __restrict__ eloc, int n, double* __restrict__ ws,
                         int* __restrict__ bad) {
  __shared__ double red[8];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) {
    const double v = eloc[2 * i];
    if (!isfinite(v) || !isfinite(eloc[2 * i + 1])) atomicOr(bad, 1);
    s += v;
  }
  s = block_sum(s, red);
  const double mu = s / n;
  double q = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) {
    const double v = eloc[2 * i] - mu;
    q += v * v;
  }
  q = block_sum(q, red);
  if (threadIdx.x == 0) {
    ws[0] = mu;
    ws[1] = q / n;
  }
}

// Masked Gram G[s,s'] over compact columns, 64 x 64 tiles of the lower
// triangle, 4 x 4 outputs per thread; written with the centring and eps
// already applied: T = (G - a_s - a_s' + |m|^2)/n + eps delta.
#define GT 64
#define GK 16
template <typename TO>
__global__ void __launch_bounds__(256)
k_gram(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
       const uint8_t* __restrict__ samples, int n, const double* __restrict__ a, double eps,
       double* __restrict__ Tm) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  __shared__ double As[GK][GT + 1], Bs[GK][GT + 1];
  __shared__ uint8_t Pa[GK][GT], Pb[GK][GT];
  const int tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;
  double acc[4][4];
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
      double va = 0.0, vb = 0.0;
      uint8_t pa = 0, pb = 0;
      if (jc < L.n_compact) {
        const int site = tab[L.off_csite + jc];
        if (sa < n) {
          va = (double)O[(size_t)sa * L.n_compact + jc];
          pa = pbit(samples[(size_t)sa * L.N + site]);
        }
        if (sb < n) {
          vb = (double)O[(size_t)sb * L.n_compact + jc];
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
      double av[4], bv[4];
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
        for (int j = 0; j < 4; ++j) acc[i][j] += (ap[i] == bp[j]) ? av[i] * bv[j] : 0.0;
    }
    __syncthreads();
  }
  const double m2 = a[n];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = s0 + tr * 4 + i, t = t0 + tc * 4 + j;
      if (s < n && t < n && t <= s) {
        double v = (acc[i][j] - a[s] - a[t] + m2) / n;
        if (s == t) v += eps;
        Tm[(size_t)s * n + t] = v;
        Tm[(size_t)t * n + s] = v;
      }
    }
}

// trace of T (before eps) into ws[2], smallest diagonal into ws[3]
__global__ void k_trace(const double* __restrict__ Tm, int n, double eps, double* __restrict__ ws) {
  __shared__ double red[8];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) s += Tm[(size_t)i * n + i] - eps;
  s = block_sum(s, red);
  if (threadIdx.x == 0) ws[2] = s;
}

// ---- blocked Cholesky, lower, in place on the full symmetric matrix ----
#define CB 64
// factor the diagonal block kb (one block of 256 threads, in LDS)
__global__ void __launch_bounds__(256) k_chol_diag(double* __restrict__ A, int n, int kb,
                                                   double* __restrict__ ws) {
  __shared__ double S[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = (n - k0) < CB ? (n - k0) : CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    S[i][j] = A[(size_t)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    __shared__ double piv;
    if (tid == 0) {
      double d = S[j][j];
      if (!(d > 0.0)) {
        ws[4] = 1.0;  // not positive definite
        d = 1e-300;
      }
      piv = sqrt(d);
      if (piv < ws[5]) ws[5] = piv;
      S[j][j] = piv;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < nb; i += 256) S[i][j] /= piv;
    __syncthreads();
    const int rem = nb - j - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int i = j + 1 + e / rem, c = j + 1 + e % rem;
      if (c <= i) S[i][c] -= S[i][j] * S[c][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    A[(size_t)(k0 + i) * n + k0 + j] = (j <= i) ? S[i][j] : 0.0;
  }
}

// rows below the diagonal block: X L_kk^T = A_ik  (one thread per row)
__global__ void __launch_bounds__(256) k_chol_trsm(double* __restrict__ A, int n, int kb) {
  __shared__ double Lk[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = (n - k0) < CB ? (n - k0) : CB;
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    Lk[i][j] = A[(size_t)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  const int row = k0 + nb + blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  double x[CB];
  double* a = A + (size_t)row * n + k0;
#pragma unroll
  for (int j = 0; j < CB; ++j) x[j] = (j < nb) ? a[j] : 0.0;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    if (j < nb) {
      double v = x[j];
#pragma unroll
      for (int i = 0; i < CB; ++i)
        if (i < j) v -= x[i] * Lk[j][i];
      x[j] = v / Lk[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < CB; ++j)
    if (j < nb) a[j] = x[j];
}

// trailing update A_ij -= L_ik L_jk^T for the lower triangle, 64 x 64 tiles
__global__ void __launch_bounds__(256) k_chol_syrk(double* __restrict__ A, int n, int kb) {
  const int k0 = kb * CB;
  const int base = k0 + CB;
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  const int i0 = base + bi * GT, j0 = base + bj * GT;
  __shared__ double As[CB][GT + 1], Bs[CB][GT + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * GT; e += 256) {
    const int r = e / CB, kk = e - r * CB;
    As[kk][r] = (i0 + r < n) ? A[(size_t)(i0 + r) * n + k0 + kk] : 0.0;
    Bs[kk][r] = (j0 + r < n) ? A[(size_t)(j0 + r) * n + k0 + kk] : 0.0;
  }
  __syncthreads();
  const int tr = tid / 16, tc = tid % 16;
  double acc[4][4] = {};
  for (int kk = 0; kk < CB; ++kk) {
    double av[4], bv[4];
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

// y = L^-T L^-1 ebar in one block: ebar = (Re E - mean)/sqrt(n)
__global__ void __launch_bounds__(256) k_chol_solve(const double* __restrict__ Lm, int n,
                                                    const double* __restrict__ eloc,
                                                    const double* __restrict__ ws,
                                                    double* __restrict__ y) {
  const int tid = threadIdx.x;
  const double mu = ws[0], isn = 1.0 / sqrt((double)n);
  for (int i = tid; i < n; i += 256) y[i] = (eloc[2 * i] - mu) * isn;
  __syncthreads();
  // forward: L z = ebar
  for (int j = 0; j < n; ++j) {
    __shared__ double yj;
    if (tid == 0) {
      yj = y[j] / Lm[(size_t)j * n + j];
      y[j] = yj;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += 256) y[i] -= Lm[(size_t)i * n + j] * yj;
    __syncthreads();
  }
  // backward: L^T y = z
  for (int j = n - 1; j >= 0; --j) {
    __shared__ double yj;
    if (tid == 0) {
      yj = y[j] / Lm[(size_t)j * n + j];
      y[j] = yj;
    }
    __syncthreads();
    for (int i = tid; i < j; i += 256) y[i] -= Lm[(size_t)j * n + i] * yj;
    __syncthreads();
  }
}

// dtheta_k = (sum_s O_sk y_s - m_k sum_s y_s)/sqrt(n); certificate failure -> NaN
template <typename TO>
__global__ void k_dtheta(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
                         const uint8_t* __restrict__ samples, int n, const double* __restrict__ y,
                         const double* __restrict__ mean, const double* __restrict__ ws,
                         double* __restrict__ dth) {
  const int jc = blockIdx.x * blockDim.x + threadIdx.x;
  if (jc >= L.n_compact) return;
  const int site = tab[L.off_csite + jc];
  const int j = jc - tab[L.off_compact + site];
  const int off = tab[L.off_param + site], blk = tab[L.off_block + site];
  const bool fail = ws[6] != 0.0;
  double acc0 = 0.0, acc1 = 0.0;
  for (int s = 0; s < n; ++s) {
    const double v = (double)O[(size_t)s * L.n_compact + jc] * y[s];
    if (pbit(samples[(size_t)s * L.N + site])) acc1 += v;
    else acc0 += v;
  }
  const double sy = ws[7], isn = 1.0 / sqrt((double)n);
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  dth[off + j] = fail ? nan : (acc0 - mean[off + j] * sy) * isn;
  dth[off + blk + j] = fail ? nan : (acc1 - mean[off + blk + j] * sy) * isn;
}

__global__ void k_sum_y(const double* __restrict__ y, int n, double* __restrict__ ws) {
  __shared__ double red[8];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) s += y[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) ws[7] = s;
}

// certificate: no eigenvalue of T + eps I is dropped if trace(T) + eps <= eps / rcond
__global__ void k_certify(int n, double eps, double rcond, double* __restrict__ ws,
                          double* __restrict__ diag) {
  if (threadIdx.x != 0) return;
  const double bound = ws[2] + eps;
  const bool ok = (eps > 0.0) && (bound * rcond <= eps);
  ws[6] = ok ? 0.0 : 1.0;
  if (ws[4] != 0.0) ws[6] = 1.0;
  diag[0] = bound;
  diag[1] = eps;
  diag[2] = 0.0;
  diag[3] = ws[6];
  diag[4] = ws[0];
  diag[5] = ws[1];
  diag[6] = (double)n;
  diag[7] = ws[5];
}

__global__ void k_init_ws(double* ws) {
  if (threadIdx.x == 0) {
    ws[4] = 0.0;
    ws[5] = 1e300;
    ws[6] = 0.0;
  }
}

template <typename TO>
static hipError_t minsr_impl(const Lattice& L, const int* tab, const TO* O, const uint8_t* samples,
                             int n, const double* eloc, double eps, double rcond, double* dtheta,
                             double* diag, double* mean, double* Tm, double* vec,
                             hipStream_t st) {
  // vec layout: a[n+1] | y[n] | ws[16] | bad (int)
  double* a = vec;
  double* y = vec + n + 1;
  double* ws = y + n;
  int* bad = (int*)(ws + 16);
  hipLaunchKernelGGL(k_init_ws, dim3(1), dim3(64), 0, st, ws);
  hipMemsetAsync(bad, 0, sizeof(int), st);
  const int cb = (L.n_compact + 255) / 256;
  hipLaunchKernelGGL(k_colmean<TO>, dim3(cb), dim3(256), 0, st, L, tab, O, samples, n, mean);
  hipLaunchKernelGGL(k_proj_mean<TO>, dim3(n + 1), dim3(256), 0, st, L, tab, O, samples, n,
                     (const double*)mean, a);
  hipLaunchKernelGGL(k_estats, dim3(1), dim3(256), 0, st, eloc, n, ws, bad);
  const int nt = (n + GT - 1) / GT;
  hipLaunchKernelGGL(k_gram<TO>, dim3(nt, nt), dim3(256), 0, st, L, tab, O, samples, n,
                     (const double*)a, eps, Tm);
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, st, (const double*)Tm, n, eps, ws);
  const int nkb = (n + CB - 1) / CB;
  for (int kb = 0; kb < nkb; ++kb) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, Tm, n, kb, ws);
    const int rest = n - (kb + 1) * CB;
    if (rest > 0) {
      hipLaunchKernelGGL(k_chol_trsm, dim3((rest + 255) / 256), dim3(256), 0, st, Tm, n, kb);
      const int nr = (rest + GT - 1) / GT;
      hipLaunchKernelGGL(k_chol_syrk, dim3(nr, nr), dim3(256), 0, st, Tm, n, kb);
    }
  }
  hipLaunchKernelGGL(k_certify, dim3(1), dim3(64), 0, st, n, eps, rcond, ws, diag);
  hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(256), 0, st, (const double*)Tm, n, eloc,
                     (const double*)ws, y);
  hipLaunchKernelGGL(k_sum_y, dim3(1), dim3(256), 0, st, (const double*)y, n, ws);
  hipLaunchKernelGGL(k_dtheta<TO>, dim3(cb), dim3(256), 0, st, L, tab, O, samples, n,
                     (const double*)y, (const double*)mean, (const double*)ws, dtheta);
  return hipGetLastError();
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

hipError_t launch_minsr(const Lattice& L, const int* tab, int mode, const void* O,
                        const uint8_t* samples, int n, const double* eloc, double eps,
                        double rcond, double* dtheta, double* diag, double* ws_mean,
                        double* ws_T, double* ws_vec, hipStream_t st) {
  if (mode == MODE_F64)
    return minsr_impl<double>(L, tab, (const double*)O, samples, n, eloc, eps, rcond, dtheta, diag,
                              ws_mean, ws_T, ws_vec, st);
  return minsr_impl<float>(L, tab, (const float*)O, samples, n, eloc, eps, rcond, dtheta, diag,
                           ws_mean, ws_T, ws_vec, st);
}

}  // namespace pm
