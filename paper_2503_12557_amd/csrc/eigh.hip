// Eigendecomposition solve of the minSR system (Sec. "Reformulation of the
// imaginary-time Schroedinger equation for sampling techniques",
// Eq. tdvp_fast): y = (T + eps I)^+ ebar with the eigenvalues at or below
// rcond * (largest) dropped, for a Hermitian (or real symmetric) FP64 T
// already holding T + eps I.
//
//   1. T = Q Tri Q^H by Householder reflectors (Tri real symmetric
//      tridiagonal: each reflector is chosen so that the new subdiagonal
//      entry is real), one column at a time over the whole device;
//   2. the eigenvalues of Tri by bisection on Sturm counts;
//   3. the eigenvectors Z of Tri for the kept eigenvalues by inverse
//      iteration, orthogonalised inside clusters of close eigenvalues;
//   4. y = Q Z diag(1/lambda) Z^T Q^H ebar: only products of vectors with
//      Q, Z and Z^T, so no n x n back-transformation is formed.
//
// Every kernel reads the device flag `on` first and returns at once when it
// is zero, so the path can be queued behind the Cholesky certificate without
// a host round trip (it then runs only when the certificate failed).
#include "common.h"
#include "kernels.h"

namespace pm {

#define EIG_EPS 2.220446049250313e-16

__device__ __forceinline__ double cabs2(double v) { return v * v; }
__device__ __forceinline__ double cabs2(cplx<double> v) { return v.re * v.re + v.im * v.im; }

// 1a. reflector of column k: x = T[k+1.., k] (read as the conjugate of row
// k, which the updates keep equal to it), H^H x = beta e1 with beta real,
// H = I - tau v v^H, v[0] = 1. v is stored over row k (entries k+1..),
// which no later step reads as part of T.
template <typename S>
__global__ void __launch_bounds__(256) k_hh_reflect(S* __restrict__ T, int n, int k,
                                                    const int* __restrict__ on,
                                                    S* __restrict__ tau, double* __restrict__ d,
                                                    double* __restrict__ e) {
  if (!*on) return;
  __shared__ double red[4];
  S* row = T + (size_t)k * n;
  const int m = n - k - 1;
  double x2 = 0.0;
  for (int i = 1 + threadIdx.x; i < m; i += 256) x2 += cabs2(row[k + 1 + i]);
  x2 = block_sum(x2, red);
  const S alpha = conjx(row[k + 1]);
  double ar, ai;
  if constexpr (IsCplx<S>::value) {
    ar = alpha.re;
    ai = alpha.im;
  } else {
    ar = alpha;
    ai = 0.0;
  }
  S t = S(0.0), scal = S(0.0);
  double beta = ar;
  if (x2 != 0.0 || ai != 0.0) {
    beta = -copysign(sqrt(ar * ar + ai * ai + x2), ar);
    t = (S(beta) - alpha) * (1.0 / beta);
    const S den = alpha - S(beta);
    if constexpr (IsCplx<S>::value) scal = conjx(den) * (1.0 / cabs2(den));
    else scal = 1.0 / den;
  }
  __syncthreads();  // every lane has read row[k + 1] (alpha)
  for (int i = 1 + threadIdx.x; i < m; i += 256) row[k + 1 + i] = conjx(row[k + 1 + i]) * scal;
  if (threadIdx.x == 0) {
    row[k + 1] = S(1.0);
    tau[k] = t;
    d[k] = realx(row[k]);
    e[k] = beta;
    if (k == n - 2) d[n - 1] = realx(T[(size_t)(n - 1) * n + n - 1]);
  }
}

// 1b. p = tau A22 v over rows k+1.., one wave per row
template <typename S>
__global__ void __launch_bounds__(256) k_hh_symv(const S* __restrict__ T, int n, int k,
                                                 const int* __restrict__ on,
                                                 const S* __restrict__ tau, S* __restrict__ p) {
  if (!*on) return;
  const int lane = threadIdx.x & 63;
  const int i = k + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const S* v = T + (size_t)k * n;
  const S* r = T + (size_t)i * n;
  S acc = S(0.0);
  for (int j = k + 1 + lane; j < n; j += 64) acc += r[j] * v[j];
  acc = wave_sum(acc);
  if (lane == 0) p[i] = tau[k] * acc;
}

// 1c. A22 -= w v^H + v w^H with w = p - (conj(tau)/2)(v^H p) v; each
// workgroup takes 64 rows x 256 columns and forms the scalar itself
template <typename S>
__global__ void __launch_bounds__(256) k_hh_update(S* __restrict__ T, int n, int k,
                                                   const int* __restrict__ on,
                                                   const S* __restrict__ tau,
                                                   const S* __restrict__ p) {
  if (!*on) return;
  __shared__ S red[4];
  __shared__ S wr[64], vr[64];
  const int tid = threadIdx.x;
  const S* v = T + (size_t)k * n;
  S dot = S(0.0);
  for (int i = k + 1 + tid; i < n; i += 256) dot += conjx(v[i]) * p[i];
  dot = block_sum(dot, red);
  const S kc = conjx(tau[k]) * dot * 0.5;
  const int r0 = k + 1 + blockIdx.y * 64, c = k + 1 + blockIdx.x * 256 + tid;
  if (tid < 64) {
    const int i = r0 + tid;
    const S vi = i < n ? v[i] : S(0.0);
    vr[tid] = vi;
    wr[tid] = i < n ? p[i] - kc * vi : S(0.0);
  }
  __syncthreads();
  if (c >= n) return;
  const S vc = conjx(v[c]);
  const S wc = conjx(p[c] - kc * v[c]);
  const int rows = min(64, n - r0);
  for (int r = 0; r < rows; ++r) {
    S* a = T + (size_t)(r0 + r) * n + c;
    *a -= wr[r] * vc + vr[r] * wc;
  }
}

// number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence)
__device__ __forceinline__ int sturm_count(const double* __restrict__ d,
                                           const double* __restrict__ e, int n, double x,
                                           double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int j = 1; j < n; ++j) {
    q = d[j] - x - e[j - 1] * e[j - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// 2. eigenvalue i (ascending) by bisection, one thread each
__global__ void __launch_bounds__(256) k_tri_bisect(const double* __restrict__ d,
                                                    const double* __restrict__ e, int n,
                                                    const int* __restrict__ on,
                                                    double* __restrict__ lam) {
  if (!*on) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double lo = 1e308, hi = -1e308, emax = 1.0;
  for (int j = 0; j < n; ++j) {
    const double r = (j > 0 ? fabs(e[j - 1]) : 0.0) + (j < n - 1 ? fabs(e[j]) : 0.0);
    lo = fmin(lo, d[j] - r);
    hi = fmax(hi, d[j] + r);
    if (j < n - 1) emax = fmax(emax, e[j] * e[j]);
  }
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = 2.2250738585072014e-308 * emax;
  lo -= 2.0 * EIG_EPS * tnorm + pivmin;
  hi += 2.0 * EIG_EPS * tnorm + pivmin;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hi - lo <= 2.0 * EIG_EPS * fmax(fabs(lo), fabs(hi)) + pivmin || mid <= lo ||
        mid >= hi)
      break;
    if (sturm_count(d, e, n, mid, pivmin) <= i) lo = mid;
    else hi = mid;
  }
  lam[i] = 0.5 * (lo + hi);
}

// deterministic start vector entry in (-1, 1) (splitmix64 of (j, k))
__device__ __forceinline__ double start_entry(int j, int k) {
  unsigned long long z = ((unsigned long long)j << 32 | (unsigned)k) + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// 3. eigenvectors of the kept eigenvalues: one wave per cluster (a run of
// kept eigenvalues with neighbouring gaps <= 1e-6 |Tri|), started by the
// wave of its first member. Inverse iteration leaves in the vector of an
// eigenvalue at gap g from another about u |Tri| / g of the other's vector,
// and in y an error of the same relative size; gaps above 1e-6 |Tri| keep
// that near 1e-10 without orthogonalisation, while (near-)degenerate
// eigenvalues, such as the eps-shifted null space of a rank-deficient Gram,
// are orthogonalised. Each member: inverse iteration (Tri - s I) x = b
// with a partial-pivot LU formed row by row on lane 0 (U bands and d, e in
// LDS), the iterate orthogonalised against the cluster's earlier vectors
// and normalised; shifts of equal eigenvalues are separated by a few ulps
// of |Tri| so that successive members start from different solves.
#define EIG_ITERS 4
__global__ void __launch_bounds__(64) k_tri_vec(const double* __restrict__ dg,
                                                const double* __restrict__ eg, int n,
                                                const int* __restrict__ on,
                                                const double* __restrict__ lam, double rcond,
                                                double* __restrict__ z) {
  if (!*on) return;
  extern __shared__ double eig_lds[];
  double* d = eig_lds;
  double* e = d + n;
  double* u0 = e + n;
  double* u1 = u0 + n;
  double* u2 = u1 + n;
  double* x = u2 + n;
  const int i = blockIdx.x, lane = threadIdx.x;
  const double lmax = lam[n - 1];
  const double thr = rcond * lmax;
  const double tnorm = fmax(fabs(lam[0]), fabs(lmax));
  const double gtol = 1e-6 * tnorm;
  if (!(lam[i] > thr)) return;
  if (i > 0 && lam[i - 1] > thr && lam[i] - lam[i - 1] <= gtol) return;  // not the first member
  int last = i;
  while (last + 1 < n && lam[last + 1] - lam[last] <= gtol) ++last;
  for (int k = lane; k < n; k += 64) {
    d[k] = dg[k];
    e[k] = k < n - 1 ? eg[k] : 0.0;
  }
  const double pmin = EIG_EPS * fmax(tnorm, 1e-300);
  double prev = -1e308;
  for (int j = i; j <= last; ++j) {
    double s = lam[j];
    if (j > i && s <= prev + 4.0 * EIG_EPS * tnorm) s = prev + 4.0 * EIG_EPS * tnorm;
    prev = s;
    for (int k = lane; k < n; k += 64) x[k] = start_entry(j, k);
    for (int it = 0; it < EIG_ITERS; ++it) {
      // unit 2-norm right-hand side
      double q = 0.0;
      for (int k = lane; k < n; k += 64) q += x[k] * x[k];
      q = wave_sum(q);
      const double inv = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
      for (int k = lane; k < n; k += 64) x[k] *= inv;
      __syncthreads();
      if (lane == 0) {
        // forward elimination with row interchanges, right-hand side along
        double a = d[0] - s, b = n > 1 ? e[0] : 0.0, c2 = 0.0, r = x[0];
        for (int k = 0; k < n - 1; ++k) {
          const double sub = e[k];
          const double dn = d[k + 1] - s, sn = k + 1 < n - 1 ? e[k + 1] : 0.0;
          const double rn = x[k + 1];
          if (fabs(a) >= fabs(sub)) {
            if (fabs(a) < pmin) a = a < 0.0 ? -pmin : pmin;
            const double mlt = sub / a;
            u0[k] = a;
            u1[k] = b;
            u2[k] = c2;
            x[k] = r;
            a = dn - mlt * b;
            b = sn;
            c2 = 0.0;
            r = rn - mlt * r;
          } else {
            const double mlt = a / sub;
            u0[k] = sub;
            u1[k] = dn;
            u2[k] = sn;
            x[k] = rn;
            const double na = b - mlt * dn;
            b = -mlt * sn;
            c2 = 0.0;
            r = r - mlt * rn;
            a = na;
          }
        }
        if (fabs(a) < pmin) a = a < 0.0 ? -pmin : pmin;
        u0[n - 1] = a;
        u1[n - 1] = 0.0;
        u2[n - 1] = 0.0;
        x[n - 1] = r;
        // back substitution
        double x1 = 0.0, x2v = 0.0;
        for (int k = n - 1; k >= 0; --k) {
          const double v = (x[k] - u1[k] * x1 - u2[k] * x2v) / u0[k];
          x[k] = v;
          x2v = x1;
          x1 = v;
        }
      }
      __syncthreads();
      // orthogonalise against the cluster's earlier vectors
      for (int jj = i; jj < j; ++jj) {
        const double* zp = z + (size_t)jj * n;
        double dot = 0.0;
        for (int k = lane; k < n; k += 64) dot += zp[k] * x[k];
        dot = wave_sum(dot);
        for (int k = lane; k < n; k += 64) x[k] -= dot * zp[k];
      }
      __syncthreads();
    }
    double q = 0.0;
    for (int k = lane; k < n; k += 64) q += x[k] * x[k];
    q = wave_sum(q);
    const double inv = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    double* zj = z + (size_t)j * n;
    for (int k = lane; k < n; k += 64) zj[k] = x[k] * inv;
    __syncthreads();
  }
}

// 4a. c <- Q^H c (apply H_0^H first) or c <- Q c (H_{n-2} first), one
// workgroup: H_k^H c = c - conj(tau_k) v (v^H c), H_k c = c - tau_k v (v^H c)
template <typename S>
__global__ void __launch_bounds__(256) k_hh_apply(const S* __restrict__ T, int n,
                                                  const int* __restrict__ on,
                                                  const S* __restrict__ tau, int adjoint,
                                                  S* __restrict__ c) {
  if (!*on) return;
  __shared__ S red[4];
  for (int s = 0; s < n - 1; ++s) {
    const int k = adjoint ? s : n - 2 - s;
    const S* v = T + (size_t)k * n;
    S dot = S(0.0);
    for (int i = k + 1 + threadIdx.x; i < n; i += 256) dot += conjx(v[i]) * c[i];
    dot = block_sum(dot, red);
    const S f = (adjoint ? conjx(tau[k]) : tau[k]) * dot;
    for (int i = k + 1 + threadIdx.x; i < n; i += 256) c[i] -= f * v[i];
    __syncthreads();
  }
}

// 4b. u_j = (z_j . c) / lambda_j for the kept eigenvalues, one wave each
template <typename S>
__global__ void __launch_bounds__(256) k_eig_project(const double* __restrict__ z, int n,
                                                     const int* __restrict__ on,
                                                     const double* __restrict__ lam,
                                                     double rcond, const S* __restrict__ c,
                                                     S* __restrict__ u) {
  if (!*on) return;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const bool keep = lam[j] > rcond * lam[n - 1];
  S acc = S(0.0);
  if (keep) {
    const double* zj = z + (size_t)j * n;
    for (int k = lane; k < n; k += 64) acc += c[k] * zj[k];
    acc = wave_sum(acc);
  }
  if (lane == 0) u[j] = keep ? acc * (1.0 / lam[j]) : S(0.0);
}

// 4c. c_k = sum_j z_j[k] u_j over the kept eigenvalues
template <typename S>
__global__ void __launch_bounds__(256) k_eig_combine(const double* __restrict__ z, int n,
                                                     const int* __restrict__ on,
                                                     const double* __restrict__ lam,
                                                     double rcond, const S* __restrict__ u,
                                                     S* __restrict__ c) {
  if (!*on) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double thr = rcond * lam[n - 1];
  S acc = S(0.0);
  for (int j = 0; j < n; ++j)
    if (lam[j] > thr) acc += u[j] * z[(size_t)j * n + k];
  c[k] = acc;
}

// 4d. the step is valid: clear the failure flag the certificate may have
// set; diag[2] = number of dropped eigenvalues
__global__ void k_eig_finish(int n, const int* __restrict__ on, const double* __restrict__ lam,
                             double rcond, double* __restrict__ ws, double* __restrict__ diag) {
  if (!*on || threadIdx.x != 0) return;
  const double thr = rcond * lam[n - 1];
  int drop = 0;
  for (int j = 0; j < n; ++j) drop += !(lam[j] > thr);
  ws[6] = 0.0;
  diag[2] = (double)drop;
  diag[3] = 0.0;
}

size_t eigh_ws_bytes(int n, bool is_cplx) {
  const size_t es = is_cplx ? 16 : 8;
  return ((size_t)3 * n * 8 + (size_t)2 * n * es + 255) / 256 * 256 + (size_t)n * n * 8;
}

size_t eigh_lds_bytes(int n) { return (size_t)6 * n * sizeof(double); }

template <typename S>
static hipError_t eigh_impl(S* Tm, int n, double rcond, const int* on, double* ws, double* diag,
                            S* y, void* eig_ws, hipStream_t st) {
  double* d = (double*)eig_ws;
  double* e = d + n;
  double* lam = e + n;
  S* tau = (S*)(lam + n);
  S* p = tau + n;  // also u of the solve
  double* z = (double*)((char*)eig_ws + ((size_t)3 * n * 8 + (size_t)2 * n * sizeof(S) + 255) /
                                            256 * 256);
  for (int k = 0; k + 1 < n; ++k) {
    hipLaunchKernelGGL(k_hh_reflect<S>, dim3(1), dim3(256), 0, st, Tm, n, k, on, tau, d, e);
    const int m = n - k - 1;
    hipLaunchKernelGGL(k_hh_symv<S>, dim3((m + 3) / 4), dim3(256), 0, st, (const S*)Tm, n, k, on,
                       (const S*)tau, p);
    hipLaunchKernelGGL(k_hh_update<S>, dim3((m + 255) / 256, (m + 63) / 64), dim3(256), 0, st,
                       Tm, n, k, on, (const S*)tau, (const S*)p);
  }
  hipLaunchKernelGGL(k_tri_bisect, dim3((n + 255) / 256), dim3(256), 0, st, (const double*)d,
                     (const double*)e, n, on, lam);
  const size_t lds = eigh_lds_bytes(n);
  hipError_t err = hipFuncSetAttribute((const void*)k_tri_vec,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_tri_vec, dim3(n), dim3(64), lds, st, (const double*)d, (const double*)e, n,
                     on, (const double*)lam, rcond, z);
  hipLaunchKernelGGL(k_hh_apply<S>, dim3(1), dim3(256), 0, st, (const S*)Tm, n, on,
                     (const S*)tau, 1, y);
  hipLaunchKernelGGL(k_eig_project<S>, dim3((n + 3) / 4), dim3(256), 0, st, (const double*)z, n,
                     on, (const double*)lam, rcond, (const S*)y, p);
  hipLaunchKernelGGL(k_eig_combine<S>, dim3((n + 255) / 256), dim3(256), 0, st, (const double*)z,
                     n, on, (const double*)lam, rcond, (const S*)p, y);
  hipLaunchKernelGGL(k_hh_apply<S>, dim3(1), dim3(256), 0, st, (const S*)Tm, n, on,
                     (const S*)tau, 0, y);
  hipLaunchKernelGGL(k_eig_finish, dim3(1), dim3(64), 0, st, n, on, (const double*)lam, rcond, ws,
                     diag);
  return hipGetLastError();
}

hipError_t launch_eigh_solve(bool is_cplx, void* Tm, int n, double rcond, const int* on, double* ws,
                             double* diag, void* y, void* eig_ws, hipStream_t st) {
  if (is_cplx)
    return eigh_impl<cplx<double>>((cplx<double>*)Tm, n, rcond, on, ws, diag, (cplx<double>*)y,
                                   eig_ws, st);
  return eigh_impl<double>((double*)Tm, n, rcond, on, ws, diag, (double*)y, eig_ws, st);
}

}  // namespace pm
