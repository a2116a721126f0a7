// Boundary-MPS environments by the density-matrix MPS-MPO truncation (Sec.
// "On the boundary MPS method": the density-matrix algorithm the paper
// uses), with every large contraction on the matrix cores.
//
// One workgroup of 512 threads owns one (sample, direction) task at a time
// and loops over tasks (a persistent grid). For each absorbed row:
//   left to right : G_{y+1} = sum_k P_k^H G_y P_k, the Gram (left density
//                   environment) of the untruncated product MPS, where
//                   P_k[(a,l),(b,r)] = sum_in E[a,in,b] A[l,r,in,k];
//   right to left : Z_y = P_y W_{y+1}, rho_y = Z_y^H G_y Z_y, and the chi
//                   eigenvectors of rho_y with the largest eigenvalues v_j
//                   give the new tensor B_y[j, :] = conj(v_j) and the weight
//                   W_y = Z_y [v_0 .. v_{chi-1}] carried to the left.
// The eigenvalues of rho_y are the squared singular values of the canonical
// centre matrix, and the kept eigenvectors its dominant right singular
// vectors, so the truncated state equals the canonical QR -> SVD sweep's.
//
// The Gram is contracted one tensor at a time (G_y with E, A, conj(A),
// conj(E); no P_k is formed), and it, Z_y, G_y Z_y, rho_y and W_y run as
// MFMA products (v_mfma_f32_16x16x4_f32 for FP32 / complex64,
// v_mfma_f64_16x16x4_f64 for FP64 / complex128, bfloat16 operands in BF16
// mode; a complex product is four real ones). The Hermitian
// eigenproblem of rho_y is solved by Householder tridiagonalisation (rho in
// LDS as a packed lower triangle), multisection bisection on Sturm counts
// for the leading eigenvalues, inverse iteration with partial-pivoting LU
// for their eigenvectors (Gram-Schmidt inside clusters), and the stored
// reflectors applied back. Matrices between phases live in a per-workgroup
// slab of global memory (L2 / MALL resident).
#include "common.h"
#include "env_dev.h"
#include "kernels.h"
#include "mfma.h"

namespace pm {

// Reduction over the workgroup without a trailing barrier: `red` holds two
// slots of 16 values and consecutive reductions alternate between them, so
// the barrier of one reduction orders the reads of the one before.
template <typename T>
__device__ __forceinline__ T blk_sum2(T v, T* red, int& slot) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  T* r = red + 16 * slot;
  slot ^= 1;
  if (l == 0) r[w] = v;
  __syncthreads();
  T s = r[0];
  for (int i = 1; i < PEPS_NT / 64; ++i) s += r[i];
  return s;
}

// packed lower triangle: element (i, j), j <= i
__device__ __forceinline__ int pk(int i, int j) { return (i * (i + 1)) / 2 + j; }

__host__ __device__ inline int dm_np(int bmax, int D) { return (bmax * D + 31) / 32 * 32; }
__host__ __device__ inline int dm_rmax(int chi) { return chi + 1; }

// Slab of one workgroup (elements of T unless noted):
//   G   : Ly x NP x NP  left Gram environments G_0 .. G_{Ly-1}
//   then the right sweep's Pk, X, Z, T1, W, Hv (NP x NP each) and reals Yt
//   (RMAX x NP), lu (RMAX x 6 x NP): the iterates and U bands of the
//   eigenvector phase when they do not fit in LDS; the left sweep's two
//   intermediates W1, W2 (B^2 D^3 each) overlay the same region
__host__ __device__ inline size_t dm_wsz(int bmax, int D) {
  return (size_t)bmax * bmax * D * D * D;
}
__host__ __device__ inline size_t dm_slab_elems(int Ly, int bmax, int D, int chi, size_t tsize,
                                                size_t rsize) {
  const size_t np = dm_np(bmax, D);
  const size_t rm = dm_rmax(chi);
  const size_t r_bytes = rm * np * 7 * rsize;
  const size_t right = 6 * np * np + (r_bytes + tsize - 1) / tsize;
  const size_t left = 2 * dm_wsz(bmax, D);
  return (size_t)Ly * np * np + (right > left ? right : left) + 64;
}

// LDS: one big region (the staged E and A of a site, then the packed
// density matrix, then the eigenvector phase: the U bands of the inverse
// iterations under Xe, then their iterates Y, when that fits under the
// dynamic-LDS cap, else U and Y stay in the slab) and the small vectors.
#define DM_LDS_CAP (150 * 1024)
__host__ __device__ inline size_t dm_small_bytes(int np, size_t tsize, size_t rsize) {
  return (3 * (size_t)np + 32) * tsize + (3 * (size_t)np + 2 * 64 + 8) * rsize + 64;
}
__host__ __device__ inline size_t dm_big_elems(int bmax, int D, int chi, size_t tsize,
                                               size_t rsize, bool* eig_lds) {
  const size_t np = dm_np(bmax, D);
  const size_t rm = dm_rmax(chi);
  size_t big = (size_t)bmax * D * bmax + (size_t)D * D * D * D;
  const size_t rho = np * (np + 1) / 2;
  if (rho > big) big = rho;
  if (np * rm > big) big = np * rm;
  // U bands and multipliers (4 np rm, R) under Xe (np rm, T), then Y (np rm, R)
  const size_t xe_b = np * rm * tsize, u_b = 4 * np * rm * rsize;
  const size_t eig = ((xe_b > u_b ? xe_b : u_b) + np * rm * rsize + tsize - 1) / tsize;
  const size_t with = (eig > big ? eig : big);
  // FP32 modes run two workgroups per CU: each keeps below half the LDS
  const size_t cap = rsize == 4 ? DM_LDS_CAP / 2 : DM_LDS_CAP;
  const bool fits = ((with + 1) / 2 * 2) * tsize + dm_small_bytes((int)np, tsize, rsize) <= cap;
  if (eig_lds) *eig_lds = fits;
  big = fits ? with : big;
  return (big + 1) / 2 * 2;
}
__host__ __device__ inline size_t dm_lds_bytes(int bmax, int D, int chi, size_t tsize,
                                               size_t rsize) {
  const size_t big = dm_big_elems(bmax, D, chi, tsize, rsize, nullptr);
  return big * tsize + dm_small_bytes(dm_np(bmax, D), tsize, rsize);
}

template <typename T>
struct DmSh {
  typedef typename RealOf<T>::type R;
  T *big, *tau, *vb, *wb, *red;
  R *dd, *ee, *e2, *lam;
  bool eig_lds;  // U bands and iterates of the eigenvector phase in LDS
  __device__ DmSh(unsigned char* lds, int bmax, int D, int chi) {
    const size_t np = dm_np(bmax, D);
    const size_t bg = dm_big_elems(bmax, D, chi, sizeof(T), sizeof(R), &eig_lds);
    big = reinterpret_cast<T*>(lds);
    tau = big + bg;
    vb = tau + np;
    wb = vb + np;
    red = wb + np;
    dd = reinterpret_cast<R*>(red + 32);
    ee = dd + np;
    e2 = ee + np;
    lam = e2 + np;
  }
};

// a / b on the serial chains of the eigensolver (the reflectors of the
// tridiagonalisation, Sturm counts, inverse iteration): FP32 takes the hardware reciprocal (1 ulp) times a,
// FP64 the hardware reciprocal refined by one Newton step, r (2 - b r),
// which squares its relative error, times a (a few ulp). Both recurrences
// only need the quotient to a few ulp: a Sturm count changes only for
// shifts within rounding of an eigenvalue, and inverse iteration converges
// from any nearby solve.
template <typename R>
__device__ __forceinline__ R quot(R a, R b);
template <>
__device__ __forceinline__ float quot<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
template <>
__device__ __forceinline__ double quot<double>(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return a * r;
}

// 1 / x on the same chains (complex: Smith's scaling, no overflow of |x|^2)
template <typename R>
__device__ __forceinline__ R rcpq(R x) { return quot(R(1), x); }
template <typename R>
__device__ __forceinline__ cplx<R> rcpq(cplx<R> x) {
  if (fabs(x.re) >= fabs(x.im)) {
    const R r = quot(x.im, x.re), d = quot(R(1), x.re + x.im * r);
    return cplx<R>(d, -r * d);
  }
  const R r = quot(x.re, x.im), d = quot(R(1), x.re * r + x.im);
  return cplx<R>(r * d, -d);
}

// Multiply-adds as fused FMAs (four per complex product): u + a b,
// u + conj(a) b and u - a conj(b).
__device__ __forceinline__ float fmac(float u, float a, float b) { return fmaf(a, b, u); }
__device__ __forceinline__ double fmac(double u, double a, double b) { return fma(a, b, u); }
template <typename R>
__device__ __forceinline__ cplx<R> fmac(cplx<R> u, cplx<R> a, cplx<R> b) {
  u.re = fma(a.re, b.re, u.re);
  u.re = fma(-a.im, b.im, u.re);
  u.im = fma(a.re, b.im, u.im);
  u.im = fma(a.im, b.re, u.im);
  return u;
}
__device__ __forceinline__ float fmac_ca(float u, float a, float b) { return fmaf(a, b, u); }
__device__ __forceinline__ double fmac_ca(double u, double a, double b) { return fma(a, b, u); }
template <typename R>
__device__ __forceinline__ cplx<R> fmac_ca(cplx<R> u, cplx<R> a, cplx<R> b) {
  u.re = fma(a.re, b.re, u.re);
  u.re = fma(a.im, b.im, u.re);
  u.im = fma(a.re, b.im, u.im);
  u.im = fma(-a.im, b.re, u.im);
  return u;
}
__device__ __forceinline__ float fnmac_cb(float u, float a, float b) { return fmaf(-a, b, u); }
__device__ __forceinline__ double fnmac_cb(double u, double a, double b) { return fma(-a, b, u); }
template <typename R>
__device__ __forceinline__ cplx<R> fnmac_cb(cplx<R> u, cplx<R> a, cplx<R> b) {
  u.re = fma(-a.re, b.re, u.re);
  u.re = fma(-a.im, b.im, u.re);
  u.im = fma(-a.im, b.re, u.im);
  u.im = fma(a.re, b.im, u.im);
  return u;
}

// ---------------------------------------------------------------------------
// Householder reduction of the Hermitian nz x nz matrix held as a packed
// lower triangle (rho) to a real symmetric tridiagonal (dd, ee): reflector j
// H_j = I - tau_j v_j v_j^H acts on rows j+1..nz-1, v_j[j+1] = 1, and maps
// column j below the diagonal to (beta_j, 0, ...) with beta_j real, so
// rho = Q T Q^H with Q = H_0 H_1 ... H_{nz-2}. v_j goes to Hv row j.
// ---------------------------------------------------------------------------
template <typename T>
__device__ void tridiag(T* rho, int nz, T* Hv, int ldh, const DmSh<T>& sh, int& slot) {
  typedef typename RealOf<T>::type R;
  const int tid = threadIdx.x, NT = PEPS_NT;
  // symv: TPR lanes per row of the trailing block (full rows through the
  // symmetric storage, balanced); update: groups of G8 lanes per pair of
  // rows (one from the top, one from the bottom of the trailing triangle),
  // so every group has about the same number of elements. Both widths grow
  // as the trailing block shrinks (powers of two up to a wave), so every
  // step spreads its rows over the whole workgroup.
  R s2 = 0;
  for (int i = 2 + tid; i < nz; i += NT) s2 += abs2x(rho[pk(i, 0)]);
  s2 = blk_sum2(s2, reinterpret_cast<R*>(sh.red), slot);
  for (int j = 0; j + 1 < nz; ++j) {
    const int n1 = nz - j - 1, npair = (n1 + 1) / 2;
    int lt = 0, lg = 3;
    while (lt < 6 && (NT >> (lt + 1)) >= n1) ++lt;
    while (lg < 6 && (NT >> (lg + 1)) >= npair) ++lg;
    const int TPR = 1 << lt, rpp = NT >> lt;
    const int ri = tid >> lt, q = tid & (TPR - 1);
    const int G8 = 1 << lg, ng = NT >> lg, grp = tid >> lg, q8 = tid & (G8 - 1);
    const T alpha = rho[pk(j + 1, j)];
    // this thread's entry of column j below the diagonal, loaded while the
    // reflector's scalars form (n1 <= NT: one entry per thread)
    const int iv = j + 1 + tid;
    const T rv = iv < nz ? rho[pk(iv, j)] : T(0);
    R ar, aim;
    split(alpha, ar, aim);
    T tau = T(0), sc = T(0);
    R beta = ar;
    if (!(s2 == R(0) && aim == R(0))) {
      const R nrm = sqrt(ar * ar + aim * aim + s2);
      beta = ar >= R(0) ? -nrm : nrm;
      const R rb = rcpq(beta);
      tau = join<T>((beta - ar) * rb, -aim * rb);
      sc = rcpq(alpha - T(beta));
    }
    if (tid == 0) {
      sh.dd[j] = realx(rho[pk(j, j)]);
      sh.ee[j] = beta;
      sh.tau[j] = tau;
    }
    // v_i = 1 (i = j+1), rho[i][j] sc below, once into LDS and Hv row j
    if (iv < nz) {
      const T v = iv == j + 1 ? T(1) : rv * sc;
      sh.vb[iv] = v;
      Hv[(size_t)j * ldh + iv] = v;
    }
    for (int i = iv + NT; i < nz; i += NT) {
      const T v = rho[pk(i, j)] * sc;
      sh.vb[i] = v;
      Hv[(size_t)j * ldh + i] = v;
    }
    if (tau == T(0)) {
      R t = 0;
      for (int i = j + 3 + tid; i < nz; i += NT) t += abs2x(rho[pk(i, j + 1)]);
      s2 = blk_sum2(t, reinterpret_cast<R*>(sh.red), slot);
      continue;
    }
    __syncthreads();
    // u = B v for the trailing block B (rows / columns j+1..), then
    // w = tau u - (|tau|^2 / 2) (v^H u) v
    T vhu = T(0);
    T ui[2] = {T(0), T(0)};
    for (int p = 0; p < 2; ++p) {
      const int i = j + 1 + ri + p * rpp;
      T u = T(0);
      if (i < nz) {
        // row part (k <= i) then the column part through the symmetry, the
        // packed index of (kk, i) stepped by kk TPR + TPR (TPR + 1) / 2
        int kk = j + 1 + q;
        const T* rr = rho + pk(i, 0);
        for (; kk <= i; kk += TPR) u = fmac(u, rr[kk], sh.vb[kk]);
        int a = pk(kk, i);
        const int step0 = TPR * (TPR + 1) / 2;
        for (; kk < nz; kk += TPR) {
          u = fmac_ca(u, rho[a], sh.vb[kk]);
          a += TPR * kk + step0;
        }
      }
      u = group_sum(u, TPR);
      ui[p] = u;
      if (i < nz && q == 0) vhu += conjx(sh.vb[i]) * u;
    }
    const R vhu_r = blk_sum2(realx(vhu), reinterpret_cast<R*>(sh.red), slot);
    const R t2 = abs2x(tau) * R(0.5) * vhu_r;
    for (int p = 0; p < 2; ++p) {
      const int i = j + 1 + ri + p * rpp;
      if (i < nz && q == 0) sh.wb[i] = tau * ui[p] - sh.vb[i] * t2;
    }
    __syncthreads();
    // B -= v w^H + w v^H on the lower triangle, rows paired top / bottom;
    // column j+1's new squares below row j+2 feed the next reflector
    R t = 0;
    for (int g = grp; g < npair; g += ng) {
      for (int h = 0; h < 2; ++h) {
        const int i = h == 0 ? j + 1 + g : nz - 1 - g;
        if (h == 1 && i <= j + 1 + g) break;
        const T vi = sh.vb[i], wi = sh.wb[i];
        T* rr = rho + pk(i, 0);
        for (int kk = j + 1 + q8; kk <= i; kk += G8) {
          const T nv = fnmac_cb(fnmac_cb(rr[kk], vi, sh.wb[kk]), wi, sh.vb[kk]);
          rr[kk] = nv;
          if (kk == j + 1 && i >= j + 3) t += abs2x(nv);
        }
      }
    }
    s2 = blk_sum2(t, reinterpret_cast<R*>(sh.red), slot);
  }
  if (tid == 0) {
    sh.dd[nz - 1] = realx(rho[pk(nz - 1, nz - 1)]);
    sh.ee[nz - 1] = 0;
  }
  __syncthreads();
}

// The same reduction with the matrix in registers (nz <= 128, 512 threads;
// every mode but BF16, whose kernel spills in it). Thread (r, c) = (tid / 16, tid % 16) holds the full
// Hermitian matrix's elements (r + 32 a, c + 16 b), a < 4, b < 8: u = B v is
// a per-thread partial over its columns summed over the 16 lanes that share
// its rows, and the rank-2 update touches registers only. LDS carries the
// vectors: the column that makes the next reflector, written by its owners
// during the update with its partial squared norms (two buffers, the
// current column still being read), and u. Two barriers per reflector
// instead of four, and O(nz) LDS traffic per reflector instead of O(nz^2).
// rhoG: the full matrix (lower triangle read, row stride ldg).
template <typename T>
__device__ void tridiag_reg(const T* rhoG, int ldg, int nz, T* Hv, int ldh, const DmSh<T>& sh) {
  typedef typename RealOf<T>::type R;
  const int tid = threadIdx.x;
  const int c = tid & 15, r = tid >> 4, w = tid >> 6;
  // u and v of the current reflector (zero outside rows j+1 .. nz-1)
  T* ub = sh.big;
  T* vv = ub + 128;
  R* nrm = reinterpret_cast<R*>(vv + 128);
  R* vhp = nrm + 8;
  if (tid < 128) {
    ub[tid] = T(0);
    vv[tid] = T(0);
  }
  T B[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = r + 32 * a, k = c + 16 * b;
      T x = T(0);
      if (i < nz && k < nz) x = k <= i ? rhoG[(size_t)i * ldg + k] : conjx(rhoG[(size_t)k * ldg + i]);
      B[a][b] = x;
    }
  // column jc from rows jc.. into cb, its squares below row jc + 1 summed per wave
  auto put_col = [&](int jc, T* cb) {
    R s = 0;
    if (c == (jc & 15)) {
      const int bj = jc >> 4;
#pragma unroll
      for (int b = 0; b < 8; ++b)
        if (b == bj) {
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int i = r + 32 * a;
            if (i >= jc && i < nz) cb[i] = B[a][b];
            if (i >= jc + 2 && i < nz) s += abs2x(B[a][b]);
          }
        }
    }
    // nonzero on the owners only: lanes jc % 16 + 16 m of each wave
    s += shfl_xor_x(s, 16);
    s += shfl_xor_x(s, 32);
    if ((tid & 63) == (jc & 15)) nrm[w] = s;
  };
  put_col(0, sh.vb);
  __syncthreads();
  for (int j = 0; j + 1 < nz; ++j) {
    const T* cb = (j & 1) ? sh.wb : sh.vb;
    T* cbn = (j & 1) ? sh.vb : sh.wb;
    const R s2 = ((nrm[0] + nrm[1]) + (nrm[2] + nrm[3])) + ((nrm[4] + nrm[5]) + (nrm[6] + nrm[7]));
    const T alpha = cb[j + 1];
    R ar, aim;
    split(alpha, ar, aim);
    T tau = T(0), sc = T(0);
    R beta = ar;
    if (!(s2 == R(0) && aim == R(0))) {
      const R nv = sqrt(ar * ar + aim * aim + s2);
      beta = ar >= R(0) ? -nv : nv;
      const R rb = rcpq(beta);
      tau = join<T>((beta - ar) * rb, -aim * rb);
      sc = rcpq(alpha - T(beta));
    }
    if (tid == 0) {
      sh.dd[j] = realx(cb[j]);
      sh.ee[j] = beta;
      sh.tau[j] = tau;
    }
    // v_i = 1 (i = j+1), column j's entry times sc below, 0 elsewhere
    auto vval = [&](int i) -> T {
      return i == j + 1 ? T(1) : ((i > j + 1 && i < nz) ? cb[i] * sc : T(0));
    };
    // row slots a < a0 and column slots b < b0 hold finished rows / columns
    // (index <= j) only: the same for every thread, skipped
    const int a0 = (j + 1) >> 5, b0 = (j + 1) >> 4;
    // u = B v for the rows of the trailing block (zero for the others),
    // from the unscaled column: u = sc (B x) + B[:, j+1] with x the column
    // below row j+1 (v = sc x there, v_{j+1} = 1)
    T acc[4], e1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      acc[a] = T(0);
      e1[a] = T(0);
    }
    const int b1 = (j + 1) >> 4;
    const bool own1 = c == ((j + 1) & 15);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b < b0) continue;
      const int k = c + 16 * b;
      const T xk = (k > j + 1 && k < nz) ? cb[k] : T(0);
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (a >= a0) acc[a] = fmac(acc[a], B[a][b], xk);
      if (b == b1) {
#pragma unroll
        for (int a = 0; a < 4; ++a) e1[a] = own1 ? B[a][b] : T(0);
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a] = acc[a] * sc + e1[a];
    R vh = 0;
    // u and v of row j (finished now) read as zero from here on
    if (tid == 0) {
      ub[j] = T(0);
      vv[j] = T(0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a < a0) continue;
      const int i = r + 32 * a;
      const T u = group_sum(acc[a], 16);
      if (c == 0 && i < nz) {
        // each row's sum is held by its 16 lanes: one of them stores and counts it
        const T vi = vval(i);
        const T ui = i > j ? u : T(0);
        ub[i] = ui;
        vv[i] = vi;
        if (i > j) Hv[(size_t)j * ldh + i] = vi;
        vh += realx(conjx(vi) * ui);
      }
    }
    // nonzero on lanes 0, 16, 32, 48 of each wave only
    vh += shfl_xor_x(vh, 16);
    vh += shfl_xor_x(vh, 32);
    if ((tid & 63) == 0) vhp[w] = vh;
    __syncthreads();
    const R vhu_r = ((vhp[0] + vhp[1]) + (vhp[2] + vhp[3])) + ((vhp[4] + vhp[5]) + (vhp[6] + vhp[7]));
    // w = tau u - (|tau|^2 / 2) (v^H u) v; B -= v w^H + w v^H
    const R t2 = abs2x(tau) * R(0.5) * vhu_r;
    T vr[4], wr[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = r + 32 * a;
      vr[a] = T(0);
      wr[a] = T(0);
      if (a < a0) continue;
      vr[a] = vv[i];
      wr[a] = tau * ub[i] - vr[a] * t2;
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b < b0) continue;
      const int k = c + 16 * b;
      const T vk = vv[k];
      const T wk = tau * ub[k] - vk * t2;
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (a >= a0) B[a][b] = fnmac_cb(fnmac_cb(B[a][b], vr[a], wk), wr[a], vk);
    }
    put_col(j + 1, cbn);
    __syncthreads();
  }
  if (tid == 0) {
    const T* cb = ((nz - 1) & 1) ? sh.wb : sh.vb;
    sh.dd[nz - 1] = realx(cb[nz - 1]);
    sh.ee[nz - 1] = 0;
  }
  __syncthreads();
}

// Eigenvalues below x of the symmetric tridiagonal (d, e^2): Sturm count.
template <typename R>
__device__ __forceinline__ int sturm(const R* d, const R* e2, int n, R x, R pivmin) {
  int c = 0;
  R qv = d[0] - x;
  if (fabs(qv) < pivmin) qv = -pivmin;
  c += qv < R(0);
  for (int i = 1; i < n; ++i) {
    qv = (d[i] - x) - quot(e2[i - 1], qv);
    if (fabs(qv) < pivmin) qv = -pivmin;
    c += qv < R(0);
  }
  return c;
}

// The rr largest eigenvalues of (dd, ee), descending, into lam[0..rr):
// LPE lanes per eigenvalue evaluate Sturm counts at LPE-1 interior points
// of its bracket and keep the sub-interval that holds it.
template <typename R>
__device__ void top_eigenvalues(const R* dd, const R* ee, R* e2, R* lam, int nz, int rr,
                                R* red, int& slot, R& tnorm_out) {
  const int tid = threadIdx.x, NT = PEPS_NT;
  R lo = R(1e300 > 1e30 ? 0 : 0), hi = 0;
  R gl = 0, gu = 0;
  for (int i = tid; i < nz; i += NT) {
    const R a = i > 0 ? fabs(ee[i - 1]) : R(0);
    const R b = i + 1 < nz ? fabs(ee[i]) : R(0);
    e2[i] = ee[i] * ee[i];
    const R l0 = dd[i] - a - b, u0 = dd[i] + a + b;
    if (i == tid) {
      gl = l0;
      gu = u0;
    } else {
      gl = l0 < gl ? l0 : gl;
      gu = u0 > gu ? u0 : gu;
    }
  }
  // block min / max through the sum slots: -max(-x)
  R mn = tid < nz ? -gl : -R(1e30);
  R mx = tid < nz ? gu : -R(1e30);
  mn = wave_max(mn);
  mx = wave_max(mx);
  {
    const int w = tid >> 6, l = tid & 63;
    R* r = red + 16 * slot;
    slot ^= 1;
    if (l == 0) {
      r[w] = mn;
      r[8 + w] = mx;
    }
    __syncthreads();
    mn = r[0];
    mx = r[8];
    for (int i = 1; i < NT / 64; ++i) {
      mn = r[i] > mn ? r[i] : mn;
      mx = r[8 + i] > mx ? r[8 + i] : mx;
    }
  }
  gl = -mn;
  gu = mx;
  const R tnorm = fabs(gl) > fabs(gu) ? fabs(gl) : fabs(gu);
  tnorm_out = tnorm;
  const R epsr = Eps<R>::v;
  const R pad = R(2) * epsr * tnorm * nz + (tnorm > R(0) ? R(0) : R(1));
  gl -= pad;
  gu += pad;
  // pivmin: the smallest pivot magnitude kept in a Sturm count
  R emax = 0;
  for (int i = 0; i + 1 < nz; ++i) emax = e2[i] > emax ? e2[i] : emax;
  const R pivmin = (std::is_same<R, double>::value ? R(2.2250738585072014e-308)
                                                     : R(1.17549435e-38f)) *
                   (emax > R(1) ? emax : R(1));
  int LPE = 16;
  while (LPE > 2 && rr * LPE > NT) LPE >>= 1;
  const int qe = tid / LPE, p = tid - qe * LPE;
  const int iters = std::is_same<R, double>::value ? (LPE >= 16 ? 15 : 20) : (LPE >= 16 ? 8 : 11);
  lo = gl;
  hi = gu;
  const bool act = qe < rr;
  const int m = nz - 1 - qe;  // ascending index of the wanted eigenvalue
  for (int it = 0; it < iters; ++it) {
    int pbest = 0;
    if (act && p > 0) {
      const R x = lo + (hi - lo) * (R)p / (R)LPE;
      if (sturm(dd, e2, nz, x, pivmin) <= m) pbest = p;
    }
    // largest interior point that still has at most m eigenvalues below
    int g = pbest;
    for (int o = 1; o < LPE; o <<= 1) {
      const int h = __shfl_xor(g, o, 64);
      g = h > g ? h : g;
    }
    const R w = hi - lo;
    const R nlo = lo + w * (R)g / (R)LPE;
    const R nhi = (g + 1 == LPE) ? hi : lo + w * (R)(g + 1) / (R)LPE;
    lo = nlo;
    hi = nhi;
  }
  if (act && p == 0) lam[qe] = R(0.5) * (lo + hi);
  __syncthreads();
}

// The row-swap flag of an LU step kept in the lowest mantissa bit of its
// multiplier (which moves the multiplier by at most one ulp).
__device__ __forceinline__ float with_flag(float v, bool f) {
  return __uint_as_float((__float_as_uint(v) & ~1u) | (f ? 1u : 0u));
}
__device__ __forceinline__ double with_flag(double v, bool f) {
  return __longlong_as_double((__double_as_longlong(v) & ~1ll) | (f ? 1ll : 0ll));
}
__device__ __forceinline__ bool flag_of(float v) { return __float_as_uint(v) & 1u; }
__device__ __forceinline__ bool flag_of(double v) { return __double_as_longlong(v) & 1ll; }

// Eigenvector of the tridiagonal for eigenvalue x by inverse iteration:
// three solves of (T - x I) y = b from b = ones. The first forms the
// partial-pivoting LU of T - x I row by row with b eliminated alongside,
// keeping the three bands of U and each step's multiplier (its row swap in
// the multiplier's last bit); the next two apply the stored steps to their
// right-hand sides. y is scaled by its largest entry after each solve.
// Serial in the calling lane; the bands u (4 n) and y (n) are interleaved
// across lanes with stride ld (element i of this lane at [i * ld]), so the
// lanes' accesses of one step are consecutive.
template <typename R>
__device__ void inv_iter_lane(const R* dd, const R* ee, int n, R x, R tnorm, R* u, R* y,
                              int ld) {
  R* u0 = u;
  R* u1 = u + (size_t)n * ld;
  R* u2 = u + (size_t)2 * n * ld;
  R* um = u + (size_t)3 * n * ld;
  const R tiny = Eps<R>::v * (tnorm > R(0) ? tnorm : R(1));
  for (int i = 0; i < n; ++i) y[(size_t)i * ld] = R(1);
  for (int it = 0; it < 3; ++it) {
    if (it == 0) {
      // rows i, i+1 with pivoting on the sub-diagonal; (c0, c1) the current
      // row's entries at columns i, i+1 and r0 its right-hand side
      R c0 = dd[0] - x, c1 = n > 1 ? ee[0] : R(0), r0 = y[0];
      for (int i = 0; i + 1 < n; ++i) {
        const R s0 = ee[i], s1 = dd[i + 1] - x, s2 = i + 2 < n ? ee[i + 1] : R(0);
        const R rn = y[(size_t)(i + 1) * ld];
        const size_t o = (size_t)i * ld;
        if (fabs(s0) > fabs(c0)) {
          const R mm = quot(c0, s0);
          u0[o] = s0;
          u1[o] = s1;
          u2[o] = s2;
          um[o] = with_flag(mm, true);
          y[o] = rn;
          c0 = c1 - mm * s1;
          c1 = -(mm * s2);
          r0 = r0 - mm * rn;
        } else {
          if (c0 == R(0)) c0 = tiny;
          const R mm = quot(s0, c0);
          u0[o] = c0;
          u1[o] = c1;
          u2[o] = R(0);
          um[o] = with_flag(mm, false);
          y[o] = r0;
          c0 = s1 - mm * c1;
          c1 = s2;
          r0 = rn - mm * r0;
        }
      }
      if (c0 == R(0)) c0 = tiny;
      const size_t ol = (size_t)(n - 1) * ld;
      u0[ol] = c0;
      u1[ol] = R(0);
      u2[ol] = R(0);
      y[ol] = r0;
    } else {
      R r0 = y[0];
      for (int i = 0; i + 1 < n; ++i) {
        const size_t o = (size_t)i * ld;
        const R rn = y[o + ld], m = um[o];
        if (flag_of(m)) {
          y[o] = rn;
          r0 = r0 - m * rn;
        } else {
          y[o] = r0;
          r0 = rn - m * r0;
        }
      }
      y[(size_t)(n - 1) * ld] = r0;
    }
    R nrm = 0, y1 = 0, y2 = 0;
    for (int i = n - 1; i >= 0; --i) {
      const size_t o = (size_t)i * ld;
      R s = y[o];
      if (i + 1 < n) s -= u1[o] * y1;
      if (i + 2 < n) s -= u2[o] * y2;
      s = quot(s, u0[o]);
      y[o] = s;
      y2 = y1;
      y1 = s;
      nrm = fabs(s) > nrm ? fabs(s) : nrm;
    }
    const R inv = nrm > R(0) ? R(1) / nrm : R(1);
    for (int i = 0; i < n; ++i) y[(size_t)i * ld] *= inv;
  }
}

// ---------------------------------------------------------------------------
// The r leading eigenvectors of the Hermitian nz x nz matrix rho (full, in
// the slab, row stride NP): on exit Xe (LDS, nz x r, row stride r) holds
// them as columns, lam[0..rr) the rr = min(r + 1, nz) largest eigenvalues.
// REG (every mode but BF16; up to 128 x 128, 512 threads): the reduction
// to tridiagonal form holds rho in registers; otherwise rho is copied to LDS
// as a packed lower triangle (sh.big) first. Xe overlays sh.big after it.
// ---------------------------------------------------------------------------
template <typename T, bool REG>
__device__ void dm_eig(const T* rhoG, int np, int nz, int r, int rr, T* Hv, typename RealOf<T>::type* Yt,
                       typename RealOf<T>::type* lu, const DmSh<T>& sh, int& slot,
                       typename RealOf<T>::type& tnorm) {
  typedef typename RealOf<T>::type R;
  const int tid = threadIdx.x, NT = PEPS_NT;
  if (REG && NT == 512 && nz <= 128) {
    tridiag_reg(rhoG, np, nz, Hv, np, sh);
  } else {
    T* rho = sh.big;
    const int tot = nz * (nz + 1) / 2;
    for (int idx = tid; idx < tot; idx += NT) {
      // invert idx = i (i + 1) / 2 + j
      int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while (pk(i + 1, 0) <= idx) ++i;
      while (pk(i, 0) > idx) --i;
      const int j = idx - pk(i, 0);
      rho[idx] = rhoG[(size_t)i * np + j];
    }
    __syncthreads();
    tridiag(rho, nz, Hv, np, sh, slot);
  }
  top_eigenvalues(sh.dd, sh.ee, sh.e2, sh.lam, nz, rr, reinterpret_cast<R*>(sh.red), slot, tnorm);
  // eigenvectors of the tridiagonal, one lane each, vector c's element e at
  // Y[e * r + c]; in LDS when they fit (the packed matrix is dead now): the
  // U bands over the area Xe takes later, Y after both
  R* U = lu;
  R* Y = Yt;
  if (sh.eig_lds) {
    const size_t xe_b = (size_t)nz * r * sizeof(T), u_b = (size_t)4 * nz * r * sizeof(R);
    U = reinterpret_cast<R*>(sh.big);
    Y = reinterpret_cast<R*>(reinterpret_cast<char*>(sh.big) + (xe_b > u_b ? xe_b : u_b));
  }
  if (tid < r) inv_iter_lane(sh.dd, sh.ee, nz, sh.lam[tid], tnorm, U + tid, Y + tid, r);
  __syncthreads();
  // Gram-Schmidt inside clusters of close eigenvalues (wave 0, in order)
  if (tid < 64) {
    const R ctol = R(1e-3) * tnorm;
    for (int j = 0; j < r; ++j) {
      R* yj = Y + j;
      for (int i = 0; i < j; ++i) {
        if (!(fabs(sh.lam[i] - sh.lam[j]) <= ctol)) continue;
        const R* yi = Y + i;
        R d = 0;
        for (int e = tid; e < nz; e += 64) d += yi[(size_t)e * r] * yj[(size_t)e * r];
        d = wave_sum(d);
        for (int e = tid; e < nz; e += 64) yj[(size_t)e * r] -= d * yi[(size_t)e * r];
      }
      R s = 0;
      for (int e = tid; e < nz; e += 64) s += yj[(size_t)e * r] * yj[(size_t)e * r];
      s = wave_sum(s);
      const R inv = s > R(0) ? R(1) / sqrt(s) : R(0);
      for (int e = tid; e < nz; e += 64) yj[(size_t)e * r] *= inv;
    }
  }
  __syncthreads();
  // Xe = Q Y: reflectors applied last to first; column c owned by P lanes
  // of one wave (no barrier: columns are independent)
  T* Xe = sh.big;
  for (int idx = tid; idx < nz * r; idx += NT) Xe[idx] = T(Y[idx]);
  __syncthreads();
  int P = 64;
  while (P > 1 && r * P > NT) P >>= 1;
  const int col = tid / P, part = tid - col * P;
  constexpr int VPL = 8;  // column entries a lane holds when they fit
  if (col < r && (nz + P - 1) / P <= VPL) {
    // lane `part` keeps rows part + u P of its column in registers for the
    // whole transformation; reflector j touches the rows below j (the
    // others read as zero), and the next reflector's entries are loaded
    // while the current one is applied, so the slab's latency is off the
    // dependent chain
    T xe[VPL], vc[VPL], vn[VPL];
#pragma unroll
    for (int u = 0; u < VPL; ++u) {
      const int e = part + u * P;
      xe[u] = e < nz ? Xe[e * r + col] : T(0);
    }
    auto load = [&](int j, T* dst) {
      const T* v = Hv + (size_t)j * np;
#pragma unroll
      for (int u = 0; u < VPL; ++u) {
        const int e = part + u * P;
        dst[u] = (e > j && e < nz) ? v[e] : T(0);
      }
    };
    load(nz - 2, vc);
    for (int j = nz - 2; j >= 0; --j) {
      if (j > 0) load(j - 1, vn);
      const T tj = sh.tau[j];
      if (tj != T(0)) {
        T sdot = T(0);
#pragma unroll
        for (int u = 0; u < VPL; ++u) sdot += conjx(vc[u]) * xe[u];
        sdot = group_sum(sdot, P) * tj;
#pragma unroll
        for (int u = 0; u < VPL; ++u) xe[u] -= vc[u] * sdot;
      }
#pragma unroll
      for (int u = 0; u < VPL; ++u) vc[u] = vn[u];
    }
#pragma unroll
    for (int u = 0; u < VPL; ++u) {
      const int e = part + u * P;
      if (e < nz) Xe[e * r + col] = xe[u];
    }
  } else if (col < r) {
    for (int j = nz - 2; j >= 0; --j) {
      const T tj = sh.tau[j];
      if (tj == T(0)) continue;
      const T* v = Hv + (size_t)j * np;
      T sdot = T(0);
      for (int e = j + 1 + part; e < nz; e += P) sdot += conjx(v[e]) * Xe[e * r + col];
      sdot = group_sum(sdot, P) * tj;
      for (int e = j + 1 + part; e < nz; e += P) Xe[e * r + col] -= v[e] * sdot;
    }
  }
  __syncthreads();
}

// Stored bonds of environment slot sp (left bond of every site, then 1):
// the kept bonds of an environment read over its chi-wide layout.
__device__ __forceinline__ void dm_first_bonds(const Lattice& L, const int* tab, int sp, int* kb) {
  const int* ed = tab + L.off_env;
  for (int y = threadIdx.x; y <= L.Ly; y += PEPS_NT) kb[y] = y < L.Ly ? ed[(sp * L.Ly + y) * 3] : 1;
  __syncthreads();
}

// The leading [bl][din][br] block of a boundary tensor stored as
// [.][din][brs] (kept bonds of a truncated-weight cut inside the chi-wide
// layout), packed.
template <typename T>
__device__ __forceinline__ void load_block(T* dst, const T* src, int bl, int din, int br,
                                           int brs) {
  const int cnt = bl * din * br;
  for (int i = threadIdx.x; i < cnt; i += PEPS_NT) {
    const int ai = i / br, b = i - ai * br;
    dst[i] = src[(size_t)ai * brs + b];
  }
}

// One row absorbed by the density-matrix truncation (see the file header).
// kprev[y] / kprev[y+1]: the kept left / right bond of site y of the
// previous environment (kprev[Ly] = 1); the bonds kept here go to knew.
// Every contraction runs over the kept bonds only; the tensors are stored
// in the chi-wide layout with zeros beyond them.
template <int M>
__device__ __forceinline__ void dm_absorb_row(const Lattice& L, const int* tab, const typename ModeT<M>::T* theta,
                              const uint8_t* s, bool bottom, int t, typename ModeT<M>::T* envs,
                              double* lg, typename ModeT<M>::T* slab, const DmSh<typename ModeT<M>::T>& sh,
                              int* flp, int& slot, const int* kprev, int* knew) {
  typedef typename ModeT<M>::T T;
  typedef typename RealOf<T>::type R;
  const int tid = threadIdx.x, NT = PEPS_NT;
  const int np = dm_np(L.bmax, L.D);
  const size_t np2 = (size_t)np * np;
  T* Gs = slab;
  T* Pk = Gs + (size_t)L.Ly * np2;
  T* X = Pk + np2;
  T* Z = X + np2;
  T* T1 = Z + np2;
  T* W = T1 + np2;
  T* Hv = W + np2;
  R* Yt = reinterpret_cast<R*>(Hv + np2);
  R* lu = Yt + (size_t)dm_rmax(L.chi) * np;
  T* W1 = Pk;
  T* W2 = W1 + dm_wsz(L.bmax, L.D);
  constexpr bool CX = IsCplx<T>::value, BFM = M == MODE_BF16;
  T* Ebuf = sh.big;
  T* Abuf = Ebuf + L.bmax * L.D * L.bmax;
  int& fl = *flp;
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  const int* edims = tab + L.off_env;
  const int x = bottom ? L.Lx - 1 - t : t;
  const int sp = bottom ? slot_bottom(L, x + 1) : slot_top(L, x - 1);
  const int sn = bottom ? slot_bottom(L, x) : slot_top(L, x);
  const T* Eprev = envs + (size_t)sp * slot_elems;
  T* Enew = envs + (size_t)sn * slot_elems;

  // ---- left to right: Gram environments ----
  if (tid == 0) Gs[0] = T(1);  // G_0 = [1]
  __syncthreads();
  for (int y = 0; y < L.Ly - 1; ++y) {
    const SiteView v = site_view(tab, L, x * L.Ly + y, bottom);
    const int bl = kprev[y], br = kprev[y + 1];
    const int brs = edims[(sp * L.Ly + y) * 3 + 2];
    const int Pl = bl * v.Dl, Pr = br * v.Dr;
    load_block(Ebuf, Eprev + (size_t)y * L.site_box, bl, v.Din, br, brs);
    load_lds(Abuf, site_tensor(theta, tab, L, s, x * L.Ly + y), v.Dl * v.Dr * v.Din * v.Dout);
    __syncthreads();
    const T* Gy = Gs + (size_t)y * np2;
    T* Gn = Gs + (size_t)(y + 1) * np2;
    // G_{y+1} = sum_k P_k^H G_y P_k contracted one tensor at a time (no P_k
    // is formed): E, A, conj(A), conj(E), each step one matrix-core product
    // W1[(a,l,l'),(in,b)] = sum_a' G[(a,l),(a',l')] E[a',in,b]
    const int n1 = v.Din * br;
    mgemm_map<T, false, false, BFM, CX>(Pl * v.Dl, n1, bl, Gy, IMap(v.Dl, np, 1), IMap(v.Dl), Ebuf,
                                    IMap(n1), IMap(1), W1, IMap(n1), IMap(1), false, false);
    __syncthreads();
    // W2[(a,l,b),(r,k)] = sum_{(l',in)} W1[(a,l,l'),(in,b)] A[l',r,in,k]
    const int n2 = v.Dr * v.Dout;
    mgemm_map<T, false, false, BFM, CX>(Pl * br, n2, v.Dl * v.Din, W1, IMap(br, v.Dl * n1, 1),
                                    IMap(v.Din, n1, br), Abuf, IMap(v.Din, v.s_l, v.s_in),
                                    IMap(v.Dout, v.s_r, v.s_out), W2, IMap(n2), IMap(1), false,
                                    false);
    __syncthreads();
    // W3[(a,b,r'),(in',r)] = sum_{(l,k)} W2[(a,l,b),(r',k)] conj(A[l,r,in',k])
    // (into W1)
    const int n3 = v.Din * v.Dr;
    mgemm_map<T, false, CX, BFM, CX>(bl * br * v.Dr, n3, v.Dl * v.Dout, W2,
                                 IMap(br * v.Dr, v.Dl * br * n2, v.Dout), IMap(v.Dout, br * n2, 1),
                                 Abuf, IMap(v.Dout, v.s_l, v.s_out), IMap(v.Dr, v.s_in, v.s_r), W1,
                                 IMap(n3), IMap(1), false, false);
    __syncthreads();
    // G_{y+1}[(b,r),(b',r')] = sum_{(a,in')} W3[(a,b',r'),(in',r)] conj(E[a,in',b]),
    // rows (b',r',r) of the product scattered to their places in G_{y+1}
    mgemm_map<T, false, CX, BFM, CX>(br * v.Dr * v.Dr, br, bl * v.Din, W1, IMap(v.Dr, n3, 1),
                                 IMap(v.Din, br * v.Dr * n3, v.Dr), Ebuf, IMap(br), IMap(1), Gn,
                                 IMap(v.Dr, 1, np), IMap(v.Dr * np), false, false);
    __syncthreads();
    // unit scale: the Gram only fixes directions
    R mx = 0;
    for (int i = tid; i < Pr; i += NT) {
      const R a = absx(Gn[(size_t)i * np + i]);
      mx = a > mx ? a : mx;
    }
    mx = block_max(mx, reinterpret_cast<R*>(sh.red + 16 * slot));
    const int e = pow2_exponent((double)mx);
    if (e != 0) {
      const R f = (R)ldexp(1.0, -e);
      for (int i = tid; i < Pr * Pr; i += NT) Gn[(size_t)(i / Pr) * np + (i % Pr)] *= f;
    }
    __syncthreads();
  }

  // ---- right to left: density matrices and their leading eigenvectors ----
  int nbr = 1;
  double logrow = 0.0;
  if (tid == 0) W[0] = T(1);
  __syncthreads();
  for (int y = L.Ly - 1; y >= 0; --y) {
    const int nsite = x * L.Ly + y;
    const SiteView v = site_view(tab, L, nsite, bottom);
    const int bl = kprev[y], br = kprev[y + 1];
    const int brs = edims[(sp * L.Ly + y) * 3 + 2];
    const int Pl = bl * v.Dl;
    const int zc = v.Dout * nbr;
    // the new tensor's stored (chi-wide) left and right bonds
    const int rs = edims[(sn * L.Ly + y) * 3 + 0];
    const int nbrs = edims[(sn * L.Ly + y) * 3 + 2];
    load_block(Ebuf, Eprev + (size_t)y * L.site_box, bl, v.Din, br, brs);
    load_lds(Abuf, site_tensor(theta, tab, L, s, nsite), v.Dl * v.Dr * v.Din * v.Dout);
    __syncthreads();
    // T1[(a,in),(r,c)] = sum_b E[(a,in), b] W[(b,r), c]: one product with
    // columns (r,c)
    mgemm_map<T, false, false, M == MODE_BF16, IsCplx<T>::value>(
        bl * v.Din, v.Dr * nbr, br, Ebuf, IMap(br), IMap(1), W, IMap(v.Dr * np),
        IMap(nbr, np, 1), T1, IMap(v.Dr * nbr), IMap(1), false, false);
    __syncthreads();
    // Z[(a,l),(k,c)] = sum_{in,r} T1[(a,in),(r,c)] A[l,r,in,k]: one product
    // with rows (a,c), columns (l,k) and contracted (in,r)
    mgemm_map<T, false, false, M == MODE_BF16, IsCplx<T>::value>(
        bl * nbr, v.Dl * v.Dout, v.Din * v.Dr, T1, IMap(nbr, v.Din * v.Dr * nbr, 1), IMap(nbr),
        Abuf, IMap(v.Dr, v.s_in, v.s_r), IMap(v.Dout, v.s_l, v.s_out), Z,
        IMap(nbr, v.Dl * np, 1), IMap(v.Dout, np, nbr), false, false);
    __syncthreads();
    int rnew;
    int rkeep_row = 1;
    if (y > 0) {
      const T* Gy = Gs + (size_t)y * np2;
      // Y = G_y Z, rho = Z^H Y (Hermitian)
      mgemm<T, IsCplx<T>::value, false, M == MODE_BF16, IsCplx<T>::value>(Pl, zc, Pl, Gy, 1, np, Z, np, 1, X, np, false, false);
      __syncthreads();
      mgemm<T, IsCplx<T>::value, false, M == MODE_BF16, IsCplx<T>::value>(zc, zc, Pl, Z, 1, np, X, np, 1, Pk, np, true, false);
      __syncthreads();
      // unit scale (eigenvectors only)
      R mx = 0;
      for (int i = tid; i < zc; i += NT) {
        const R a = absx(Pk[(size_t)i * np + i]);
        mx = a > mx ? a : mx;
      }
      mx = block_max(mx, reinterpret_cast<R*>(sh.red + 16 * slot));
      const int es = pow2_exponent((double)mx);
      const R fsc = (R)ldexp(1.0, -es);
      // trace (for the truncated weight) at unit scale
      double trc = 0;
      for (int i = tid; i < zc; i += NT) trc += (double)realx(Pk[(size_t)i * np + i]) * (double)fsc;
      if (es != 0)
        for (int i = tid; i < zc * zc; i += NT) Pk[(size_t)(i / zc) * np + (i % zc)] *= fsc;
      trc = block_sum(trc, reinterpret_cast<double*>(sh.red + 16 * slot));
      __syncthreads();
      rnew = rs < zc ? rs : zc;
      const int rr = rnew + 1 < zc ? rnew + 1 : zc;
      R tnorm;
      dm_eig<T, M != MODE_BF16>(Pk, np, zc, rnew, rr, Hv, Yt, lu, sh, slot, tnorm);
      // kept count and cut flags from the eigenvalues (lam = sigma^2)
      __shared__ int s_keep;
      if (tid == 0) {
        int keep = rnew;
        if (L.trunc_w > 0.0) {
          double kept = 0;
          for (int j = 0; j < rnew; ++j) kept += (double)(sh.lam[j] > R(0) ? sh.lam[j] : R(0));
          const double lim = L.trunc_w * trc;
          double tail = trc - kept;
          if (tail < 0) tail = 0;
          if (tail <= lim) {
            for (int j = rnew - 1; j >= 1; --j) {
              const double lj = sh.lam[j] > R(0) ? (double)sh.lam[j] : 0.0;
              if (tail + lj > lim) break;
              tail += lj;
              keep = j;
            }
          }
          const double marg = std::is_same<R, double>::value ? 1e-8 : 1e-4;
          bool near = fabs(tail - lim) <= marg * lim;
          if (keep > 1 && tail <= lim) {
            const double lp = sh.lam[keep - 1] > R(0) ? (double)sh.lam[keep - 1] : 0.0;
            near = near || fabs(tail + lp - lim) <= marg * lim;
          }
          if (near) fl |= 8;
        }
        if (keep < zc && keep < rr) {
          const double sa = sqrt(fmax((double)sh.lam[keep - 1], 0.0));
          const double sb = sqrt(fmax((double)sh.lam[keep], 0.0));
          if (sa > 0.0 && (sa - sb) < 1e-8 * sa) fl |= 8;
        }
        s_keep = keep;
      }
      __syncthreads();
      const int rkeep = s_keep;
      rkeep_row = rkeep;
      // discarded columns of the kept block are zero
      T* Xe = sh.big;
      if (rkeep < rnew)
        for (int i = tid; i < zc * rnew; i += NT)
          if (i % rnew >= rkeep) Xe[i] = T(0);
      __syncthreads();
      // W_y = Z [v_0 .. v_{rnew-1}]
      mgemm<T, false, false, M == MODE_BF16, IsCplx<T>::value>(Pl, rnew, zc, Z, np, 1, Xe, rnew, 1, W, np, false, false);
      // the new tensor B[j, e] = conj(v_j[e]) / max |v|
      R bm = 0;
      for (int i = tid; i < zc * rnew; i += NT) {
        const R a = absx(Xe[i]);
        bm = a > bm ? a : bm;
      }
      bm = block_max(bm, reinterpret_cast<R*>(sh.red + 16 * slot));
      const R binv = bm > R(0) ? R(1) / bm : R(1);
      if (!(bm > R(0)) || !isfinite((double)bm)) {
        if (tid == 0) fl |= (bm == R(0)) ? 1 : 2;
      } else {
        logrow += log((double)bm);
      }
      T* dst = Enew + (size_t)y * L.site_box;
      const int kc = v.Dout * nbrs;
      for (int i = tid; i < rs * kc; i += NT) {
        const int j = i / kc, rem = i - j * kc, k = rem / nbrs, c = rem - k * nbrs;
        dst[i] = (j < rkeep && c < nbr) ? conjx(Xe[(k * nbr + c) * rnew + j]) * binv : T(0);
      }
      if (tid == 0) knew[y] = rkeep;
      __syncthreads();
      // W carries the weight of the sites to its right: unit scale, the
      // power of two into the log scale
      R wm = 0;
      for (int i = tid; i < Pl * rnew; i += NT) {
        const R a = absx(W[(size_t)(i / rnew) * np + (i % rnew)]);
        wm = a > wm ? a : wm;
      }
      wm = block_max(wm, reinterpret_cast<R*>(sh.red + 16 * slot));
      const int ew = pow2_exponent((double)wm);
      if (ew != 0) {
        const R f = (R)ldexp(1.0, -ew);
        for (int i = tid; i < Pl * rnew; i += NT) W[(size_t)(i / rnew) * np + (i % rnew)] *= f;
      }
      logrow += ew * 0.69314718055994530942;
      __syncthreads();
    } else {
      rnew = 1;
      // the leftmost tensor is Z itself (1 x zc)
      R zm = 0;
      for (int i = tid; i < zc; i += NT) {
        const R a = absx(Z[i]);
        zm = a > zm ? a : zm;
      }
      zm = block_max(zm, reinterpret_cast<R*>(sh.red + 16 * slot));
      if (!(zm > R(0)) || !isfinite((double)zm)) {
        if (tid == 0) fl |= (zm == R(0)) ? 1 : 2;
        zm = R(1);
      } else {
        logrow += log((double)zm);
      }
      const R zinv = R(1) / zm;
      T* dst = Enew + (size_t)y * L.site_box;
      for (int i = tid; i < v.Dout * nbrs; i += NT) {
        const int k = i / nbrs, c = i - k * nbrs;
        dst[i] = c < nbr ? Z[k * nbr + c] * zinv : T(0);
      }
      if (tid == 0) {
        knew[0] = 1;
        knew[L.Ly] = 1;
      }
      __syncthreads();
    }
    nbr = y > 0 ? rkeep_row : 1;
  }
  if (tid == 0) lg[sn] = lg[sp] + logrow;
  __syncthreads();
}

// Persistent grid over (sample, direction) tasks.
// FP32 modes: two workgroups per CU (four waves per SIMD: registers capped at
// 128 per lane) so
// one workgroup's eigensolver overlaps the other's matrix-core products
template <int M>
__global__ void __launch_bounds__(512, (M == MODE_F32 || M == MODE_BF16 || M == MODE_C64) ? 4 : 2)
k_env_dm(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
         const uint8_t* __restrict__ samples, typename ModeT<M>::T* __restrict__ env,
         double* __restrict__ logs, int* __restrict__ flags, int n, int ndir, int dir0,
         typename ModeT<M>::T* __restrict__ slabs, size_t slab) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const DmSh<T> sh(smem_raw, L.bmax, L.D, L.chi);
  T* myslab = slabs + (size_t)blockIdx.x * slab;
  __shared__ int fl;
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  for (int task = blockIdx.x; task < n * ndir; task += gridDim.x) {
    const int smp = task / ndir;
    const int dir = dir0 + (task - smp * ndir);
    const bool bottom = dir == 1;
    if (threadIdx.x == 0) fl = 0;
    __syncthreads();
    int slot = 0;
    const uint8_t* s = samples + (size_t)smp * L.N;
    T* envs = env + (size_t)smp * L.n_slots * slot_elems;
    double* lg = logs + (size_t)smp * L.n_slots;
    // the first row of the sweep read as an MPS (Ebuf and red of the
    // canonical kernel's carve-up)
    EnvSmem<T> es(sh.big, sh.red, L, false);
    es.Ebuf = sh.big;
    es.red = sh.red;
    env_first_row<M>(L, tab, theta, s, bottom, envs, lg, es, &fl);
    // kept bonds of the environment absorbed next (the first row's: exact)
    __shared__ int kb[2][33];
    dm_first_bonds(L, tab, bottom ? slot_bottom(L, L.Lx - 1) : slot_top(L, 0), kb[0]);
    for (int t = 1; t <= L.Lx - 2; ++t)
      dm_absorb_row<M>(L, tab, theta, s, bottom, t, envs, lg, myslab, sh, &fl, slot,
                       kb[(t - 1) & 1], kb[t & 1]);
    if (threadIdx.x == 0 && fl && flags) atomicOr(flags + smp, fl);
    __syncthreads();
  }
}

// The sampler's environment phase with the density-matrix truncation: one
// workgroup per chain (grid = chains); row < 0 rebuilds the bottom
// environments of the chain's state, row >= 0 absorbs that row into the top
// environment (row 0: the first row read as an MPS).
template <int M>
__global__ void __launch_bounds__(512, (M == MODE_F32 || M == MODE_BF16 || M == MODE_C64) ? 4 : 2)
k_smp_env_dm(Lattice L, const int* __restrict__ tab,
             const typename ModeT<M>::T* __restrict__ theta, int n_chains, int row,
             const uint8_t* __restrict__ state, typename ModeT<M>::T* __restrict__ env,
             double* __restrict__ logs, typename ModeT<M>::T* __restrict__ slabs, size_t slab) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int chain = blockIdx.x;
  if (chain >= n_chains) return;
  const DmSh<T> sh(smem_raw, L.bmax, L.D, L.chi);
  T* myslab = slabs + (size_t)chain * slab;
  __shared__ int fl;
  if (threadIdx.x == 0) fl = 0;
  __syncthreads();
  int slot = 0;
  const bool bottom = row < 0;
  const uint8_t* s = state + (size_t)chain * L.N;
  T* envs = env + (size_t)chain * L.n_slots * ((size_t)L.Ly * L.site_box);
  double* lg = logs + (size_t)chain * L.n_slots;
  if (row <= 0) {
    EnvSmem<T> es(sh.big, sh.red, L, false);
    es.Ebuf = sh.big;
    es.red = sh.red;
    env_first_row<M>(L, tab, theta, s, bottom, envs, lg, es, &fl);
  }
  const int t0 = bottom ? 1 : row, t1 = bottom ? L.Lx - 2 : row;
  // kept bonds carried within this launch; a top row absorbed alone reads
  // the previous row's tensors over their stored (chi-wide, zero-padded)
  // bonds
  __shared__ int kb[2][33];
  const int tf = t0 > 1 ? t0 : 1;
  dm_first_bonds(L, tab, bottom ? slot_bottom(L, L.Lx - 1) : slot_top(L, tf - 1), kb[0]);
  for (int t = tf; t <= t1; ++t)
    dm_absorb_row<M>(L, tab, theta, s, bottom, t, envs, lg, myslab, sh, &fl, slot,
                     kb[(t - tf) & 1], kb[(t - tf + 1) & 1]);
}

// ---- host side ----
static size_t dm_rsize(int mode) {
  return (mode == MODE_F64 || mode == MODE_C128) ? 8 : 4;
}

size_t env_dm_slab_elems(const Lattice& L, int mode) {
  return (dm_slab_elems(L.Ly, L.bmax, L.D, L.chi, mode_elem_bytes(mode), dm_rsize(mode)) + 63) /
         64 * 64;
}
size_t env_dm_lds_bytes(const Lattice& L, int mode) {
  return dm_lds_bytes(L.bmax, L.D, L.chi, mode_elem_bytes(mode), dm_rsize(mode));
}
// Resident workgroups of the persistent grid: the occupancy of the
// kernel's instance times the compute units, at most one per task.
template <int M>
static int dm_blocks_m(const Lattice& L) {
  int dev = 0, cus = 256, per = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  const size_t lds = env_dm_lds_bytes(L, M);
  hipFuncSetAttribute((const void*)k_env_dm<M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_env_dm<M>, 512, lds) ==
          hipSuccess &&
      nb > 0)
    per = nb;
  return per * cus;
}
int env_dm_grid(const Lattice& L, int mode, int tasks) {
  int g = 0;
  switch (mode) {
    case MODE_F64: g = dm_blocks_m<MODE_F64>(L); break;
    case MODE_F32: g = dm_blocks_m<MODE_F32>(L); break;
    case MODE_BF16: g = dm_blocks_m<MODE_BF16>(L); break;
    case MODE_C128: g = dm_blocks_m<MODE_C128>(L); break;
    default: g = dm_blocks_m<MODE_C64>(L); break;
  }
  return tasks < g ? (tasks > 0 ? tasks : 1) : g;
}

template <int M>
hipError_t launch_env_dm(const Lattice& L, const int* tab, const void* theta,
                         const uint8_t* samples, void* env, double* logs, int* flags, int n,
                         void* slabs, int grid, hipStream_t st, bool bottom_only) {
  typedef typename ModeT<M>::T T;
  const size_t lds = env_dm_lds_bytes(L, M);
  hipError_t e = hipFuncSetAttribute((const void*)k_env_dm<M>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_env_dm<M>), dim3(grid), dim3(512), lds, st, L, tab, (const T*)theta,
                     samples, (T*)env, logs, flags, n, bottom_only ? 1 : 2, bottom_only ? 1 : 0,
                     (T*)slabs, env_dm_slab_elems(L, M));
  return hipGetLastError();
}

#define INST(M)                                                                              \
  template hipError_t launch_env_dm<M>(const Lattice&, const int*, const void*, const uint8_t*, \
                                       void*, double*, int*, int, void*, int, hipStream_t, bool);
INST(MODE_F64)
INST(MODE_F32)
INST(MODE_BF16)
INST(MODE_C128)
INST(MODE_C64)
#undef INST

template <int M>
static hipError_t smp_env_dm_m(const Lattice& L, const int* tab, const void* theta, int n_chains,
                               int row, const uint8_t* state, void* env, double* logs,
                               void* slabs, hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const size_t lds = env_dm_lds_bytes(L, M);
  const hipError_t e = hipFuncSetAttribute((const void*)k_smp_env_dm<M>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_smp_env_dm<M>, dim3(n_chains), dim3(512), lds, st, L, tab,
                     (const T*)theta, n_chains, row, state, (T*)env, logs, (T*)slabs,
                     env_dm_slab_elems(L, M));
  return hipGetLastError();
}

hipError_t launch_smp_env_dm(const Lattice& L, const int* tab, int mode, const void* theta,
                             int n_chains, int row, const uint8_t* state, void* env, double* logs,
                             void* slabs, hipStream_t st) {
  switch (mode) {
    case MODE_F64:
      return smp_env_dm_m<MODE_F64>(L, tab, theta, n_chains, row, state, env, logs, slabs, st);
    case MODE_F32:
      return smp_env_dm_m<MODE_F32>(L, tab, theta, n_chains, row, state, env, logs, slabs, st);
    case MODE_BF16:
      return smp_env_dm_m<MODE_BF16>(L, tab, theta, n_chains, row, state, env, logs, slabs, st);
    case MODE_C128:
      return smp_env_dm_m<MODE_C128>(L, tab, theta, n_chains, row, state, env, logs, slabs, st);
    default:
      return smp_env_dm_m<MODE_C64>(L, tab, theta, n_chains, row, state, env, logs, slabs, st);
  }
}

}  // namespace pm
