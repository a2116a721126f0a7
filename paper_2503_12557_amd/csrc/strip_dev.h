// Device-side strip building blocks shared by the strip kernels and the
// sampler: one-row and two-row partial contractions, move coefficients.
#pragma once

#include "common.h"
#include "kernels.h"

namespace pm {

struct EnvRef {
  const void* p;
  int a, k, b;  // dims; p == nullptr means the trivial bond-1 environment
};

template <typename T>
__device__ __forceinline__ const T* env_site(const T* envs, const Lattice& L, int slot, int y) {
  return envs + ((size_t)slot * L.Ly + y) * L.site_box;
}

template <typename T>
__device__ __forceinline__ const T* tensor_of(const T* theta, const int* tab, const Lattice& L,
                                             int n, int p) {
  return theta + tab[L.off_param + n] + p * tab[L.off_block + n];
}

__device__ __forceinline__ void legs_of(const int* tab, const Lattice& L, int n, int& Dl, int& Dr,
                                        int& Du, int& Dd) {
  const int* lg = tab + L.off_legs + 4 * n;
  Dl = lg[0];
  Dr = lg[1];
  Du = lg[2];
  Dd = lg[3];
}

// ---------------------------------------------------------------------------
// One-row strip helpers. Up env U_y[a,u,b], down env B_y[c,d,e],
// site A[m,r,u,d], left partial L[a,m,c], right partial R[b,r,e].
// ---------------------------------------------------------------------------
template <int M, typename T>
__device__ void s1_step_left(const T* Lp, const T* U, int ua, int ub, const T* A, int Dl, int Dr,
                             int Du, int Dd, const T* Bt, int ba, int bb, T* X1, T* X2, T* Lout) {
  // X1[(m,c),(u,b)] = sum_a L[a,(m,c)] U[a,(u,b)]
  gemm<M>(Dl * ba, Du * ub, ua, Lp, 1, Dl * ba, U, Du * ub, 1, X1, Du * ub, 1, false);
  __syncthreads();
  // X2[b,r,c,d] = sum_{m,u} X1[m,c,u,b] A[m,r,u,d]
  const int tot = ub * Dr * ba * Dd;
  const FastDiv fDd(Dd), fba(ba), fDr(Dr);
  for (int i = threadIdx.x; i < tot; i += PEPS_NT) {
    int t = i;
    const int d = divmod(t, fDd);
    const int c = divmod(t, fba);
    const int r = divmod(t, fDr);
    const int b = t;
    T acc = 0;
    for (int m = 0; m < Dl; ++m)
      for (int u = 0; u < Du; ++u)
        acc += opnd<M>(X1[((m * ba + c) * Du + u) * ub + b]) *
               opnd<M>(A[((m * Dr + r) * Du + u) * Dd + d]);
    X2[i] = acc;
  }
  __syncthreads();
  // L'[(b,r), e] = sum_{(c,d)} X2[(b,r),(c,d)] B[(c,d), e]
  gemm<M>(ub * Dr, bb, ba * Dd, X2, ba * Dd, 1, Bt, bb, 1, Lout, bb, 1, false);
  __syncthreads();
}

template <int M, typename T>
__device__ void s1_step_right(const T* Rp, const T* U, int ua, int ub, const T* A, int Dl, int Dr,
                              int Du, int Dd, const T* Bt, int ba, int bb, T* X1, T* X2, T* Rout) {
  // X1[(a,u),(r,e)] = sum_b U[(a,u),b] R[b,(r,e)]
  gemm<M>(ua * Du, Dr * bb, ub, U, ub, 1, Rp, Dr * bb, 1, X1, Dr * bb, 1, false);
  __syncthreads();
  // X2[(a,m),(d,e)] = sum_{u,r} X1[a,u,r,e] A[m,r,u,d]
  const int tot = ua * Dl * Dd * bb;
  const FastDiv fbb(bb), fDd(Dd), fDl(Dl);
  for (int i = threadIdx.x; i < tot; i += PEPS_NT) {
    int t = i;
    const int e = divmod(t, fbb);
    const int d = divmod(t, fDd);
    const int m = divmod(t, fDl);
    const int a = t;
    T acc = 0;
    for (int u = 0; u < Du; ++u)
      for (int r = 0; r < Dr; ++r)
        acc += opnd<M>(X1[((a * Du + u) * Dr + r) * bb + e]) *
               opnd<M>(A[((m * Dr + r) * Du + u) * Dd + d]);
    X2[i] = acc;
  }
  __syncthreads();
  // R'[(a,m), c] = sum_{(d,e)} X2[(a,m),(d,e)] B[c,(d,e)]
  gemm<M>(ua * Dl, ba, Dd * bb, X2, Dd * bb, 1, Bt, 1, Dd * bb, Rout, ba, 1, false);
  __syncthreads();
}

template <typename T>
__device__ T lds_dot(const T* a, const T* b, int cnt, T* red) {
  T s = 0;
  for (int i = threadIdx.x; i < cnt; i += PEPS_NT) s += a[i] * b[i];
  return block_sum(s, red);
}

// Sum of <S|h_t|S'> over the contributions of a move: the coefficient of
// the move's amplitude ratio in E_loc(S).
__device__ void move_coef(const HamDev& H, const int* mv, const uint8_t* s, double& cre,
                          double& cim) {
  cre = 0.0;
  cim = 0.0;
  const int cs = mv[6], cc = mv[7];
  for (int q = 0; q < cc; ++q) {
    const int t = H.contrib[2 * (cs + q)], mask = H.contrib[2 * (cs + q) + 1];
    const int* tt = H.terms + 4 * t;
    const int k = tt[0];
    int c = 0;
    for (int j = 0; j < k; ++j) c = 2 * c + pbit(s[tt[1 + j]]);
    const int c2 = c ^ mask;
    const double* h = H.mats + ((size_t)t * 64 + c * 8 + c2) * 2;
    cre += h[0];
    cim += h[1];
  }
}

__device__ __forceinline__ bool in_move(const int* mv, int n) {
  const int ns = mv[2];
  for (int j = 0; j < ns; ++j)
    if (mv[3 + j] == n) return true;
  return false;
}

// ---------------------------------------------------------------------------
// Two-row strip: rows x (A1[m1,r1,u,t]) and x+1 (A2[m2,s,t,d]) between
// U = E^u[x-1] and B = E^l[x+2]. Left partial L[a,m1,m2,c], right partial
// R[b,r1,s,e]. Contractions are chunked over the outer environment bond, S2G
// bond indices per chunk, so the intermediates stay O(S2G chi D^3) and each
// chunk costs four workgroup barriers.
// ---------------------------------------------------------------------------
#define S2G 2

template <int M, typename T>
__device__ void s2_step_left(const T* Lp, const T* U, int ua, int uk, int ub, const T* A1,
                             int Dl1, int Dr1, int Dd1, const T* A2, int Dl2, int Dr2, int Dd2,
                             const T* Bt, int ba, int bb, T* X1, T* X2, T* X3, T* Lout) {
  const int inner = Dl1 * Dl2 * ba;
  const int n1 = inner * uk, n2 = Dl2 * ba * Dr1 * Dd1, n3 = Dr1 * Dr2 * ba * Dd2;
  const FastDiv fDd1(Dd1), fDr1(Dr1), fba(ba), fn2(n2);
  const FastDiv fDd2(Dd2), fDr2(Dr2), fn3(n3);
  for (int b0 = 0; b0 < ub; b0 += S2G) {
    const int nb = ub - b0 < S2G ? ub - b0 : S2G;
    // X1[g][(m1,m2,c), u] = sum_a L[a,(m1,m2,c)] U[a,u,b0+g]
    for (int g = 0; g < nb; ++g)
      gemm<M>(inner, uk, ua, Lp, 1, inner, U + b0 + g, uk * ub, ub, X1 + g * n1, uk, 1, false);
    __syncthreads();
    // X2[g][m2,c,r1,t] = sum_{m1,u} X1[g][m1,m2,c,u] A1[m1,r1,u,t]
    for (int i = threadIdx.x; i < nb * n2; i += PEPS_NT) {
      int q = i;
      const int j = divmod(q, fn2);
      const int g = q;
      q = j;
      const int t = divmod(q, fDd1);
      const int r1 = divmod(q, fDr1);
      const int c = divmod(q, fba);
      const int m2 = q;
      const T* x1 = X1 + g * n1;
      T acc = 0;
      for (int m1 = 0; m1 < Dl1; ++m1)
        for (int u = 0; u < uk; ++u)
          acc += opnd<M>(x1[((m1 * Dl2 + m2) * ba + c) * uk + u]) *
                 opnd<M>(A1[((m1 * Dr1 + r1) * uk + u) * Dd1 + t]);
      X2[i] = acc;
    }
    __syncthreads();
    // X3[g][r1,s,c,d] = sum_{m2,t} X2[g][m2,c,r1,t] A2[m2,s,t,d]
    for (int i = threadIdx.x; i < nb * n3; i += PEPS_NT) {
      int q = i;
      const int j = divmod(q, fn3);
      const int g = q;
      q = j;
      const int d = divmod(q, fDd2);
      const int c = divmod(q, fba);
      const int sidx = divmod(q, fDr2);
      const int r1 = q;
      const T* x2 = X2 + g * n2;
      T acc = 0;
      for (int m2 = 0; m2 < Dl2; ++m2)
        for (int t = 0; t < Dd1; ++t)
          acc += opnd<M>(x2[((m2 * ba + c) * Dr1 + r1) * Dd1 + t]) *
                 opnd<M>(A2[((m2 * Dr2 + sidx) * Dd1 + t) * Dd2 + d]);
      X3[i] = acc;
    }
    __syncthreads();
    // L'[b0+g,(r1,s),e] = sum_{(c,d)} X3[g][(r1,s),(c,d)] B[(c,d),e]
    gemm<M>(nb * Dr1 * Dr2, bb, ba * Dd2, X3, ba * Dd2, 1, Bt, bb, 1,
            Lout + b0 * (Dr1 * Dr2 * bb), bb, 1, false);
    __syncthreads();
  }
}

template <int M, typename T>
__device__ void s2_step_right(const T* Rp, const T* U, int ua, int uk, int ub, const T* A1,
                              int Dl1, int Dr1, int Dd1, const T* A2, int Dl2, int Dr2, int Dd2,
                              const T* Bt, int ba, int bb, T* Y1, T* Y2, T* Y3, T* Rout) {
  const int rw = Dr1 * Dr2 * bb;
  const int n1 = uk * rw, n2 = Dl1 * Dd1 * Dr2 * bb, n3 = Dl1 * Dl2 * Dd2 * bb;
  const FastDiv fbb(bb), fDr2(Dr2), fDd1(Dd1), fn2(n2);
  const FastDiv fDd2(Dd2), fDl2(Dl2), fn3(n3);
  for (int a0 = 0; a0 < ua; a0 += S2G) {
    const int na = ua - a0 < S2G ? ua - a0 : S2G;
    // Y1[g][u,(r1,s,e)] = sum_b U[a0+g,u,b] R[b,(r1,s,e)]: rows (g, u)
    gemm<M>(na * uk, rw, ub, U + a0 * uk * ub, ub, 1, Rp, rw, 1, Y1, rw, 1, false);
    __syncthreads();
    // Y2[g][m1,t,s,e] = sum_{u,r1} A1[m1,r1,u,t] Y1[g][u,r1,s,e]
    for (int i = threadIdx.x; i < na * n2; i += PEPS_NT) {
      int q = i;
      const int j = divmod(q, fn2);
      const int g = q;
      q = j;
      const int e = divmod(q, fbb);
      const int sidx = divmod(q, fDr2);
      const int t = divmod(q, fDd1);
      const int m1 = q;
      const T* y1 = Y1 + g * n1;
      T acc = 0;
      for (int u = 0; u < uk; ++u)
        for (int r1 = 0; r1 < Dr1; ++r1)
          acc += opnd<M>(A1[((m1 * Dr1 + r1) * uk + u) * Dd1 + t]) *
                 opnd<M>(y1[((u * Dr1 + r1) * Dr2 + sidx) * bb + e]);
      Y2[i] = acc;
    }
    __syncthreads();
    // Y3[g][(m1,m2),(d,e)] = sum_{t,s} A2[m2,s,t,d] Y2[g][m1,t,s,e]
    for (int i = threadIdx.x; i < na * n3; i += PEPS_NT) {
      int q = i;
      const int j = divmod(q, fn3);
      const int g = q;
      q = j;
      const int e = divmod(q, fbb);
      const int d = divmod(q, fDd2);
      const int m2 = divmod(q, fDl2);
      const int m1 = q;
      const T* y2 = Y2 + g * n2;
      T acc = 0;
      for (int t = 0; t < Dd1; ++t)
        for (int sidx = 0; sidx < Dr2; ++sidx)
          acc += opnd<M>(A2[((m2 * Dr2 + sidx) * Dd1 + t) * Dd2 + d]) *
                 opnd<M>(y2[((m1 * Dd1 + t) * Dr2 + sidx) * bb + e]);
      Y3[i] = acc;
    }
    __syncthreads();
    // R'[a0+g,(m1,m2),c] = sum_{(d,e)} Y3[g][(m1,m2),(d,e)] B[c,(d,e)]
    gemm<M>(na * Dl1 * Dl2, ba, Dd2 * bb, Y3, Dd2 * bb, 1, Bt, 1, Dd2 * bb,
            Rout + a0 * (Dl1 * Dl2 * ba), ba, 1, false);
    __syncthreads();
  }
}

}  // namespace pm
