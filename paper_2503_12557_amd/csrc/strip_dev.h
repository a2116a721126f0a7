// Device-side strip building blocks shared by the strip kernels and the
// sampler: one-row and two-row partial contractions, move coefficients.
#pragma once

#include "common.h"
#include "kernels.h"
#include "mfma.h"

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

// ---------------------------------------------------------------------------
// FP32 / BF16 two-row steps for the bulk of a D = 4 lattice: the physical
// legs that carry the inner products (up leg of the upper row, down legs of
// both rows) have dimension 4, so every contraction keeps four outputs per
// thread and reads its operands as 16-byte vectors. Same contractions, same
// chunking and buffers as the general steps below; each sum runs over its
// index in the same order, only its partial sums are grouped differently.
// Every operand (partials, staged environments and tensors, chunk
// intermediates) must be 16-byte aligned.
// ---------------------------------------------------------------------------

// left step with uk = Dd1 = Dd2 = 4 and Dl1 Dl2 ba a multiple of 4
template <int M>
__device__ __forceinline__ void s2_step_left_f4(const float* Lp, const float* U, int ua, int ub, const float* A1,
                                int Dl1, int Dr1, const float* A2, int Dl2, int Dr2,
                                const float* Bt, int ba, int bb, float* X1, float* X2, float* X3,
                                float* Lout) {
  const int tid = threadIdx.x;
  const int inner = Dl1 * Dl2 * ba;
  const int n1 = inner * 4, n2 = Dl2 * ba * Dr1 * 4, n3 = Dr1 * Dr2 * ba * 4;
  const int q1 = inner >> 2, K4 = ba * 4, nrs = Dr1 * Dr2;
  const FastDiv fq1(q1), fDr1(Dr1), fDr2(Dr2), fba(ba), fDl2(Dl2), fbb(bb), fnrs(nrs);
  for (int b0 = 0; b0 < ub; b0 += S2G) {
    const int nb = ub - b0 < S2G ? ub - b0 : S2G;
    // X1[g][row][u] = sum_a L[a][row] U[a][u][b0+g]: four rows per thread
    for (int task = tid; task < nb * inner; task += PEPS_NT) {
      const int u = task & 3;
      int q = task >> 2;
      const int rq = divmod(q, fq1);
      const int g = q;
      const float* lp = Lp + rq * 4;
      const float* up = U + u * ub + b0 + g;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 4
      for (int a = 0; a < ua; ++a) fma4(acc, opnd<M>(up[a * 4 * ub]), op4<M>(ld4(lp + a * inner)));
      float* x1 = X1 + g * n1 + rq * 16 + u;
      x1[0] = acc.x;
      x1[4] = acc.y;
      x1[8] = acc.z;
      x1[12] = acc.w;
    }
    __syncthreads();
    // X2[g][m2][c][r1][t] = sum_{m1,u} X1[g][m1][m2][c][u] A1[m1][r1][u][t]
    for (int task = tid; task < nb * Dl2 * ba * Dr1; task += PEPS_NT) {
      int q = task;
      const int r1 = divmod(q, fDr1);
      const int c = divmod(q, fba);
      const int m2 = divmod(q, fDl2);
      const int g = q;
      const float* x1 = X1 + g * n1 + (m2 * ba + c) * 4;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 2
      for (int m1 = 0; m1 < Dl1; ++m1) {
        const float4 xv = op4<M>(ld4(x1 + m1 * Dl2 * ba * 4));
        const float* ap = A1 + (m1 * Dr1 + r1) * 16;
        fma4(acc, xv.x, op4<M>(ld4(ap)));
        fma4(acc, xv.y, op4<M>(ld4(ap + 4)));
        fma4(acc, xv.z, op4<M>(ld4(ap + 8)));
        fma4(acc, xv.w, op4<M>(ld4(ap + 12)));
      }
      st4(X2 + g * n2 + ((m2 * ba + c) * Dr1 + r1) * 4, acc);
    }
    __syncthreads();
    // X3[g][r1][s][c][d] = sum_{m2,t} X2[g][m2][c][r1][t] A2[m2][s][t][d]
    for (int task = tid; task < nb * nrs * ba; task += PEPS_NT) {
      int q = task;
      const int c = divmod(q, fba);
      const int sx = divmod(q, fDr2);
      const int r1 = divmod(q, fDr1);
      const int g = q;
      const float* x2 = X2 + g * n2 + (c * Dr1 + r1) * 4;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 2
      for (int m2 = 0; m2 < Dl2; ++m2) {
        const float4 xv = op4<M>(ld4(x2 + m2 * ba * Dr1 * 4));
        const float* ap = A2 + (m2 * Dr2 + sx) * 16;
        fma4(acc, xv.x, op4<M>(ld4(ap)));
        fma4(acc, xv.y, op4<M>(ld4(ap + 4)));
        fma4(acc, xv.z, op4<M>(ld4(ap + 8)));
        fma4(acc, xv.w, op4<M>(ld4(ap + 12)));
      }
      st4(X3 + g * n3 + ((r1 * Dr2 + sx) * ba + c) * 4, acc);
    }
    __syncthreads();
    // L'[b0+g][r1 s][e] = sum_{(c,d)} X3[g][r1 s][(c,d)] B[(c,d)][e]
    for (int task = tid; task < nb * nrs * bb; task += PEPS_NT) {
      int q = task;
      const int e = divmod(q, fbb);
      const int rs = divmod(q, fnrs);
      const int g = q;
      const float* x3 = X3 + g * n3 + rs * K4;
      const float* bp = Bt + e;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll 2
      for (int k = 0; k < K4; k += 4) {
        const float4 xv = op4<M>(ld4(x3 + k));
        s0 = fmaf(xv.x, opnd<M>(bp[k * bb]), s0);
        s1 = fmaf(xv.y, opnd<M>(bp[(k + 1) * bb]), s1);
        s2 = fmaf(xv.z, opnd<M>(bp[(k + 2) * bb]), s2);
        s3 = fmaf(xv.w, opnd<M>(bp[(k + 3) * bb]), s3);
      }
      Lout[((b0 + g) * nrs + rs) * bb + e] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
  }
}

// right step with uk = Dd1 = Dd2 = 4 and bb a multiple of 4
template <int M>
__device__ __forceinline__ void s2_step_right_f4(const float* Rp, const float* U, int ua, int ub, const float* A1,
                                 int Dl1, int Dr1, const float* A2, int Dl2, int Dr2,
                                 const float* Bt, int ba, int bb, float* Y1, float* Y2, float* Y3,
                                 float* Rout) {
  const int tid = threadIdx.x;
  const int rw = Dr1 * Dr2 * bb;
  const int n1 = 4 * rw, n2 = Dl1 * 4 * Dr2 * bb, n3 = Dl1 * Dl2 * 4 * bb;
  const int q1 = rw >> 2, eq = bb >> 2, K = 4 * bb, nrow = Dl1 * Dl2;
  const FastDiv fq1(q1), feq(eq), fDr2(Dr2), fDl1(Dl1), fDl2(Dl2), fba(ba), fnrow(nrow);
  for (int a0 = 0; a0 < ua; a0 += S2G) {
    const int na = ua - a0 < S2G ? ua - a0 : S2G;
    // Y1[g][u][(r1,s,e)] = sum_b U[a0+g][u][b] R[b][(r1,s,e)]: four columns per thread
    for (int task = tid; task < na * 4 * q1; task += PEPS_NT) {
      int q = task;
      const int cq = divmod(q, fq1);
      const int u = q & 3;
      const int g = q >> 2;
      const float* up = U + ((a0 + g) * 4 + u) * ub;
      const float* rp = Rp + cq * 4;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 4
      for (int b = 0; b < ub; ++b) fma4(acc, opnd<M>(up[b]), op4<M>(ld4(rp + b * rw)));
      st4(Y1 + g * n1 + u * rw + cq * 4, acc);
    }
    __syncthreads();
    // Y2[g][m1][t][s][e] = sum_{u,r1} A1[m1][r1][u][t] Y1[g][u][r1][s][e]
    for (int task = tid; task < na * Dl1 * 4 * Dr2 * eq; task += PEPS_NT) {
      int q = task;
      const int ei = divmod(q, feq);
      const int sx = divmod(q, fDr2);
      const int t = q & 3;
      q >>= 2;
      const int m1 = divmod(q, fDl1);
      const int g = q;
      const float* y1 = Y1 + g * n1 + sx * bb + ei * 4;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int u = 0; u < 4; ++u)
#pragma unroll 2
        for (int r1 = 0; r1 < Dr1; ++r1)
          fma4(acc, opnd<M>(A1[((m1 * Dr1 + r1) * 4 + u) * 4 + t]),
               op4<M>(ld4(y1 + u * rw + r1 * Dr2 * bb)));
      st4(Y2 + g * n2 + ((m1 * 4 + t) * Dr2 + sx) * bb + ei * 4, acc);
    }
    __syncthreads();
    // Y3[g][m1][m2][d][e] = sum_{t,s} A2[m2][s][t][d] Y2[g][m1][t][s][e]
    for (int task = tid; task < na * nrow * 4 * eq; task += PEPS_NT) {
      int q = task;
      const int ei = divmod(q, feq);
      const int d = q & 3;
      q >>= 2;
      const int m2 = divmod(q, fDl2);
      const int m1 = divmod(q, fDl1);
      const int g = q;
      const float* y2 = Y2 + g * n2 + m1 * 4 * Dr2 * bb + ei * 4;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int t = 0; t < 4; ++t)
#pragma unroll 2
        for (int sx = 0; sx < Dr2; ++sx)
          fma4(acc, opnd<M>(A2[((m2 * Dr2 + sx) * 4 + t) * 4 + d]),
               op4<M>(ld4(y2 + (t * Dr2 + sx) * bb)));
      st4(Y3 + g * n3 + ((m1 * Dl2 + m2) * 4 + d) * bb + ei * 4, acc);
    }
    __syncthreads();
    // R'[a0+g][(m1,m2)][c] = sum_{(d,e)} Y3[g][(m1,m2)][(d,e)] B[c][(d,e)]
    for (int task = tid; task < na * nrow * ba; task += PEPS_NT) {
      int q = task;
      const int c = divmod(q, fba);
      const int mm = divmod(q, fnrow);
      const int g = q;
      const float* y3 = Y3 + g * n3 + mm * K;
      const float* bp = Bt + c * K;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 2
      for (int k = 0; k < K; k += 4) {
        const float4 yv = op4<M>(ld4(y3 + k));
        const float4 bv = op4<M>(ld4(bp + k));
        acc.x = fmaf(yv.x, bv.x, acc.x);
        acc.y = fmaf(yv.y, bv.y, acc.y);
        acc.z = fmaf(yv.z, bv.z, acc.z);
        acc.w = fmaf(yv.w, bv.w, acc.w);
      }
      Rout[((a0 + g) * nrow + mm) * ba + c] = (acc.x + acc.y) + (acc.z + acc.w);
    }
    __syncthreads();
  }
}

template <int M, typename T>
__device__ __forceinline__ void s2_step_left(const T* Lp, const T* U, int ua, int uk, int ub, const T* A1,
                             int Dl1, int Dr1, int Dd1, const T* A2, int Dl2, int Dr2, int Dd2,
                             const T* Bt, int ba, int bb, T* X1, T* X2, T* X3, T* Lout) {
  if constexpr (std::is_same<T, float>::value) {
    if (uk == 4 && Dd1 == 4 && Dd2 == 4 && ((Dl1 * Dl2 * ba) & 3) == 0) {
      s2_step_left_f4<M>(Lp, U, ua, ub, A1, Dl1, Dr1, A2, Dl2, Dr2, Bt, ba, bb, X1, X2, X3, Lout);
      return;
    }
  }
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
__device__ __forceinline__ void s2_step_right(const T* Rp, const T* U, int ua, int uk, int ub, const T* A1,
                              int Dl1, int Dr1, int Dd1, const T* A2, int Dl2, int Dr2, int Dd2,
                              const T* Bt, int ba, int bb, T* Y1, T* Y2, T* Y3, T* Rout) {
  if constexpr (std::is_same<T, float>::value) {
    if (uk == 4 && Dd1 == 4 && Dd2 == 4 && (bb & 3) == 0) {
      s2_step_right_f4<M>(Rp, U, ua, ub, A1, Dl1, Dr1, A2, Dl2, Dr2, Bt, ba, bb, Y1, Y2, Y3, Rout);
      return;
    }
  }
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


// ---------------------------------------------------------------------------
// One-row steps on the matrix cores for the large shapes: three products
// per step over the whole outer bond (index maps absorb the leg order), the
// intermediates (B^2 D^2 elements each) in X1 / X2. Same contractions and
// output layouts as s1_step_left / s1_step_right.
// ---------------------------------------------------------------------------
template <typename T, bool BF = false>
__device__ __forceinline__ void s1_step_left_mm(const T* Lp, const T* U, int ua, int ub, const T* A, int Dl,
                                int Dr, int Du, int Dd, const T* Bt, int ba, int bb, T* X1, T* X2,
                                T* Lout) {
  // X1[(m,c),(u,b)] = sum_a L[a,(m,c)] U[a,(u,b)]
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(Dl * ba, Du * ub, ua, Lp, IMap(1), IMap(Dl * ba), U, IMap(Du * ub),
                             IMap(1), X1, IMap(Du * ub), IMap(1), false, false);
  __syncthreads();
  // X2[(c,b),(r,d)] = sum_{(m,u)} X1[(m,c),(u,b)] A[m,r,u,d]
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ba * ub, Dr * Dd, Dl * Du, X1, IMap(ub, Du * ub, 1),
                             IMap(Du, ba * Du * ub, ub), A, IMap(Du, Dr * Du * Dd, Dd),
                             IMap(Dd, Du * Dd, 1), X2, IMap(Dr * Dd), IMap(1), false, false);
  __syncthreads();
  // L'[(b,r),e] = sum_{(c,d)} X2[(c,b),(r,d)] B[(c,d),e]
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ub * Dr, bb, ba * Dd, X2, IMap(Dr, Dr * Dd, Dd),
                             IMap(Dd, ub * Dr * Dd, 1), Bt, IMap(bb), IMap(1), Lout, IMap(bb),
                             IMap(1), false, false);
  __syncthreads();
}

template <typename T, bool BF = false>
__device__ void s1_step_right_mm(const T* Rp, const T* U, int ua, int ub, const T* A, int Dl,
                                 int Dr, int Du, int Dd, const T* Bt, int ba, int bb, T* X1,
                                 T* X2, T* Rout) {
  // X1[(a,u),(r,e)] = sum_b U[(a,u),b] R[b,(r,e)]
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ua * Du, Dr * bb, ub, U, IMap(ub), IMap(1), Rp, IMap(Dr * bb),
                             IMap(1), X1, IMap(Dr * bb), IMap(1), false, false);
  __syncthreads();
  // X2[(a,e),(m,d)] = sum_{(u,r)} X1[(a,u),(r,e)] A[m,r,u,d]
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ua * bb, Dl * Dd, Du * Dr, X1, IMap(bb, Du * Dr * bb, 1), IMap(bb),
                             A, IMap(Dr, Dd, Du * Dd), IMap(Dd, Dr * Du * Dd, 1), X2,
                             IMap(Dl * Dd), IMap(1), false, false);
  __syncthreads();
  // R'[(a,m),c] = sum_{(d,e)} X2[(a,e),(m,d)] B[c,(d,e)]
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ua * Dl, ba, Dd * bb, X2, IMap(Dl, bb * Dl * Dd, Dd),
                             IMap(bb, 1, Dl * Dd), Bt, IMap(1), IMap(Dd * bb), Rout, IMap(ba),
                             IMap(1), false, false);
  __syncthreads();
}

// Hole tensor of a one-row strip site on the matrix cores:
// Env[m,r,u,d] = sum_{(c,b)} X1[(m,c),(u,b)] Q[(b,r),(c,d)] with
// X1 = L U and Q[(b,r),(c,d)] = sum_e R[(b,r),e] B[(c,d),e].
template <typename T, bool BF = false>
__device__ void s1_hole_mm(const T* Lp, const T* U, int ua, int ub, int Dl, int Dr, int Du,
                           int Dd, const T* Rn, const T* Bt, int ba, int bb, T* X1, T* X2,
                           T* Env) {
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(Dl * ba, Du * ub, ua, Lp, IMap(1), IMap(Dl * ba), U, IMap(Du * ub),
                             IMap(1), X1, IMap(Du * ub), IMap(1), false, false);
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ub * Dr, ba * Dd, bb, Rn, IMap(bb), IMap(1), Bt, IMap(1), IMap(bb),
                             X2, IMap(ba * Dd), IMap(1), false, false);
  __syncthreads();
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(Dl * Du, Dr * Dd, ba * ub, X1, IMap(Du, ba * Du * ub, ub),
                             IMap(ub, Du * ub, 1), X2, IMap(ub, Dd, Dr * ba * Dd),
                             IMap(Dd, ba * Dd, 1), Env, IMap(Du, Dr * Du * Dd, Dd),
                             IMap(Dd, Du * Dd, 1), false, false);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Two-row steps on the matrix cores for the large shapes (working sets in a
// global slab): each step is four products over the whole outer bond, the
// intermediates X1 and X2 (B^2 D^3 elements each) in the slab, X3 reusing
// X1. Same contractions and output layouts as s2_step_left / s2_step_right.
// ---------------------------------------------------------------------------
template <typename T, bool BF = false>
__device__ __forceinline__ void s2_step_left_mm(const T* Lp, const T* U, int ua, int uk, int ub, const T* A1,
                                int Dl1, int Dr1, int Dd1, const T* A2, int Dl2, int Dr2,
                                int Dd2, const T* Bt, int ba, int bb, T* X1, T* X2, T* Lout,
                                T* xl = nullptr, int xcap = 0) {
  const int inner = Dl1 * Dl2 * ba;
  const int q1 = Dl1 * uk * ub;
  if (xl != nullptr && xcap >= q1) {
    // with an LDS buffer, X1 goes chunk by chunk over q = (m2,c) and stays on
    // chip: xl[(m1,qq),(u,b)] for q = q0 + qq, then the chunk's rows of X2
    const int gq = xcap / q1, nq = Dl2 * ba;
    for (int q0 = 0; q0 < nq; q0 += gq) {
      const int g = nq - q0 < gq ? nq - q0 : gq;
      mgemm_map<T, false, false, BF, IsCplx<T>::value>(
          Dl1 * g, uk * ub, ua, Lp + q0, IMap(g, Dl2 * ba, 1), IMap(inner), U, IMap(uk * ub),
          IMap(1), xl, IMap(uk * ub), IMap(1), false, false);
      __syncthreads();
      mgemm_map<T, false, false, BF, IsCplx<T>::value>(
          g * ub, Dr1 * Dd1, Dl1 * uk, xl, IMap(ub, uk * ub, 1), IMap(uk, g * uk * ub, ub), A1,
          IMap(uk, Dr1 * uk * Dd1, Dd1), IMap(Dd1, uk * Dd1, 1),
          X2 + (size_t)q0 * ub * Dr1 * Dd1, IMap(Dr1 * Dd1), IMap(1), false, false);
      __syncthreads();
    }
  } else {
    // X1[(m1,m2,c),(u,b)] = sum_a L[a,(m1,m2,c)] U[a,(u,b)]
    mgemm_map<T, false, false, BF, IsCplx<T>::value>(inner, uk * ub, ua, Lp, IMap(1), IMap(inner), U,
                                                     IMap(uk * ub), IMap(1), X1, IMap(uk * ub),
                                                     IMap(1), false, false);
    __syncthreads();
    // X2[(m2,c,b),(r1,t)] = sum_{(m1,u)} X1[(m1,m2,c),(u,b)] A1[m1,r1,u,t]
    mgemm_map<T, false, false, BF, IsCplx<T>::value>(
        Dl2 * ba * ub, Dr1 * Dd1, Dl1 * uk, X1, IMap(ub, uk * ub, 1),
        IMap(uk, Dl2 * ba * uk * ub, ub), A1, IMap(uk, Dr1 * uk * Dd1, Dd1),
        IMap(Dd1, uk * Dd1, 1), X2, IMap(Dr1 * Dd1), IMap(1), false, false);
    __syncthreads();
  }
  // with an LDS buffer xl (xcap elements), X3 and L' go chunk by chunk over
  // the carried bond b, X3 of a chunk staying in LDS: X3[(c,bb,r1),(s,d)]
  // for b = b0 + bb, then the chunk's rows of L'
  const int per = ba * Dr1 * Dr2 * Dd2;
  if (xl != nullptr && xcap >= per) {
    const int gb = xcap / per;
    for (int b0 = 0; b0 < ub; b0 += gb) {
      const int g = ub - b0 < gb ? ub - b0 : gb;
      mgemm_map<T, false, false, BF, IsCplx<T>::value>(
          ba * g * Dr1, Dr2 * Dd2, Dl2 * Dd1, X2 + (size_t)b0 * Dr1 * Dd1,
          IMap(g * Dr1, ub * Dr1 * Dd1, Dd1), IMap(Dd1, ba * ub * Dr1 * Dd1, 1), A2,
          IMap(Dd1, Dr2 * Dd1 * Dd2, Dd2), IMap(Dd2, Dd1 * Dd2, 1), xl, IMap(Dr2 * Dd2), IMap(1),
          false, false);
      __syncthreads();
      mgemm_map<T, false, false, BF, IsCplx<T>::value>(
          g * Dr1 * Dr2, bb, ba * Dd2, xl, IMap(Dd2), IMap(Dd2, g * Dr1 * Dr2 * Dd2, 1), Bt,
          IMap(bb), IMap(1), Lout + (size_t)b0 * Dr1 * Dr2 * bb, IMap(bb), IMap(1), false, false);
      __syncthreads();
    }
    return;
  }
  // X3[(c,b,r1),(s,d)] = sum_{(m2,t)} X2[(m2,c,b),(r1,t)] A2[m2,s,t,d]  (into X1)
  T* X3 = X1;
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ba * ub * Dr1, Dr2 * Dd2, Dl2 * Dd1, X2, IMap(Dd1),
                             IMap(Dd1, ba * ub * Dr1 * Dd1, 1), A2, IMap(Dd1, Dr2 * Dd1 * Dd2, Dd2),
                             IMap(Dd2, Dd1 * Dd2, 1), X3, IMap(Dr2 * Dd2), IMap(1), false, false);
  __syncthreads();
  // L'[(b,r1,s),e] = sum_{(c,d)} X3[(c,b,r1),(s,d)] B[(c,d),e]
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ub * Dr1 * Dr2, bb, ba * Dd2, X3, IMap(Dd2),
                             IMap(Dd2, ub * Dr1 * Dr2 * Dd2, 1), Bt, IMap(bb), IMap(1), Lout,
                             IMap(bb), IMap(1), false, false);
  __syncthreads();
}

template <typename T, bool BF = false>
__device__ void s2_step_right_mm(const T* Rp, const T* U, int ua, int uk, int ub, const T* A1,
                                 int Dl1, int Dr1, int Dd1, const T* A2, int Dl2, int Dr2,
                                 int Dd2, const T* Bt, int ba, int bb, T* Y1, T* Y2, T* Rout,
                                 T* xl = nullptr, int xcap = 0) {
  const int rw = Dr1 * Dr2 * bb;
  if (xl != nullptr && xcap >= uk * rw) {
    // with an LDS buffer, Y1 goes chunk by chunk over a and stays on chip,
    // then the chunk's rows of Y2
    const int ga = xcap / (uk * rw);
    for (int a0 = 0; a0 < ua; a0 += ga) {
      const int g = ua - a0 < ga ? ua - a0 : ga;
      mgemm_map<T, false, false, BF, IsCplx<T>::value>(
          g * uk, rw, ub, U + (size_t)a0 * uk * ub, IMap(ub), IMap(1), Rp, IMap(rw), IMap(1), xl,
          IMap(rw), IMap(1), false, false);
      __syncthreads();
      mgemm_map<T, false, false, BF, IsCplx<T>::value>(
          g * Dr2 * bb, Dl1 * Dd1, uk * Dr1, xl, IMap(Dr2 * bb, uk * rw, 1),
          IMap(Dr1, rw, Dr2 * bb), A1, IMap(Dr1, Dd1, uk * Dd1), IMap(Dd1, Dr1 * uk * Dd1, 1),
          Y2 + (size_t)a0 * Dr2 * bb * Dl1 * Dd1, IMap(Dl1 * Dd1), IMap(1), false, false);
      __syncthreads();
    }
  } else {
    // Y1[(a,u),(r1,s,e)] = sum_b U[(a,u),b] R[b,(r1,s,e)]
    mgemm_map<T, false, false, BF, IsCplx<T>::value>(ua * uk, rw, ub, U, IMap(ub), IMap(1), Rp,
                                                     IMap(rw), IMap(1), Y1, IMap(rw), IMap(1),
                                                     false, false);
    __syncthreads();
    // Y2[(a,s,e),(m1,t)] = sum_{(u,r1)} Y1[(a,u),(r1,s,e)] A1[m1,r1,u,t]
    mgemm_map<T, false, false, BF, IsCplx<T>::value>(
        ua * Dr2 * bb, Dl1 * Dd1, uk * Dr1, Y1, IMap(Dr2 * bb, uk * rw, 1),
        IMap(Dr1, rw, Dr2 * bb), A1, IMap(Dr1, Dd1, uk * Dd1), IMap(Dd1, Dr1 * uk * Dd1, 1), Y2,
        IMap(Dl1 * Dd1), IMap(1), false, false);
    __syncthreads();
  }
  // with an LDS buffer xl (xcap elements), Y3 and R' go chunk by chunk over
  // the carried bond a, Y3 of a chunk staying in LDS
  const int per = bb * Dl1 * Dl2 * Dd2;
  if (xl != nullptr && xcap >= per) {
    const int ga = xcap / per;
    for (int a0 = 0; a0 < ua; a0 += ga) {
      const int g = ua - a0 < ga ? ua - a0 : ga;
      mgemm_map<T, false, false, BF, IsCplx<T>::value>(
          g * bb * Dl1, Dl2 * Dd2, Dr2 * Dd1, Y2 + (size_t)a0 * Dr2 * bb * Dl1 * Dd1,
          IMap(bb * Dl1, Dr2 * bb * Dl1 * Dd1, Dd1), IMap(Dd1, bb * Dl1 * Dd1, 1), A2, IMap(Dd2),
          IMap(Dd2, Dr2 * Dd1 * Dd2, 1), xl, IMap(Dl2 * Dd2), IMap(1), false, false);
      __syncthreads();
      mgemm_map<T, false, false, BF, IsCplx<T>::value>(
          g * Dl1 * Dl2, ba, Dd2 * bb, xl, IMap(Dl1 * Dl2, bb * Dl1 * Dl2 * Dd2, Dd2),
          IMap(bb, 1, Dl1 * Dl2 * Dd2), Bt, IMap(1), IMap(Dd2 * bb),
          Rout + (size_t)a0 * Dl1 * Dl2 * ba, IMap(ba), IMap(1), false, false);
      __syncthreads();
    }
    return;
  }
  // Y3[(a,e,m1),(m2,d)] = sum_{(s,t)} Y2[(a,s,e),(m1,t)] A2[m2,s,t,d]  (into Y1)
  T* Y3 = Y1;
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ua * bb * Dl1, Dl2 * Dd2, Dr2 * Dd1, Y2,
                             IMap(bb * Dl1, Dr2 * bb * Dl1 * Dd1, Dd1),
                             IMap(Dd1, bb * Dl1 * Dd1, 1), A2, IMap(Dd2),
                             IMap(Dd2, Dr2 * Dd1 * Dd2, 1), Y3, IMap(Dl2 * Dd2), IMap(1), false,
                             false);
  __syncthreads();
  // R'[(a,m1,m2),c] = sum_{(d,e)} Y3[(a,e,m1),(m2,d)] B[c,(d,e)]
  mgemm_map<T, false, false, BF, IsCplx<T>::value>(ua * Dl1 * Dl2, ba, Dd2 * bb, Y3,
                             IMap(Dl1 * Dl2, bb * Dl1 * Dl2 * Dd2, Dd2),
                             IMap(bb, 1, Dl1 * Dl2 * Dd2), Bt, IMap(1), IMap(Dd2 * bb), Rout,
                             IMap(ba), IMap(1), false, false);
  __syncthreads();
}

}  // namespace pm
