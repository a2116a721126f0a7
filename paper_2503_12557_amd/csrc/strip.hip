// Strips between cached environments (Sec. "On reusing environments"):
// local energies from amplitude ratios inside one-row and two-row strips,
// and log-derivatives from the one-row hole networks (Sec. "Finite PEPS and
// Sampling", Eq. tdvp).
//
// One workgroup owns one (sample, strip). It first builds every right
// partial contraction of the strip (kept in global scratch, read back once),
// then walks the strip left to right carrying the left partial in LDS. At
// each column it evaluates the hole tensor (one-row strips: O for that site),
// the amplitude ratio of every move whose window starts there, and extends
// the left partial. Ratios are numerator / denominator of the same strip
// (Sec. "On Numerical Stability" notes ratios are what matters).
#include "common.h"
#include "kernels.h"
#include "strip_dev.h"

namespace pm {

// working set of a one-row strip workgroup: partials and intermediates
// ("big": LDS, or a global slab for large shapes) and the hole tensor plus
// reduction scratch ("small": LDS)
static size_t strip1_big(int bmax, int D) {
  const size_t BD = (size_t)bmax * D;
  return 3 * (size_t)bmax * D * bmax + 2 * BD * BD;
}
static size_t strip1_small(int D) { return (size_t)D * D * D * D + 16; }
size_t strip1_lds_elems(int bmax, int D) { return strip1_big(bmax, D) + strip1_small(D); }

// Global-slab shapes in the FP32 modes trade registers for occupancy (the
// steps are bound by operand latency): one-row strips in workgroups of 256
// threads at most 168 VGPRs (three to a CU), two-row strips in 512 threads
// at most 128 VGPRs (two to a CU); measured best of the two forms for each.
#define STRIP_SMALL(M, GM) ((GM) && ((M) == MODE_F32 || (M) == MODE_BF16 || (M) == MODE_C64))
#define STRIP1_THREADS(M, GM) (STRIP_SMALL(M, GM) ? 256 : PEPS_BLOCK_MAX)
#define STRIP1_WAVES(M, GM) (STRIP_SMALL(M, GM) ? 3 : 1)
#define STRIP2_WAVES(M, GM) (STRIP_SMALL(M, GM) ? 4 : 1)

template <int M, bool GM>
__global__ void __launch_bounds__(STRIP1_THREADS(M, GM), STRIP1_WAVES(M, GM))
k_strip1(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
         const uint8_t* __restrict__ samples, const typename ModeT<M>::T* __restrict__ env,
         HamDev H, typename ModeT<M>::T* __restrict__ rtscr, double* __restrict__ epart,
         typename ModeT<M>::T* __restrict__ Oout, int* __restrict__ flags, int n, int want_e,
         int want_o, typename ModeT<M>::T* __restrict__ gws, size_t slab) {
  typedef typename ModeT<M>::T T;
  // matrix-core steps for the global-slab shapes (bfloat16 products in BF16
  // mode)
  constexpr bool MMP = GM;
  constexpr bool BFP = M == MODE_BF16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int smp = blockIdx.x, x = blockIdx.y;
  if (smp >= n) return;
  const int tid = threadIdx.x;
  const int B = L.bmax, D = L.D, BD = B * D;
  const int box = B * D * B;
  T* sm = GM ? gws + ((size_t)smp * gridDim.y + x) * slab : lds;
  T* Lf = sm;
  T* Lt = Lf + box;
  T* Lt2 = Lt + box;
  T* X1 = Lt2 + box;
  T* X2 = X1 + BD * BD;
  T* Env = GM ? lds : X2 + BD * BD;
  T* red = Env + D * D * D * D;
  __shared__ T one[1];
  __shared__ int fl;
  if (tid == 0) {
    one[0] = T(1);
    fl = 0;
  }
  const uint8_t* s = samples + (size_t)smp * L.N;
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  const T* envs = env + (size_t)smp * L.n_slots * slot_elems;
  T* Rt = rtscr + ((size_t)smp * L.Lx + x) * (size_t)(L.Ly + 1) * box;
  const int* ed = tab + L.off_env;
  const bool has_up = x > 0, has_dn = x < L.Lx - 1;
  const int su = has_up ? slot_top(L, x - 1) : -1;
  const int sd = has_dn ? slot_bottom(L, x + 1) : -1;
  __syncthreads();

  auto upT = [&](int y) -> const T* { return has_up ? env_site(envs, L, su, y) : one; };
  auto dnT = [&](int y) -> const T* { return has_dn ? env_site(envs, L, sd, y) : one; };
  auto ua_ = [&](int y) { return has_up ? ed[(su * L.Ly + y) * 3 + 0] : 1; };
  auto ub_ = [&](int y) { return has_up ? ed[(su * L.Ly + y) * 3 + 2] : 1; };
  auto ba_ = [&](int y) { return has_dn ? ed[(sd * L.Ly + y) * 3 + 0] : 1; };
  auto bb_ = [&](int y) { return has_dn ? ed[(sd * L.Ly + y) * 3 + 2] : 1; };

  // right partials Rt[y] (y = Ly .. 0), Rt[y] has dims (ua(y), Dl(y), ba(y)),
  // each brought to unit scale by a power of two 2^dex[y]; the left steps
  // take out the same powers column by column, so every ratio and hole
  // tensor sees one common scale and nothing leaves the FP32 range
  __shared__ int dex[32];
  T* RtL = Rt + (size_t)L.Ly * box;
  if (tid == 0) RtL[0] = T(1);
  __syncthreads();
  for (int y = L.Ly - 1; y >= 0; --y) {
    const int ns = x * L.Ly + y;
    int Dl, Dr, Du, Dd;
    legs_of(tab, L, ns, Dl, Dr, Du, Dd);
    const T* A = tensor_of(theta, tab, L, ns, pbit(s[ns]));
    T* Ry = Rt + (size_t)y * box;
    if constexpr (MMP)
      s1_step_right_mm<T, BFP>(Rt + (size_t)(y + 1) * box, upT(y), ua_(y), ub_(y), A, Dl, Dr, Du, Dd,
                       dnT(y), ba_(y), bb_(y), X1, X2, Ry);
    else
      s1_step_right<M>(Rt + (size_t)(y + 1) * box, upT(y), ua_(y), ub_(y), A, Dl, Dr, Du, Dd,
                       dnT(y), ba_(y), bb_(y), X1, X2, Ry);
    const int cnt = ua_(y) * Dl * ba_(y);
    const int e = pow2_exponent((double)block_absmax(Ry, 1, cnt, cnt, red));
    scale_pow2(Ry, cnt, e);
    if (tid == 0) dex[y] = e;
    __syncthreads();
  }
  const T psi_row = Rt[0];
  if (tid == 0 && (psi_row == T(0) || !finitex(psi_row))) fl |= (psi_row == T(0)) ? 1 : 2;

  // moves of this strip
  const int m0 = H.n_strips ? H.mstart[x] : 0;
  const int m1 = H.n_strips ? H.mstart[x + 1] : 0;
  int mi = m0;
  double ere = 0.0, eim = 0.0;
  // numerators summed per window end y1; each is divided by the strip value
  // taken along the same left-partial path, <L_y1, R_y1+1>, so the two
  // carry the same rounding
  __shared__ double nre[32], nim[32], zre[32], zim[32];
  if (tid < 32) {
    nre[tid] = 0.0;
    nim[tid] = 0.0;
    zre[tid] = 1.0;
    zim[tid] = 0.0;
  }
  if (tid == 0) Lf[0] = T(1);
  __syncthreads();
  for (int y = 0; y < L.Ly; ++y) {
    const int ns = x * L.Ly + y;
    int Dl, Dr, Du, Dd;
    legs_of(tab, L, ns, Dl, Dr, Du, Dd);
    const int ua = ua_(y), ub = ub_(y), ba = ba_(y), bb = bb_(y);
    const T* U = upT(y);
    const T* Bt = dnT(y);
    const T* A = tensor_of(theta, tab, L, ns, pbit(s[ns]));
    const T* Rn = Rt + (size_t)(y + 1) * box;
    const int nA = Dl * Dr * Du * Dd;
    if (want_o) {
      if constexpr (MMP) {
        s1_hole_mm<T, BFP>(Lf, U, ua, ub, Dl, Dr, Du, Dd, Rn, Bt, ba, bb, X1, X2, Env);
      } else {
        // X1[(m,c),(u,b)] = sum_a L[a,(m,c)] U[a,(u,b)]
        gemm<M>(Dl * ba, Du * ub, ua, Lf, 1, Dl * ba, U, Du * ub, 1, X1, Du * ub, 1, false);
        // Q[(b,r),(c,d)] = sum_e R[(b,r),e] B[(c,d),e]
        gemm<M>(ub * Dr, ba * Dd, bb, Rn, bb, 1, Bt, 1, bb, X2, ba * Dd, 1, false);
        __syncthreads();
        // Env[m,r,u,d] = sum_{c,b} X1[m,c,u,b] Q[b,r,c,d]
        const FastDiv fDd(Dd), fDu(Du), fDr(Dr);
        for (int i = tid; i < nA; i += PEPS_NT) {
          int t = i;
          const int d = divmod(t, fDd);
          const int u = divmod(t, fDu);
          const int r = divmod(t, fDr);
          const int m = t;
          T acc = 0;
          for (int c = 0; c < ba; ++c)
            for (int b = 0; b < ub; ++b)
              acc += opnd<M>(X1[((m * ba + c) * Du + u) * ub + b]) *
                     opnd<M>(X2[((b * Dr + r) * ba + c) * Dd + d]);
          Env[i] = acc;
        }
        __syncthreads();
      }
      const T psi_loc = lds_dot(Env, A, nA, red);
      T* o = Oout + (size_t)smp * L.n_compact + tab[L.off_compact + ns];
      const T inv = recipx(psi_loc);
      for (int i = tid; i < nA; i += PEPS_NT) o[i] = Env[i] * inv;
    }
    if (want_e) {
      while (mi < m1 && H.moves[8 * mi] == y) {
        const int* mv = H.moves + 8 * mi;
        double cre, cim;
        move_coef(H, mv, s, cre, cim);
        if (cre != 0.0 || cim != 0.0) {
          const int y1 = mv[1];
          // L_tmp = Lf, then step through the window with the moved tensors
          const T* cur = Lf;
          T* nxt = Lt;
          for (int yy = y; yy <= y1; ++yy) {
            const int n2 = x * L.Ly + yy;
            int dl, dr, du, dd;
            legs_of(tab, L, n2, dl, dr, du, dd);
            const int p = in_move(mv, n2) ? 1 - pbit(s[n2]) : pbit(s[n2]);
            if constexpr (MMP)
              s1_step_left_mm<T, BFP>(cur, upT(yy), ua_(yy), ub_(yy), tensor_of(theta, tab, L, n2, p),
                              dl, dr, du, dd, dnT(yy), ba_(yy), bb_(yy), X1, X2, nxt);
            else
              s1_step_left<M>(cur, upT(yy), ua_(yy), ub_(yy), tensor_of(theta, tab, L, n2, p),
                              dl, dr, du, dd, dnT(yy), ba_(yy), bb_(yy), X1, X2, nxt);
            scale_pow2(nxt, ub_(yy) * dr * bb_(yy), dex[yy]);
            __syncthreads();
            cur = nxt;
            nxt = (nxt == Lt) ? Lt2 : Lt;
          }
          const int cnt = ub_(y1) * tab[L.off_legs + 4 * (x * L.Ly + y1) + 1] * bb_(y1);
          const T num = lds_dot(cur, (const T*)(Rt + (size_t)(y1 + 1) * box), cnt, red);
          if (tid == 0) {
            const double nr = (double)realx(num), ni = (double)imagx(num);
            nre[y1] += cre * nr - cim * ni;
            nim[y1] += cre * ni + cim * nr;
          }
        }
        ++mi;
      }
    }
    // Lf <- step(Lf, A_y)
    if constexpr (MMP)
      s1_step_left_mm<T, BFP>(Lf, U, ua, ub, A, Dl, Dr, Du, Dd, Bt, ba, bb, X1, X2, Lt);
    else
      s1_step_left<M>(Lf, U, ua, ub, A, Dl, Dr, Du, Dd, Bt, ba, bb, X1, X2, Lt);
    {
      typedef typename RealOf<T>::type R;
      const R f = (R)ldexp(1.0, -dex[y]);
      for (int i = tid; i < ub * Dr * bb; i += PEPS_NT) Lf[i] = Lt[i] * f;
    }
    __syncthreads();
    if (want_e) {
      const T z = lds_dot(Lf, (const T*)Rn, ub * Dr * bb, red);
      if (tid == 0) {
        zre[y] = (double)realx(z);
        zim[y] = (double)imagx(z);
      }
    }
  }
  if (tid == 0) {
    if (want_e) {
      for (int y = 0; y < L.Ly; ++y)
        if (nre[y] != 0.0 || nim[y] != 0.0) {
          double qr, qi;
          cdiv(nre[y], nim[y], zre[y], zim[y], qr, qi);
          ere += qr;
          eim += qi;
        }
      const int nparts = 1 + L.Lx + (L.Lx - 1);
      epart[((size_t)smp * nparts + 1 + x) * 2] = ere;
      epart[((size_t)smp * nparts + 1 + x) * 2 + 1] = eim;
    }
    if (fl && flags) atomicOr(flags + smp, fl);
  }
}

// Lf | Lt | Lt2 (partials) | X1 = X3 | X2 (chunk intermediates) | Us | Bs
// (environments) | A1s | A2s (site tensors): every operand of a step is
// staged on chip, so its contractions read LDS only
// With the matrix-core steps (global working set, every mode; bfloat16
// products in BF16 mode) the intermediates hold the whole outer bond:
// B^2 D^3 each; in the FP32 modes the first and last of them are formed
// and consumed in LDS chunks instead (strip2_xcap), the slab keeping X2.
__host__ __device__ inline bool strip2_mm(int mode, bool gm) { return gm; }
__host__ __device__ inline size_t strip2_xsz(int bmax, int D, bool mm) {
  return mm ? (size_t)bmax * bmax * D * D * D : (size_t)S2G * bmax * D * D * D;
}
static size_t strip2_big(int bmax, int D, bool mm = false) {
  const size_t B2D2 = (size_t)bmax * bmax * D * D;
  const size_t box = (size_t)bmax * D * bmax;
  return 3 * B2D2 + 2 * strip2_xsz(bmax, D, mm) + 2 * box + 2 * (size_t)D * D * D * D;
}
size_t strip2_lds_elems(int bmax, int D) { return strip2_big(bmax, D) + 16; }

template <int M, bool GM>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX, STRIP2_WAVES(M, GM))
k_strip2(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
         const uint8_t* __restrict__ samples, const typename ModeT<M>::T* __restrict__ env,
         HamDev H, typename ModeT<M>::T* __restrict__ rtscr, double* __restrict__ epart,
         int* __restrict__ flags, int n, typename ModeT<M>::T* __restrict__ gws, size_t slab,
         int xcap) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int smp = blockIdx.x, x = blockIdx.y;
  if (smp >= n) return;
  const int tid = threadIdx.x;
  const int B = L.bmax, D = L.D;
  const int box2 = B * B * D * D;
  const int bd3 = B * D * D * D;
  const int box = B * D * B;
  T* sm = GM ? gws + ((size_t)smp * gridDim.y + x) * slab : lds;
  T* Lf = sm;
  T* Lt = Lf + box2;
  T* Lt2 = Lt + box2;
  // X3 of a chunk is formed after X1 is consumed and takes its place
  constexpr bool MMP = GM;
  constexpr bool BFP = M == MODE_BF16;
  const size_t xsz = strip2_xsz(B, D, MMP);
  T* X1 = Lt2 + box2;
  T* X2 = X1 + xsz;
  T* Us = X2 + xsz;
  T* Bs = Us + box;
  T* A1s = Bs + box;
  T* A2s = A1s + D * D * D * D;
  T* red = GM ? lds : A2s + D * D * D * D;
  // with the global slab, the last intermediate of each step (xcap elements
  // of LDS after the reduction scratch) is formed and consumed on chip
  T* xl = GM ? lds + 16 : nullptr;
  __shared__ T one[1];
  __shared__ int fl;
  if (tid == 0) {
    one[0] = T(1);
    fl = 0;
  }
  const int strip = L.Lx + x;
  const int m0 = H.mstart[strip], m1 = H.mstart[strip + 1];
  const int nparts = 1 + L.Lx + (L.Lx - 1);
  if (m0 == m1) {
    if (tid == 0) {
      epart[((size_t)smp * nparts + strip + 1) * 2] = 0.0;
      epart[((size_t)smp * nparts + strip + 1) * 2 + 1] = 0.0;
    }
    return;
  }
  const uint8_t* s = samples + (size_t)smp * L.N;
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  const T* envs = env + (size_t)smp * L.n_slots * slot_elems;
  T* Rt = rtscr + ((size_t)smp * (L.Lx - 1) + x) * (size_t)(L.Ly + 1) * box2;
  const int* ed = tab + L.off_env;
  const bool has_up = x > 0, has_dn = x + 1 < L.Lx - 1;
  const int su = has_up ? slot_top(L, x - 1) : -1;
  const int sd = has_dn ? slot_bottom(L, x + 2) : -1;
  __syncthreads();
  auto upT = [&](int y) -> const T* { return has_up ? env_site(envs, L, su, y) : one; };
  auto dnT = [&](int y) -> const T* { return has_dn ? env_site(envs, L, sd, y) : one; };
  auto ua_ = [&](int y) { return has_up ? ed[(su * L.Ly + y) * 3 + 0] : 1; };
  auto uk_ = [&](int y) { return has_up ? ed[(su * L.Ly + y) * 3 + 1] : 1; };
  auto ub_ = [&](int y) { return has_up ? ed[(su * L.Ly + y) * 3 + 2] : 1; };
  auto ba_ = [&](int y) { return has_dn ? ed[(sd * L.Ly + y) * 3 + 0] : 1; };
  auto bb_ = [&](int y) { return has_dn ? ed[(sd * L.Ly + y) * 3 + 2] : 1; };
  // the operands of the step at column y (site tensors with physical
  // indices p1, p2) to Us, Bs, A1s, A2s
  auto stage = [&](int y, int p1, int p2) {
    const int a1 = x * L.Ly + y, a2 = a1 + L.Ly;
    const T* u = upT(y);
    const T* bt = dnT(y);
    const T* t1 = tensor_of(theta, tab, L, a1, p1);
    const T* t2 = tensor_of(theta, tab, L, a2, p2);
    const int nu = ua_(y) * uk_(y) * ub_(y);
    const int nb = ba_(y) * tab[L.off_legs + 4 * a2 + 3] * bb_(y);
    const int n1 = tab[L.off_block + a1], n2 = tab[L.off_block + a2];
    for (int i = tid; i < nu; i += PEPS_NT) Us[i] = u[i];
    for (int i = tid; i < nb; i += PEPS_NT) Bs[i] = bt[i];
    for (int i = tid; i < n1; i += PEPS_NT) A1s[i] = t1[i];
    for (int i = tid; i < n2; i += PEPS_NT) A2s[i] = t2[i];
    __syncthreads();
  };

  // right partials at unit scale, powers of two in dex[y] (as in k_strip1);
  // the running partial stays in LDS (Lt / Lt2) and each one is also kept
  // in global scratch for the ratio windows
  __shared__ int dex[32];
  T* RtL = Rt + (size_t)L.Ly * box2;
  if (tid == 0) {
    RtL[0] = T(1);
    Lt[0] = T(1);
  }
  __syncthreads();
  T* rcur = Lt;
  T* rnxt = Lt2;
  for (int y = L.Ly - 1; y >= 0; --y) {
    const int n1 = x * L.Ly + y, n2 = n1 + L.Ly;
    int Dl1, Dr1, Du1, Dd1, Dl2, Dr2, Du2, Dd2;
    legs_of(tab, L, n1, Dl1, Dr1, Du1, Dd1);
    legs_of(tab, L, n2, Dl2, Dr2, Du2, Dd2);
    stage(y, pbit(s[n1]), pbit(s[n2]));
    if constexpr (MMP)
      s2_step_right_mm<T, BFP>(rcur, Us, ua_(y), uk_(y), ub_(y), A1s, Dl1, Dr1, Dd1, A2s, Dl2, Dr2,
                          Dd2, Bs, ba_(y), bb_(y), X1, X2, rnxt, xl, xcap);
    else
      s2_step_right<M>(rcur, Us, ua_(y), uk_(y), ub_(y), A1s, Dl1, Dr1, Dd1, A2s, Dl2, Dr2, Dd2,
                       Bs, ba_(y), bb_(y), X1, X2, X1, rnxt);
    const int cnt = ua_(y) * Dl1 * Dl2 * ba_(y);
    const int e = pow2_exponent((double)block_absmax(rnxt, 1, cnt, cnt, red));
    scale_pow2(rnxt, cnt, e);
    if (tid == 0) dex[y] = e;
    __syncthreads();
    T* Ry = Rt + (size_t)y * box2;
    for (int i = tid; i < cnt; i += PEPS_NT) Ry[i] = rnxt[i];
    T* tmp = rcur;
    rcur = rnxt;
    rnxt = tmp;
  }
  const T psi2 = rcur[0];
  if (tid == 0 && (psi2 == T(0) || !finitex(psi2))) fl |= (psi2 == T(0)) ? 1 : 2;

  int mi = m0;
  double ere = 0.0, eim = 0.0;
  __shared__ double nre[32], nim[32], zre[32], zim[32];
  if (tid < 32) {
    nre[tid] = 0.0;
    nim[tid] = 0.0;
    zre[tid] = 1.0;
    zim[tid] = 0.0;
  }
  int yneed = -1;
  if (tid == 0) Lf[0] = T(1);
  __syncthreads();
  for (int y = 0; y < L.Ly; ++y) {
    if (mi >= m1 && y > yneed) break;
    while (mi < m1 && H.moves[8 * mi] == y) {
      const int* mv = H.moves + 8 * mi;
      double cre, cim;
      move_coef(H, mv, s, cre, cim);
      if (cre != 0.0 || cim != 0.0) {
        const int y1 = mv[1];
        const T* cur = Lf;
        T* nxt = Lt;
        for (int yy = y; yy <= y1; ++yy) {
          const int a1 = x * L.Ly + yy, a2 = a1 + L.Ly;
          int Dl1, Dr1, Du1, Dd1, Dl2, Dr2, Du2, Dd2;
          legs_of(tab, L, a1, Dl1, Dr1, Du1, Dd1);
          legs_of(tab, L, a2, Dl2, Dr2, Du2, Dd2);
          const int p1 = in_move(mv, a1) ? 1 - pbit(s[a1]) : pbit(s[a1]);
          const int p2 = in_move(mv, a2) ? 1 - pbit(s[a2]) : pbit(s[a2]);
          stage(yy, p1, p2);
          if constexpr (MMP)
            s2_step_left_mm<T, BFP>(cur, Us, ua_(yy), uk_(yy), ub_(yy), A1s, Dl1, Dr1, Dd1, A2s, Dl2,
                               Dr2, Dd2, Bs, ba_(yy), bb_(yy), X1, X2, nxt, xl, xcap);
          else
            s2_step_left<M>(cur, Us, ua_(yy), uk_(yy), ub_(yy), A1s, Dl1, Dr1, Dd1, A2s, Dl2,
                            Dr2, Dd2, Bs, ba_(yy), bb_(yy), X1, X2, X1, nxt);
          scale_pow2(nxt, ub_(yy) * Dr1 * Dr2 * bb_(yy), dex[yy]);
          __syncthreads();
          cur = nxt;
          nxt = (nxt == Lt) ? Lt2 : Lt;
        }
        const int a1 = x * L.Ly + y1;
        const int cnt = ub_(y1) * tab[L.off_legs + 4 * a1 + 1] *
                        tab[L.off_legs + 4 * (a1 + L.Ly) + 1] * bb_(y1);
        const T num = lds_dot(cur, (const T*)(Rt + (size_t)(y1 + 1) * box2), cnt, red);
        if (tid == 0) {
          const double nr = (double)realx(num), ni = (double)imagx(num);
          nre[y1] += cre * nr - cim * ni;
          nim[y1] += cre * ni + cim * nr;
        }
        yneed = y1 > yneed ? y1 : yneed;
      }
      ++mi;
    }
    const int n1 = x * L.Ly + y, n2 = n1 + L.Ly;
    int Dl1, Dr1, Du1, Dd1, Dl2, Dr2, Du2, Dd2;
    legs_of(tab, L, n1, Dl1, Dr1, Du1, Dd1);
    legs_of(tab, L, n2, Dl2, Dr2, Du2, Dd2);
    stage(y, pbit(s[n1]), pbit(s[n2]));
    if constexpr (MMP)
      s2_step_left_mm<T, BFP>(Lf, Us, ua_(y), uk_(y), ub_(y), A1s, Dl1, Dr1, Dd1, A2s, Dl2, Dr2, Dd2,
                         Bs, ba_(y), bb_(y), X1, X2, Lt, xl, xcap);
    else
      s2_step_left<M>(Lf, Us, ua_(y), uk_(y), ub_(y), A1s, Dl1, Dr1, Dd1, A2s, Dl2, Dr2, Dd2, Bs,
                      ba_(y), bb_(y), X1, X2, X1, Lt);
    const int cnt = ub_(y) * Dr1 * Dr2 * bb_(y);
    {
      typedef typename RealOf<T>::type R;
      const R f = (R)ldexp(1.0, -dex[y]);
      for (int i = tid; i < cnt; i += PEPS_NT) Lf[i] = Lt[i] * f;
    }
    __syncthreads();
    const T z = lds_dot(Lf, (const T*)(Rt + (size_t)(y + 1) * box2), cnt, red);
    if (tid == 0) {
      zre[y] = (double)realx(z);
      zim[y] = (double)imagx(z);
    }
  }
  if (tid == 0) {
    for (int y = 0; y < L.Ly; ++y)
      if (nre[y] != 0.0 || nim[y] != 0.0) {
        double qr, qi;
        cdiv(nre[y], nim[y], zre[y], zim[y], qr, qi);
        ere += qr;
        eim += qi;
      }
    epart[((size_t)smp * nparts + strip + 1) * 2] = ere;
    epart[((size_t)smp * nparts + strip + 1) * 2 + 1] = eim;
    if (fl && flags) atomicOr(flags + smp, fl);
  }
}

// Diagonal part of E_loc plus the sum of the strip parts, one block per sample.
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_energy_diag_sum(Lattice L, HamDev H, const uint8_t* __restrict__ samples,
                  const double* __restrict__ epart, int nparts, double* __restrict__ eloc, int n) {
  __shared__ double red[8];
  const int smp = blockIdx.x;
  if (smp >= n) return;
  const uint8_t* s = samples + (size_t)smp * L.N;
  double re = 0.0, im = 0.0;
  for (int t = threadIdx.x; t < H.n_terms; t += PEPS_NT) {
    const int* tt = H.terms + 4 * t;
    int c = 0;
    for (int j = 0; j < tt[0]; ++j) c = 2 * c + pbit(s[tt[1 + j]]);
    const double* h = H.mats + ((size_t)t * 64 + c * 8 + c) * 2;
    re += h[0];
    im += h[1];
  }
  for (int p = threadIdx.x; p < H.n_pairs; p += PEPS_NT) {
    const int i = H.pair_ij[2 * p], j = H.pair_ij[2 * p + 1];
    if (pbit(s[i]) && pbit(s[j])) re += H.pair_v[p];
  }
  if (H.onsite)
    for (int q = threadIdx.x; q < L.N; q += PEPS_NT) re += H.onsite[2 * q + pbit(s[q])];
  re = block_sum(re, red);
  im = block_sum(im, red);
  if (threadIdx.x == 0) {
    for (int k = 1; k < nparts; ++k) {
      re += epart[((size_t)smp * nparts + k) * 2];
      im += epart[((size_t)smp * nparts + k) * 2 + 1];
    }
    eloc[2 * smp] = re;
    eloc[2 * smp + 1] = im;
  }
}

// ---------------------------------------------------------------------------
// Strict local energy (Sec. "On Variational Upper Bound"): every amplitude
// of E_loc is the full contraction at the one cut i*. The neighbours
// S' = S with one move applied are listed per sample (moves whose summed
// coefficient <S|H|S'> vanishes are left out), evaluated as one amplitude
// batch, and combined as E_loc(S) = diag(S) + sum_S' coef * Psi(S')/Psi(S).
// One thread per sample: these kernels move O(moves * N) bytes per sample,
// negligible beside the contractions of the amplitudes.
// ---------------------------------------------------------------------------
__global__ void k_strict_count(Lattice L, HamDev H, int n_moves,
                               const uint8_t* __restrict__ samples, int n, int* __restrict__ cnt) {
  const int smp = blockIdx.x * blockDim.x + threadIdx.x;
  if (smp >= n) return;
  const uint8_t* s = samples + (size_t)smp * L.N;
  int k = 0;
  for (int mi = 0; mi < n_moves; ++mi) {
    double cre, cim;
    move_coef(H, H.moves + 8 * mi, s, cre, cim);
    k += (cre != 0.0 || cim != 0.0) ? 1 : 0;
  }
  cnt[smp] = k;
}

// off[i] = n + sum_{j<i} cnt[j] for i = 0..n: the neighbours of sample i sit
// at rows off[i]..off[i+1]-1 of the amplitude batch, after the n samples.
// One workgroup; every thread scans a contiguous slice.
#define STRICT_SCAN 256
__global__ void __launch_bounds__(STRICT_SCAN)
k_strict_offsets(const int* __restrict__ cnt, int n, int* __restrict__ off) {
  __shared__ int part[STRICT_SCAN];
  const int t = threadIdx.x;
  const int per = (n + STRICT_SCAN - 1) / STRICT_SCAN;
  const int b = min(n, t * per), e = min(n, b + per);
  int loc = 0;
  for (int i = b; i < e; ++i) loc += cnt[i];
  part[t] = loc;
  __syncthreads();
  if (t == 0) {
    int acc = n;
    for (int j = 0; j < STRICT_SCAN; ++j) {
      const int v = part[j];
      part[j] = acc;
      acc += v;
    }
    off[n] = acc;
  }
  __syncthreads();
  int acc = part[t];
  for (int i = b; i < e; ++i) {
    off[i] = acc;
    acc += cnt[i];
  }
}

// Rows 0..n-1 of the batch are the samples, then the listed neighbours with
// their coefficients (coef row j - n).
__global__ void k_strict_expand(Lattice L, HamDev H, int n_moves,
                                const uint8_t* __restrict__ samples, int n,
                                const int* __restrict__ off, uint8_t* __restrict__ batch,
                                double* __restrict__ coef) {
  const int smp = blockIdx.x * blockDim.x + threadIdx.x;
  if (smp >= n) return;
  const int N = L.N;
  const uint8_t* s = samples + (size_t)smp * N;
  uint8_t* self = batch + (size_t)smp * N;
  for (int q = 0; q < N; ++q) self[q] = s[q];
  int row = off[smp];
  for (int mi = 0; mi < n_moves; ++mi) {
    const int* mv = H.moves + 8 * mi;
    double cre, cim;
    move_coef(H, mv, s, cre, cim);
    if (cre == 0.0 && cim == 0.0) continue;
    uint8_t* o = batch + (size_t)row * N;
    for (int q = 0; q < N; ++q) o[q] = (uint8_t)pbit(s[q]);
    for (int j = 0; j < mv[2]; ++j) o[mv[3 + j]] ^= 1;
    coef[2 * (size_t)(row - n)] = cre;
    coef[2 * (size_t)(row - n) + 1] = cim;
    ++row;
  }
}

// eloc[i] += sum_j coef_j exp(ln Psi(S'_j) - ln Psi(S_i)); flags of the
// neighbours are ORed into the sample's.
__global__ void k_strict_combine(int n, const int* __restrict__ off,
                                 const double* __restrict__ coef, const double* __restrict__ lp,
                                 const int* __restrict__ bfl, double* __restrict__ eloc,
                                 int* __restrict__ flags) {
  const int smp = blockIdx.x * blockDim.x + threadIdx.x;
  if (smp >= n) return;
  const double l0 = lp[2 * smp], a0 = lp[2 * smp + 1];
  double re = 0.0, im = 0.0;
  int f = bfl[smp];
  for (int j = off[smp]; j < off[smp + 1]; ++j) {
    const double w = exp(lp[2 * (size_t)j] - l0);
    const double ph = lp[2 * (size_t)j + 1] - a0;
    const double xr = w * cos(ph), xi = w * sin(ph);
    const double cr = coef[2 * (size_t)(j - n)], ci = coef[2 * (size_t)(j - n) + 1];
    re += cr * xr - ci * xi;
    im += cr * xi + ci * xr;
    f |= bfl[j];
  }
  eloc[2 * smp] += re;
  eloc[2 * smp + 1] += im;
  if (flags) flags[smp] = f;
}

hipError_t launch_strict_count(const Lattice& L, const HamDev& H, int n_moves,
                               const uint8_t* samples, int n, int* cnt, int* off,
                               hipStream_t st) {
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_strict_count, dim3(nb), dim3(256), 0, st, L, H, n_moves, samples, n, cnt);
  hipLaunchKernelGGL(k_strict_offsets, dim3(1), dim3(STRICT_SCAN), 0, st, cnt, n, off);
  return hipGetLastError();
}

hipError_t launch_strict_expand(const Lattice& L, const HamDev& H, int n_moves,
                                const uint8_t* samples, int n, const int* off, uint8_t* batch,
                                double* coef, hipStream_t st) {
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_strict_expand, dim3(nb), dim3(256), 0, st, L, H, n_moves, samples, n, off,
                     batch, coef);
  return hipGetLastError();
}

hipError_t launch_strict_combine(int n, const int* off, const double* coef, const double* lp,
                                 const int* bfl, double* eloc, int* flags, hipStream_t st) {
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_strict_combine, dim3(nb), dim3(256), 0, st, n, off, coef, lp, bfl, eloc,
                     flags);
  return hipGetLastError();
}

size_t strip1_lds_bytes(int mode, const Lattice& L, bool gm) {
  return (gm ? strip1_small(L.D) : strip1_lds_elems(L.bmax, L.D)) * mode_elem_bytes(mode);
}
// LDS for the on-chip chunks of the steps' last intermediate (global slab,
// FP32 modes, two workgroups to a CU): whole multiples of one carried-bond
// slice (bmax D^3 elements) within half of a CU's 160 KiB, zero when not
// even one slice fits. The FP64 modes keep the intermediate in the slab:
// their slices are twice as large, and chunks of one to three slices leave
// most waves of the last product idle (complex128 at 10x10 D=5 chi=25: 425
// against 407 ms per launch, where complex64 gains 222 -> 212 ms).
static int strip2_xcap(int mode, const Lattice& L) {
  if (mode != MODE_F32 && mode != MODE_BF16 && mode != MODE_C64) return 0;
  const size_t budget = 76 * 1024 / mode_elem_bytes(mode);
  const size_t per = (size_t)L.bmax * L.D * L.D * L.D;
  return (int)(budget / per * per);
}
size_t strip2_lds_bytes(int mode, const Lattice& L, bool gm) {
  return (gm ? 16 + (size_t)strip2_xcap(mode, L) : strip2_lds_elems(L.bmax, L.D)) *
         mode_elem_bytes(mode);
}
size_t strip1_slab_elems(const Lattice& L) { return (strip1_big(L.bmax, L.D) + 15) / 16 * 16; }
size_t strip2_slab_elems(const Lattice& L, int mode) {
  return (strip2_big(L.bmax, L.D, strip2_mm(mode, true)) + 15) / 16 * 16;
}

template <int M>
hipError_t launch_strip1(const Lattice& L, const int* tab, const void* theta,
                         const uint8_t* samples, const void* env, const HamDev& H, void* rt,
                         double* epart, void* O, int* flags, int n, bool want_e, bool want_o,
                         void* gws, hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const bool gm = gws != nullptr;
  const size_t lds = strip1_lds_bytes(M, L, gm);
  const void* fn = gm ? (const void*)k_strip1<M, true> : (const void*)k_strip1<M, false>;
  hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (gm)
    hipLaunchKernelGGL((k_strip1<M, true>), dim3(n, L.Lx), dim3(STRIP1_THREADS(M, true)), lds, st,
                       L, tab, (const T*)theta, samples, (const T*)env, H, (T*)rt, epart, (T*)O,
                       flags, n,
                       want_e ? 1 : 0, want_o ? 1 : 0, (T*)gws, strip1_slab_elems(L));
  else
    hipLaunchKernelGGL((k_strip1<M, false>), dim3(n, L.Lx), dim3(512), lds, st, L, tab,
                       (const T*)theta, samples, (const T*)env, H, (T*)rt, epart, (T*)O, flags, n,
                       want_e ? 1 : 0, want_o ? 1 : 0, (T*)nullptr, (size_t)0);
  return hipGetLastError();
}

template <int M>
hipError_t launch_strip2(const Lattice& L, const int* tab, const void* theta,
                         const uint8_t* samples, const void* env, const HamDev& H, void* rt,
                         double* epart, int* flags, int n, void* gws, hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const bool gm = gws != nullptr;
  const size_t lds = strip2_lds_bytes(M, L, gm);
  const void* fn = gm ? (const void*)k_strip2<M, true> : (const void*)k_strip2<M, false>;
  hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (gm)
    hipLaunchKernelGGL((k_strip2<M, true>), dim3(n, L.Lx - 1), dim3(512), lds, st, L, tab,
                       (const T*)theta, samples, (const T*)env, H, (T*)rt, epart, flags, n,
                       (T*)gws, strip2_slab_elems(L, M), strip2_xcap(M, L));
  else
    hipLaunchKernelGGL((k_strip2<M, false>), dim3(n, L.Lx - 1), dim3(512), lds, st, L, tab,
                       (const T*)theta, samples, (const T*)env, H, (T*)rt, epart, flags, n,
                       (T*)nullptr, (size_t)0, 0);
  return hipGetLastError();
}

hipError_t launch_energy_diag_sum(const Lattice& L, const HamDev& H, const uint8_t* samples,
                                  const double* epart, int nparts, double* eloc, int n,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_energy_diag_sum, dim3(n), dim3(256), 0, st, L, H, samples, epart,
                     nparts, eloc, n);
  return hipGetLastError();
}

#define INST(M)                                                                                 \
  template hipError_t launch_strip1<M>(const Lattice&, const int*, const void*, const uint8_t*, \
                                       const void*, const HamDev&, void*, double*, void*, int*, \
                                       int, bool, bool, void*, hipStream_t);                    \
  template hipError_t launch_strip2<M>(const Lattice&, const int*, const void*, const uint8_t*, \
                                       const void*, const HamDev&, void*, double*, int*, int,   \
                                       void*, hipStream_t);
INST(MODE_F64)
INST(MODE_F32)
INST(MODE_BF16)
INST(MODE_C128)
INST(MODE_C64)
#undef INST

}  // namespace pm
