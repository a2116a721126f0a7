// Device-side boundary-MPS building blocks shared by the environment
// kernel and the sampler: the first row read as an MPS and the absorption
// of one further row with its truncation back to chi (see env.hip).
#pragma once

#include "common.h"

namespace pm {

// A tensor of site (x, y) seen from a sweep direction: legs (l, r, in, out)
// where "in" faces the environment being absorbed and "out" is the new
// physical leg (top sweep: in = up, out = down; bottom sweep: swapped).
struct SiteView {
  int Dl, Dr, Din, Dout;
  int s_l, s_r, s_in, s_out;  // element strides in the (l, r, u, d) tensor
};

__device__ __forceinline__ SiteView site_view(const int* tab, const Lattice& L, int n, bool bottom) {
  const int* lg = tab + L.off_legs + 4 * n;
  SiteView v;
  v.Dl = lg[0];
  v.Dr = lg[1];
  const int Du = lg[2], Dd = lg[3];
  const int s_d = 1, s_u = Dd, s_r = Du * Dd, s_l = lg[1] * Du * Dd;
  v.s_l = s_l;
  v.s_r = s_r;
  if (!bottom) {
    v.Din = Du; v.Dout = Dd; v.s_in = s_u; v.s_out = s_d;
  } else {
    v.Din = Dd; v.Dout = Du; v.s_in = s_d; v.s_out = s_u;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ const T* site_tensor(const T* theta, const int* tab, const Lattice& L,
                                               const uint8_t* s, int n) {
  return theta + tab[L.off_param + n] + pbit(s[n]) * tab[L.off_block + n];
}

template <typename T>
__device__ void load_lds(T* dst, const T* src, int cnt) {
  for (int i = threadIdx.x; i < cnt; i += PEPS_NT) dst[i] = src[i];
}

// Divide the tensor by its largest modulus; returns ln(divisor).
template <typename T>
__device__ double normalize_lds(T* t, int cnt, T* red, int* flag) {
  typedef typename RealOf<T>::type R;
  R mx = 0;
  for (int i = threadIdx.x; i < cnt; i += PEPS_NT) {
    const R a = absx(t[i]);
    mx = a > mx ? a : mx;
  }
  mx = block_max(mx, reinterpret_cast<R*>(red));
  if (!(mx > R(0)) || !isfinite((double)mx)) {
    if (threadIdx.x == 0) *flag |= (mx == R(0)) ? 1 : 2;
    __syncthreads();
    return 0.0;
  }
  const R inv = R(1) / mx;
  for (int i = threadIdx.x; i < cnt; i += PEPS_NT) t[i] *= inv;
  __syncthreads();
  return log((double)mx);
}

// ---------------------------------------------------------------------------
// Left-sweep QR on registers for FP32 / BF16 with chi*D <= 64 and D <= 4
// (four waves). Wave k builds the block M_k = R_{y-1} P_k of the stack
// [M_0; ...; M_{D-1}] with lane c holding column c (64 rows) in registers;
// the four waves then run one Householder QR of the whole stack together,
// exchanging only partial dot products through LDS.
// ---------------------------------------------------------------------------
#define TQ_N 64
#define TQ_PACK (TQ_N * (TQ_N + 1) / 2)
// partial dot products of the four waves, double buffered
#define TQ_XCH (2 * 4 * TQ_N)
// column j of each wave's block, broadcast to the wave through LDS
#define TQ_VB (4 * TQ_N)

__host__ __device__ inline bool tsqr_path(int mode, int bmax, int D) {
  return (mode == MODE_F32 || mode == MODE_BF16) && bmax * D <= TQ_N && D <= 4;
}

// Working set of one environment workgroup, in elements: the matrices
// ("big": in LDS, or in a global slab when they do not fit on chip) and
// the vectors and reduction scratch ("small": always in LDS).
__host__ __device__ inline size_t env_big_elems(int bmax, int D, int mode) {
  const size_t BD = (size_t)bmax * D;
  const size_t head = (size_t)bmax * D * bmax + (size_t)D * D * D * D;
  size_t rest = BD * BD + 2 * BD * (BD + 4) + 2 * BD * bmax;
  if (tsqr_path(mode, bmax, D)) {
    // register-QR path (launched with 256 threads): the left sweep keeps
    // the packed factor, its exchange buffers and the dense previous R from
    // P on, and the right sweep's C overlays T1 (dead once Z is formed)
    const size_t tq = (size_t)TQ_PACK + TQ_XCH + TQ_VB + (size_t)TQ_N * TQ_N;
    rest = 2 * BD * (BD + 4) + 2 * BD * bmax;
    if (rest < tq) rest = tq;
  }
  return head + rest;
}
__host__ __device__ inline size_t env_small_elems(int bmax, int D) {
  return 4 * (size_t)bmax * D + 16;
}
__host__ __device__ inline size_t env_lds_elems_(int bmax, int D, int mode) {
  return env_big_elems(bmax, D, mode) + env_small_elems(bmax, D);
}

// start of row j in a packed upper-triangular TQ_N x TQ_N matrix (by rows)
__host__ __device__ __forceinline__ int prow(int j) { return j * TQ_N - (j * (j - 1)) / 2; }

// One site of the left sweep on the register path. Each wave k < Dout
// forms its block M_k = R_{y-1} P_k (R_{y-1}: Rpk, dense 64 x 64
// column-major, zero below the diagonal and outside kprev x Pl; P_k from E
// and A in LDS), then the stack is factorised by Householder QR of
// [0; stack]: reflector j maps (0, column j) to (sqrt(s), 0), s the squared
// norm of column j, so its vector is (-sqrt(s), column j) and tau = 1/s.
// Per column each wave forms the dot products of column j (broadcast from
// lane j through LDS) with all of its columns; the four partial sums meet in
// LDS (xch: TQ_XCH floats, then TQ_VB for the column copies) behind one
// barrier, and each wave updates its block. Row j of the factor is sqrt(s)
// times the dot products over s. On exit t (packed rows, LDS)
// holds R_y. Columns j >= min(Pr, kprev * Dout) hold only rounding residue
// and are not reflected, nor is a column whose squared norm is below the
// normal range (as in LAPACK's larfg).
template <int M>
__device__ void tsqr_site(const float* Ebuf, const float* Abuf, const float* Rpk, float* t,
                          float* xch, int kprev, int bl, int br, int Dl, int Dr, int Din,
                          int Dout, int s_l, int s_r, int s_in, int s_out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int Pl = bl * Dl, Pr = br * Dr;
  const bool blk = wv < Dout;
  for (int i = threadIdx.x; i < TQ_PACK; i += PEPS_NT) t[i] = 0.f;
  float u[TQ_N];
#pragma unroll
  for (int i = 0; i < TQ_N; ++i) u[i] = 0.f;
  if (blk) {
    // u = R_{y-1} P_k for column c = (b, r) of P_k, with
    // P_k[(a,l),(b,r)] = sum_in E[a,in,b] A[l,r,in,k] formed row by row
    const int c = lane;
    const bool colok = c < Pr;
    const int b = colok ? c / Dr : 0, r = colok ? c - (c / Dr) * Dr : 0;
    for (int l = 0; l < Pl; ++l) {
      float pl = 0.f;
      if (colok) {
        const int aa = l / Dl, li = l - (l / Dl) * Dl;
        for (int in = 0; in < Din; ++in)
          pl = fmaf(opnd<M>(Ebuf[(aa * Din + in) * br + b]),
                    opnd<M>(Abuf[li * s_l + r * s_r + in * s_in + wv * s_out]), pl);
      }
      pl = opnd<M>(pl);
      const float* col = Rpk + l * TQ_N;
      // R_{y-1} is upper triangular: column l has no entries below row l
#pragma unroll
      for (int q = 0; q < TQ_N; q += 16) {
        if (q <= l) {
#pragma unroll
          for (int i = q; i < q + 16; ++i) u[i] = fmaf(opnd<M>(col[i]), pl, u[i]);
        }
      }
    }
  }
  const int kmax = min(Pr, kprev * Dout);
  float* vbw = xch + TQ_XCH + wv * TQ_N;  // this wave's copy of column j
  const int k1 = kmax < TQ_N / 2 ? kmax : TQ_N / 2;
  for (int j = 0; j < k1; ++j) {
    float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
    if (blk) {
      // lane j publishes column j to its wave; every lane reads it back as
      // 16-byte broadcasts (LDS instructions rather than 64 VALU lane reads)
      if (lane == j) {
#pragma unroll
        for (int i = 0; i < TQ_N; i += 4)
          *reinterpret_cast<float4*>(vbw + i) = make_float4(u[i], u[i + 1], u[i + 2], u[i + 3]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int i = 0; i < TQ_N; i += 4) {
        const float4 v4 = *reinterpret_cast<const float4*>(vbw + i);
        d0 = fmaf(v4.x, u[i], d0);
        d1 = fmaf(v4.y, u[i + 1], d1);
        d2 = fmaf(v4.z, u[i + 2], d2);
        d3 = fmaf(v4.w, u[i + 3], d3);
      }
    }
    float* xb = xch + (j & 1) * (4 * TQ_N);
    xb[wv * TQ_N + lane] = (d0 + d1) + (d2 + d3);
    __syncthreads();
    // the same sums in every wave: s decides uniformly
    const float dc = (xb[lane] + xb[TQ_N + lane]) + (xb[2 * TQ_N + lane] + xb[3 * TQ_N + lane]);
    const float s = (xb[j] + xb[TQ_N + j]) + (xb[2 * TQ_N + j] + xb[3 * TQ_N + j]);
    if (!(s > 1e-36f)) continue;  // column j is already zero
    const float w = dc * (1.f / s);
    if (wv == 0 && lane >= j && lane < Pr) t[prow(j) - j + lane] = sqrtf(s) * w;
    if (blk) {
      // column j again from LDS rather than 64 values held across the barrier
#pragma unroll
      for (int i = 0; i < TQ_N; i += 4) {
        const float4 v4 = *reinterpret_cast<const float4*>(vbw + i);
        u[i] = fmaf(-v4.x, w, u[i]);
        u[i + 1] = fmaf(-v4.y, w, u[i + 1]);
        u[i + 2] = fmaf(-v4.z, w, u[i + 2]);
        u[i + 3] = fmaf(-v4.w, w, u[i + 3]);
      }
    }
  }
  if (kmax > TQ_N / 2) {
    // Columns 32..63: only they are left, so the wave takes them two lanes
    // per column: lane (c, h) holds rows 32h .. 32h+31 of column 32 + c,
    // and each reflector costs half the instructions; a column's dot
    // products add over the lane pair (lanes c and c + 32)
    constexpr int HN = TQ_N / 2;
    const int h = lane >> 5, cc = lane & (HN - 1), col = HN + cc;
    if (blk) {
#pragma unroll
      for (int i = 0; i < HN; ++i) {
        const float x = shfl_xor_x(u[i], HN);
        u[i] = h == 0 ? x : u[HN + i];
      }
    }
    float* vh = vbw + HN * h;
    for (int j = HN; j < kmax; ++j) {
      float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
      if (blk) {
        if (cc == j - HN) {
#pragma unroll
          for (int i = 0; i < HN; i += 4)
            *reinterpret_cast<float4*>(vh + i) = make_float4(u[i], u[i + 1], u[i + 2], u[i + 3]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int i = 0; i < HN; i += 4) {
          const float4 v4 = *reinterpret_cast<const float4*>(vh + i);
          d0 = fmaf(v4.x, u[i], d0);
          d1 = fmaf(v4.y, u[i + 1], d1);
          d2 = fmaf(v4.z, u[i + 2], d2);
          d3 = fmaf(v4.w, u[i + 3], d3);
        }
      }
      float dh = (d0 + d1) + (d2 + d3);
      dh += shfl_xor_x(dh, HN);
      float* xb = xch + (j & 1) * (4 * TQ_N);
      if (h == 0) xb[wv * TQ_N + col] = dh;
      __syncthreads();
      const float dc = (xb[col] + xb[TQ_N + col]) + (xb[2 * TQ_N + col] + xb[3 * TQ_N + col]);
      const float s = (xb[j] + xb[TQ_N + j]) + (xb[2 * TQ_N + j] + xb[3 * TQ_N + j]);
      if (!(s > 1e-36f)) continue;  // column j is already zero
      const float w = dc * (1.f / s);
      if (wv == 0 && h == 0 && col >= j && col < Pr) t[prow(j) - j + col] = sqrtf(s) * w;
      if (blk) {
#pragma unroll
        for (int i = 0; i < HN; i += 4) {
          const float4 v4 = *reinterpret_cast<const float4*>(vh + i);
          u[i] = fmaf(-v4.x, w, u[i]);
          u[i + 1] = fmaf(-v4.y, w, u[i + 1]);
          u[i + 2] = fmaf(-v4.z, w, u[i + 2]);
          u[i + 3] = fmaf(-v4.w, w, u[i + 3]);
        }
      }
    }
  }
  __syncthreads();
}

// Carve-up of the working set.
template <typename T>
struct EnvSmem {
  T *Ebuf, *Abuf, *P, *S, *Z, *W, *Bn, *vv, *ww, *sig, *red;
  // overlay: the register-QR path, whose left sweep needs no S, so the
  // right sweep's C can take T1's place
  __device__ EnvSmem(T* big, T* small, const Lattice& L, bool overlay) {
    const int B = L.bmax, D = L.D, BD = L.bmax * L.D;
    Ebuf = big;
    Abuf = Ebuf + B * D * B;
    P = Abuf + D * D * D * D;   // P_k (left) / T1 (right)
    // stacked QR buffer (left) / C then Z (right); rows padded so rows of
    // the LDS matrices fall on different banks
    S = overlay ? P : P + BD * BD;
    Z = S + BD * (BD + 4);
    W = S + 2 * BD * (BD + 4);
    Bn = W + BD * B;
    vv = small;
    ww = vv + 2 * BD;
    sig = ww + BD;
    red = sig + BD;
  }
};

// The first row of a sweep read as an MPS, normalised, into its slot.
template <int M>
__device__ void env_first_row(const Lattice& L, const int* tab, const typename ModeT<M>::T* theta,
                              const uint8_t* s, bool bottom, typename ModeT<M>::T* envs,
                              double* lg, const EnvSmem<typename ModeT<M>::T>& sh, int* flp) {
  typedef typename ModeT<M>::T T;
  const int tid = threadIdx.x;
  T* Ebuf = sh.Ebuf;
  T* red = sh.red;
  int& fl = *flp;
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  // ---- first row read as an MPS ----
  const int x0 = bottom ? L.Lx - 1 : 0;
  const int slot0 = bottom ? slot_bottom(L, L.Lx - 1) : slot_top(L, 0);
  double logacc = 0.0;
  for (int y = 0; y < L.Ly; ++y) {
    const int nsite = x0 * L.Ly + y;
    const SiteView v = site_view(tab, L, nsite, bottom);
    const T* a = site_tensor(theta, tab, L, s, nsite);
    const int cnt = v.Dl * v.Dout * v.Dr;
    for (int i = tid; i < cnt; i += PEPS_NT) {
      const int l = i / (v.Dout * v.Dr), rem = i - l * (v.Dout * v.Dr);
      const int k = rem / v.Dr, r = rem - k * v.Dr;
      Ebuf[i] = a[l * v.s_l + r * v.s_r + k * v.s_out];
    }
    __syncthreads();
    logacc += normalize_lds(Ebuf, cnt, red, flp);
    T* dst = envs + (size_t)slot0 * slot_elems + (size_t)y * L.site_box;
    for (int i = tid; i < cnt; i += PEPS_NT) dst[i] = Ebuf[i];
    __syncthreads();
  }
  if (tid == 0) lg[slot0] = logacc;

}

// Absorb row t of the sweep (x = t from the top, Lx-1-t from the bottom) into
// the previous environment and truncate to chi; R is this sweep's scratch
// for the Ly R factors.
template <int M>
__device__ void env_absorb_row(const Lattice& L, const int* tab, const typename ModeT<M>::T* theta,
                               const uint8_t* s, bool bottom, int t, typename ModeT<M>::T* envs,
                               double* lg, typename ModeT<M>::T* R,
                               const EnvSmem<typename ModeT<M>::T>& sh, int* sel, int* sflag,
                               int* flp, int jac_sweeps) {
  typedef typename ModeT<M>::T T;
  typedef typename RealOf<T>::type Rl;
  const int tid = threadIdx.x;
  const int B = L.bmax, D = L.D, BD = L.bmax * L.D;
  T *Ebuf = sh.Ebuf, *Abuf = sh.Abuf, *P = sh.P, *S = sh.S, *Z = sh.Z, *W = sh.W, *Bn = sh.Bn;
  T* red = sh.red;
  // row norms and scales of the Jacobi (2 BD reals)
  Rl* vv = reinterpret_cast<Rl*>(sh.vv);
  Rl* sig = reinterpret_cast<Rl*>(sh.sig);  // singular values
  Rl* rred = reinterpret_cast<Rl*>(sh.red);
  int& fl = *flp;
  (void)B;
  (void)D;
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  const int* edims = tab + L.off_env;
  const Rl tol = Eps<Rl>::v * Rl(4);
    const int x = bottom ? L.Lx - 1 - t : t;
    const int sp = bottom ? slot_bottom(L, x + 1) : slot_top(L, x - 1);
    const int sn = bottom ? slot_bottom(L, x) : slot_top(L, x);
    const T* Eprev = envs + (size_t)sp * slot_elems;
    T* Enew = envs + (size_t)sn * slot_elems;

    // left-to-right QR sweep: R_y of R_{y-1} P_y
    int kprev = 1;  // rows of R_{y-1}
    bool tree = false;
    if constexpr (M == MODE_F32 || M == MODE_BF16) {
      tree = tsqr_path(M, L.bmax, L.D) && PEPS_NT == 256;
      if (tree) {
        // R_{-1} = [1], dense column-major after the factor and exchange buffers
        float* Rpk = P + TQ_PACK + TQ_XCH + TQ_VB;
        for (int i = tid; i < TQ_N * TQ_N; i += PEPS_NT) Rpk[i] = i == 0 ? 1.f : 0.f;
      }
    }
    for (int y = 0; y < L.Ly - 1; ++y) {
      const int nsite = x * L.Ly + y;
      const SiteView v = site_view(tab, L, nsite, bottom);
      const int bl = edims[(sp * L.Ly + y) * 3 + 0];
      const int br = edims[(sp * L.Ly + y) * 3 + 2];
      const int Pl = bl * v.Dl, Pr = br * v.Dr;
      load_lds(Ebuf, Eprev + (size_t)y * L.site_box, bl * v.Din * br);
      const T* a = site_tensor(theta, tab, L, s, nsite);
      load_lds(Abuf, a, v.Dl * v.Dr * v.Din * v.Dout);
      __syncthreads();
      if constexpr (M == MODE_F32 || M == MODE_BF16) {
        if (tree) {
          float* Rpk = P + TQ_PACK + TQ_XCH + TQ_VB;
          tsqr_site<M>(Ebuf, Abuf, Rpk, P, P + TQ_PACK, kprev, bl, br, v.Dl, v.Dr, v.Din,
                       v.Dout, v.s_l, v.s_r, v.s_in, v.s_out);
          const int kr = min(kprev * v.Dout, Pr);
          // R_y at unit scale (see below) to global rows and to Rpk
          const float* t0 = P;
          Rl mx = 0;
          for (int i = tid; i < kr * Pr; i += PEPS_NT) {
            const int ii = i / Pr, cc = i - ii * Pr;
            if (cc >= ii) mx = fmaxf(mx, fabsf(t0[prow(ii) - ii + cc]));
          }
          mx = block_max(mx, rred);
          const Rl fr = (Rl)ldexp(1.0, -pow2_exponent((double)mx));
          T* Ry = R + (size_t)y * BD * BD;
          for (int i = tid; i < kr * Pr; i += PEPS_NT) {
            const int ii = i / Pr, cc = i - ii * Pr;
            Ry[i] = cc >= ii ? t0[prow(ii) - ii + cc] * fr : 0.f;
          }
          for (int i = tid; i < TQ_N * TQ_N; i += PEPS_NT) {
            const int cc = i / TQ_N, ii = i - cc * TQ_N;  // column-major
            Rpk[i] = (ii <= cc && ii < kr && cc < Pr) ? t0[prow(ii) - ii + cc] * fr : 0.f;
          }
          __syncthreads();
          kprev = kr;
          continue;
        }
      }
      const T* Rp = (y > 0) ? R + (size_t)(y - 1) * BD * BD : nullptr;
      int kr = 0;
      for (int k = 0; k < v.Dout; ++k) {
        // P_k[(a,l),(b,r)] = sum_in E[a,in,b] A[l,r,in,k]
        const int tot = Pl * Pr;
        const FastDiv fPr(Pr), fDl(v.Dl), fDr(v.Dr);
        for (int i = tid; i < tot; i += PEPS_NT) {
          int row = i;
          int col = divmod(row, fPr);
          const int l = divmod(row, fDl);
          const int aa = row;
          const int r = divmod(col, fDr);
          const int b = col;
          T acc = 0;
          for (int in = 0; in < v.Din; ++in)
            acc += opnd<M>(Ebuf[(aa * v.Din + in) * br + b]) *
                   opnd<M>(Abuf[l * v.s_l + r * v.s_r + in * v.s_in + k * v.s_out]);
          P[i] = acc;
        }
        __syncthreads();
        // M_k = R_{y-1} P_k into rows kr.. of the stack
        if (y == 0) {
          for (int i = tid; i < Pr; i += PEPS_NT) S[kr * (Pr + 1) + i] = P[i];
        } else {
          gemm<M>(kprev, Pr, Pl, Rp, Pl, 1, P, Pr, 1, S + kr * (Pr + 1), Pr + 1, 1, false);
        }
        __syncthreads();
        const int m = kr + kprev;
        house_qr_stacked(S, kr, m, Pr, Pr + 1, rred);
        kr = m < Pr ? m : Pr;
      }
      // store R_y (kr x Pr, row stride Pr) at unit scale: only its row space
      // and the ratios of its singular values matter downstream, and
      // without rescaling its norm grows by |P| per column (beyond the FP32
      // range on wide lattices)
      const int er = pow2_exponent((double)block_absmax(S, kr, Pr, Pr + 1, red));
      const Rl fr = (Rl)ldexp(1.0, -er);
      T* Ry = R + (size_t)y * BD * BD;
      for (int i = tid; i < kr * Pr; i += PEPS_NT) Ry[i] = S[(i / Pr) * (Pr + 1) + i % Pr] * fr;
      __syncthreads();
      kprev = kr;
    }

    // right-to-left SVD sweep
    int nbr = 1;       // new bond to the right of site y
    double logrow = 0.0;
    for (int y = L.Ly - 1; y >= 0; --y) {
      const int nsite = x * L.Ly + y;
      const SiteView v = site_view(tab, L, nsite, bottom);
      const int bl = edims[(sp * L.Ly + y) * 3 + 0];
      const int br = edims[(sp * L.Ly + y) * 3 + 2];
      const int Pl = bl * v.Dl;
      load_lds(Ebuf, Eprev + (size_t)y * L.site_box, bl * v.Din * br);
      const T* a = site_tensor(theta, tab, L, s, nsite);
      load_lds(Abuf, a, v.Dl * v.Dr * v.Din * v.Dout);
      if (y == L.Ly - 1) {
        if (tid == 0) W[0] = T(1);
      }
      __syncthreads();
      // T1[(a,in),(r,c)] = sum_b E[(a,in), b] W[(b,r), c]
      for (int r = 0; r < v.Dr; ++r)
        gemm<M>(bl * v.Din, nbr, br, Ebuf, br, 1, W + r * nbr, v.Dr * nbr, 1, P + r * nbr,
                v.Dr * nbr, 1, false);
      __syncthreads();
      // Z[(a,l),(k,c)] = sum_{in,r} T1[(a,in),(r,c)] A[l,r,in,k]
      const int zc = v.Dout * nbr;
      bool zdone = false;
      if constexpr (std::is_same<T, float>::value) {
        if ((nbr & 3) == 0 &&
            ((reinterpret_cast<uintptr_t>(P) | reinterpret_cast<uintptr_t>(Z)) & 15) == 0) {
          // four consecutive c per thread: T1 rows read as 16-byte vectors
          const int nq = nbr >> 2, totq = Pl * v.Dout * nq;
          const FastDiv fnq(nq), fDout(v.Dout), fDl(v.Dl);
          for (int i = tid; i < totq; i += PEPS_NT) {
            int q = i;
            const int cq = divmod(q, fnq);
            const int k = divmod(q, fDout);
            const int l = divmod(q, fDl);
            const int aa = q;
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int in = 0; in < v.Din; ++in)
              for (int r = 0; r < v.Dr; ++r)
                fma4(acc, opnd<M>(Abuf[l * v.s_l + r * v.s_r + in * v.s_in + k * v.s_out]),
                     op4<M>(ld4(P + (aa * v.Din + in) * (v.Dr * nbr) + r * nbr + 4 * cq)));
            st4(Z + (aa * v.Dl + l) * zc + k * nbr + 4 * cq, acc);
          }
          zdone = true;
        }
      }
      if (!zdone) {
        const int tot = Pl * zc;
        const FastDiv fzc(zc), fDl(v.Dl), fnbr(nbr);
        for (int i = tid; i < tot; i += PEPS_NT) {
          int row = i;
          int col = divmod(row, fzc);
          const int l = divmod(row, fDl);
          const int aa = row;
          const int c = divmod(col, fnbr);
          const int k = col;
          T acc = 0;
          for (int in = 0; in < v.Din; ++in)
            for (int r = 0; r < v.Dr; ++r)
              acc += opnd<M>(P[(aa * v.Din + in) * (v.Dr * nbr) + r * nbr + c]) *
                     opnd<M>(Abuf[l * v.s_l + r * v.s_r + in * v.s_in + k * v.s_out]);
          Z[i] = acc;
        }
      }
      __syncthreads();
      int rnew;
      T* newt;
      if (y > 0) {
        // recompute kprev = rows of R_{y-1}
        int kp = 1;
        for (int yy = 0; yy < y; ++yy) {
          const int ns2 = x * L.Ly + yy;
          const SiteView v2 = site_view(tab, L, ns2, bottom);
          const int br2 = edims[(sp * L.Ly + yy) * 3 + 2];
          const int rows = kp * v2.Dout, cols = br2 * v2.Dr;
          kp = rows < cols ? rows : cols;
        }
        const T* Rp = R + (size_t)(y - 1) * BD * BD;
        // C = R_{y-1} Z  (kp x zc)
        // row stride: 16-byte aligned and shifted by 16 bytes per row so the
        // Jacobi's vector LDS accesses of neighbouring rows use other banks
        const int ldc = zc + (int)(16 / sizeof(T));
        gemm<M>(kp, zc, Pl, Rp, Pl, 1, Z, zc, 1, S, ldc, 1, false);
        __syncthreads();
        int m = kp;
        if (m > zc) {
          house_qr_stacked(S, 0, m, zc, ldc, rred);
          m = zc;
        }
        const int used = jacobi_rows(S, m, zc, ldc, tol, jac_sweeps, sflag, vv);
        if (used < 0 && tid == 0) fl |= 4;
        // row norms, four lanes per row
        for (int i4 = tid; i4 < 4 * m; i4 += PEPS_NT) {
          const int i = i4 >> 2, part = i4 & 3;
          Rl q = 0;
          for (int e = part; e < zc; e += 4) q += abs2x(S[i * ldc + e]);
          q += dppx<0xB1>(q);
          q += dppx<0x4E>(q);
          if (part == 0) sig[i] = sqrt(q);
        }
        __syncthreads();
        rnew = edims[(sn * L.Ly + y) * 3 + 0];
        // rank rows by descending norm (ties by index); the largest value and
        // the largest discarded one (for the degenerate-cut flag); squared
        // norms of all rows and of the discarded ones (truncated weight)
        Rl smx = 0, sdis = 0, wall = 0, wdis = 0;
        for (int i = tid; i < m; i += PEPS_NT) {
          int rk = 0;
          const Rl si = sig[i];
          for (int j = 0; j < m; ++j) {
            const Rl sj = sig[j];
            rk += (sj > si) || (sj == si && j < i);
          }
          if (rk < rnew) {
            sel[rk] = i;
          } else {
            sdis = si > sdis ? si : sdis;
            wdis += si * si;
          }
          smx = si > smx ? si : smx;
          wall += si * si;
        }
        const Rl smax = block_max(smx, rred);
        const Rl sb = block_max(sdis, rred);
        // kept count: rnew, or with a maximal truncated weight w the fewest
        // rows whose discarded weight is at most w times the total, the
        // discarded squares added smallest first
        __shared__ int s_keep;
        if (L.trunc_w > 0.0) {
          const Rl wa = block_sum(wall, rred);
          const Rl wd = block_sum(wdis, rred);
          if (tid == 0) {
            const Rl lim = (Rl)L.trunc_w * wa;
            int r = rnew;
            Rl tail = wd;
            if (tail <= lim) {
              for (int j = rnew - 1; j >= 1; --j) {
                const Rl sj = sig[sel[j]];
                const Rl t2 = tail + sj * sj;
                if (t2 > lim) break;
                tail = t2;
                r = j;
              }
            }
            // a decision within a relative margin of the limit could fall
            // the other way under rounding: flag it like a degenerate cut
            const Rl marg = std::is_same<Rl, double>::value ? Rl(1e-8) : Rl(1e-4);
            bool near = fabs((double)(tail - lim)) <= (double)(marg * lim);
            if (r > 1 && tail <= lim) {
              const Rl sp = sig[sel[r - 1]];
              near = near || fabs((double)(tail + sp * sp - lim)) <= (double)(marg * lim);
            }
            if (near) fl |= 8;
            s_keep = r;
          }
        } else if (tid == 0) {
          s_keep = rnew;
        }
        __syncthreads();
        const int rkeep = s_keep;
        if (tid == 0 && rkeep < m) {
          const Rl sa = sig[sel[rkeep - 1]];
          const Rl sn = rkeep < rnew ? sig[sel[rkeep]] : sb;
          if (sa > Rl(0) && (sa - sn) < Rl(1e-8) * sa) fl |= 8;
        }
        const Rl thresh = smax * Eps<Rl>::v * Rl(4);
        for (int i = tid; i < rnew * zc; i += PEPS_NT) {
          const int j = i / zc, e = i - j * zc;
          const Rl sj = sig[sel[j]];
          Bn[i] = (j < rkeep && sj > thresh) ? S[sel[j] * ldc + e] / sj : T(0);
        }
        __syncthreads();
        // W_y[(a,l), j] = sum_e Z[(a,l), e] conj(Bn[j, e])
        gemm<M, IsCplx<T>::value>(Pl, rnew, zc, Z, zc, 1, Bn, 1, zc, W, rnew, 1, false);
        __syncthreads();
        // W carries the weight of the sites to its right: keep it at unit
        // scale and move the power of two into the log scale
        const int ew = pow2_exponent((double)block_absmax(W, Pl, rnew, rnew, red));
        scale_pow2(W, Pl * rnew, ew);
        logrow += ew * 0.69314718055994530942;
        newt = Bn;
      } else {
        rnew = 1;
        newt = Z;
      }
      __syncthreads();
      const int cnt = rnew * zc;
      logrow += normalize_lds(newt, cnt, red, flp);
      T* dst = Enew + (size_t)y * L.site_box;
      for (int i = tid; i < cnt; i += PEPS_NT) dst[i] = newt[i];
      nbr = rnew;
      __syncthreads();
    }
    if (tid == 0) lg[sn] = lg[sp] + logrow;
    __syncthreads();
  }

}  // namespace pm
