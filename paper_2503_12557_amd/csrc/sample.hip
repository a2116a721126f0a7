// Local Metropolis sampling of p(S) ~ |Psi(S)|^2 with ratios taken inside
// strips (Sec. "On reusing environments"); the paper names Markov chains
// as the alternative to its direct sampler (Sec. "On Direct Sampling").
//
// A sweep of every chain is a sequence of launches, one workgroup per chain
// in each, the chain's state passed in device memory between them:
//   * rebuild the bottom environments E^l[1..Lx-1] from the current state;
//   * for each row x from the top: propose the horizontal exchanges (x,y) <->
//     (x,y+1) left to right inside the one-row strip between E^u[x-1] and
//     E^l[x+1] (or single-site flips), then the vertical exchanges
//     (x,y) <-> (x+1,y) inside the two-row strip between E^u[x-1] and
//     E^l[x+2], then absorb the updated row x into E^u[x].
// Each phase is a kernel of its own, so each holds only its own registers
// and working set; on global-slab shapes the strip phases take the
// matrix-core steps. The environment phases use the context's truncation:
// the canonical kernel's steps, or the density-matrix ones (env_dm.hip).
// Rows below x+1 do not change while row x is processed, so the bottom
// environments stay valid for the whole sweep. A move is accepted iff
// u < |R|^2 with u from Philox4x32-10 keyed by the seed and counter
// (move id, sweep + offset, chain, tag); aligned pairs are not proposed.
#include "common.h"
#include "env_dev.h"
#include "kernels.h"
#include "strip_dev.h"

namespace pm {

#define TAG_MOVE 0x4D4F5645u
#define TAG_INIT 0x494E4954u
#define SMP_RED 16  // reduction scratch of the strip phases (elements)

// Working sets of the phases, in elements ("big": LDS, or a global slab per
// chain for large shapes, shared by the phases since they run in turn).
__host__ __device__ static size_t smp_row1_big(int bmax, int D) {
  const size_t BD = (size_t)bmax * D, box = (size_t)bmax * D * bmax;
  return 3 * box + 2 * BD * BD;
}
__host__ __device__ static size_t smp_row2_big(int bmax, int D, bool mm) {
  const size_t box2 = (size_t)bmax * bmax * D * D, bd3 = (size_t)bmax * D * D * D;
  return mm ? 2 * box2 + 2 * box2 * D : 2 * box2 + 3 * S2G * bd3;
}
__host__ __device__ static size_t sample_big(int bmax, int D, int mode, bool gm) {
  size_t m = env_big_elems(bmax, D, mode);
  const size_t r1 = smp_row1_big(bmax, D), r2 = smp_row2_big(bmax, D, gm);
  m = r1 > m ? r1 : m;
  return r2 > m ? r2 : m;
}

// accept iff u < |R|^2, u from Philox keyed by (move, sweep, chain, tag)
__device__ __forceinline__ bool smp_decide(int move, uint32_t sweep, int chain, uint32_t k0,
                                           uint32_t k1, double r2) {
  u4 c;
  c.x = (uint32_t)move;
  c.y = sweep;
  c.z = (uint32_t)chain;
  c.w = TAG_MOVE;
  const u4 o = philox(c, k0, k1);
  return philox_uniform(o.x, o.y) < r2;
}
template <typename T>
__device__ __forceinline__ double smp_ratio2(const T& num, const T& den) {
  if constexpr (IsCplx<T>::value) {
    return (double)abs2x(num) / (double)abs2x(den);
  } else {
    const double ratio = (double)num / (double)den;
    return ratio * ratio;
  }
}

// Initial states: an S_z = 0 permutation by the ranks of Philox keys
// (exchange moves) or independent bits (flips); acceptance counts cleared.
__global__ void __launch_bounds__(256) k_smp_init(int N, int kind, int n_chains, uint32_t k0,
                                                  uint32_t k1, uint8_t* __restrict__ state,
                                                  int* __restrict__ acc) {
  const int chain = blockIdx.x;
  if (chain >= n_chains) return;
  __shared__ uint32_t keys[1024];
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    u4 c;
    c.x = (uint32_t)n;
    c.y = 0u;
    c.z = (uint32_t)chain;
    c.w = TAG_INIT;
    keys[n] = philox(c, k0, k1).x;
  }
  __syncthreads();
  uint8_t* s = state + (size_t)chain * N;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    if (kind == 0) {
      int rk = 0;
      const uint32_t kn = keys[n];
      for (int m = 0; m < N; ++m) rk += (keys[m] < kn) || (keys[m] == kn && m < n);
      s[n] = rk < N / 2 ? 0 : 1;
    } else {
      s[n] = (uint8_t)(keys[n] & 1u);
    }
  }
  if (threadIdx.x == 0) acc[chain] = 0;
}

// Environment phase: row < 0 rebuilds the bottom environments of the
// current state, row >= 0 absorbs that row into the top environment.
template <int M, bool GM>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_smp_env(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
          int n_chains, int row, const uint8_t* __restrict__ state,
          typename ModeT<M>::T* __restrict__ envscr, double* __restrict__ logscr,
          typename ModeT<M>::T* __restrict__ rscr, int jac_sweeps,
          typename ModeT<M>::T* __restrict__ gws, size_t slab) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int chain = blockIdx.x;
  if (chain >= n_chains) return;
  const int tid = threadIdx.x, N = L.N, BD = L.bmax * L.D;
  T* sm = GM ? gws + (size_t)chain * slab : lds;
  T* small = GM ? lds : lds + env_big_elems(L.bmax, L.D, M);
  const EnvSmem<T> sh(sm, small, L, tsqr_path(M, L.bmax, L.D) && PEPS_NT == 256);
  __shared__ uint8_t s[1024];
  __shared__ int sflag[2], fl;
  __shared__ int sel[256];
  for (int n = tid; n < N; n += PEPS_NT) s[n] = state[(size_t)chain * N + n];
  if (tid == 0) fl = 0;
  __syncthreads();
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  T* envs = envscr + (size_t)chain * L.n_slots * slot_elems;
  double* lg = logscr + (size_t)chain * L.n_slots;
  T* R = rscr + (size_t)chain * L.Ly * BD * BD;
  // one call site of each step (bottom: first row, then rows 1 .. Lx-2;
  // top: row 0 is the first row, a later row one absorption)
  const bool bottom = row < 0;
  if (row <= 0) env_first_row<M>(L, tab, theta, s, bottom, envs, lg, sh, &fl);
  const int t0 = bottom ? 1 : row, t1 = bottom ? L.Lx - 2 : row;
  for (int t = t0 > 1 ? t0 : 1; t <= t1; ++t)
    env_absorb_row<M>(L, tab, theta, s, bottom, t, envs, lg, R, sh, sel, sflag, &fl, jac_sweeps);
}

// environment bonds and tensors of the strips of row x
template <typename T>
struct SmpRowEnv {
  const Lattice& L;
  const int* ed;
  const T* envs;
  const T* one;
  int su, sd, sd2;
  __device__ SmpRowEnv(const Lattice& L_, const int* tab, const T* envs_, const T* one_, int x)
      : L(L_), ed(tab + L_.off_env), envs(envs_), one(one_) {
    su = x > 0 ? slot_top(L, x - 1) : -1;
    sd = x < L.Lx - 1 ? slot_bottom(L, x + 1) : -1;
    sd2 = x + 1 < L.Lx - 1 ? slot_bottom(L, x + 2) : -1;
  }
  __device__ const T* up(int y) const { return su >= 0 ? env_site(envs, L, su, y) : one; }
  __device__ const T* dn(int y) const { return sd >= 0 ? env_site(envs, L, sd, y) : one; }
  __device__ const T* dn2(int y) const { return sd2 >= 0 ? env_site(envs, L, sd2, y) : one; }
  __device__ int ua(int y) const { return su >= 0 ? ed[(su * L.Ly + y) * 3 + 0] : 1; }
  __device__ int uk(int y) const { return su >= 0 ? ed[(su * L.Ly + y) * 3 + 1] : 1; }
  __device__ int ub(int y) const { return su >= 0 ? ed[(su * L.Ly + y) * 3 + 2] : 1; }
  __device__ int ba(int y) const { return sd >= 0 ? ed[(sd * L.Ly + y) * 3 + 0] : 1; }
  __device__ int bb(int y) const { return sd >= 0 ? ed[(sd * L.Ly + y) * 3 + 2] : 1; }
  __device__ int ba2(int y) const { return sd2 >= 0 ? ed[(sd2 * L.Ly + y) * 3 + 0] : 1; }
  __device__ int bb2(int y) const { return sd2 >= 0 ? ed[(sd2 * L.Ly + y) * 3 + 2] : 1; }
};

#define SMP_WAVES(M, GM) ((GM) && ((M) == MODE_F32 || (M) == MODE_C64) ? 4 : 1)

// One-row phase of row x: horizontal exchanges (or flips) left to right.
template <int M, bool GM>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX, SMP_WAVES(M, GM))
k_smp_row1(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
           int kind, int n_chains, int x, uint32_t sweep_ctr, uint32_t k0, uint32_t k1,
           uint8_t* __restrict__ state, int* __restrict__ acc,
           const typename ModeT<M>::T* __restrict__ envscr, typename ModeT<M>::T* __restrict__ rt1,
           typename ModeT<M>::T* __restrict__ gws, size_t slab) {
  typedef typename ModeT<M>::T T;
  typedef typename RealOf<T>::type Rl;
  constexpr bool MMP = GM;
  constexpr bool BFP = M == MODE_BF16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int chain = blockIdx.x;
  if (chain >= n_chains) return;
  const int tid = threadIdx.x, Ly = L.Ly, N = L.N;
  const int B = L.bmax, D = L.D, BD = B * D, box = B * D * B;
  T* sm = GM ? gws + (size_t)chain * slab : lds;
  T* red = GM ? lds : lds + smp_row1_big(B, D);
  T* Lf = sm;
  T* Lt = Lf + box;
  T* Lt2 = Lt + box;
  T* X1 = Lt2 + box;
  T* X2 = X1 + BD * BD;
  __shared__ uint8_t s[1024];
  __shared__ int dex[32], nacc;
  __shared__ T one[1];
  for (int n = tid; n < N; n += PEPS_NT) s[n] = state[(size_t)chain * N + n];
  if (tid == 0) {
    one[0] = T(1);
    nacc = 0;
  }
  __syncthreads();
  const size_t slot_elems = (size_t)Ly * L.site_box;
  const SmpRowEnv<T> ev(L, tab, envscr + (size_t)chain * L.n_slots * slot_elems, one, x);
  T* Rt = rt1 + (size_t)chain * (Ly + 1) * box;
  auto tens = [&](int n, int p) -> const T* {
    return theta + tab[L.off_param + n] + p * tab[L.off_block + n];
  };
  auto left = [&](const T* Lp, int y, const T* A, int dl, int dr, int du, int dd, T* out) {
    if constexpr (MMP)
      s1_step_left_mm<T, BFP>(Lp, ev.up(y), ev.ua(y), ev.ub(y), A, dl, dr, du, dd, ev.dn(y),
                              ev.ba(y), ev.bb(y), X1, X2, out);
    else
      s1_step_left<M>(Lp, ev.up(y), ev.ua(y), ev.ub(y), A, dl, dr, du, dd, ev.dn(y), ev.ba(y),
                      ev.bb(y), X1, X2, out);
  };
  // right partials of the current row, each at unit scale (power of two in
  // dex[y], taken out of the left steps too)
  if (tid == 0) Rt[(size_t)Ly * box] = T(1);
  __syncthreads();
  for (int y = Ly - 1; y >= 0; --y) {
    const int ns = x * Ly + y;
    int Dl, Dr, Du, Dd;
    legs_of(tab, L, ns, Dl, Dr, Du, Dd);
    T* Ry = Rt + (size_t)y * box;
    if constexpr (MMP)
      s1_step_right_mm<T, BFP>(Rt + (size_t)(y + 1) * box, ev.up(y), ev.ua(y), ev.ub(y),
                               tens(ns, s[ns]), Dl, Dr, Du, Dd, ev.dn(y), ev.ba(y), ev.bb(y), X1,
                               X2, Ry);
    else
      s1_step_right<M>(Rt + (size_t)(y + 1) * box, ev.up(y), ev.ua(y), ev.ub(y),
                       tens(ns, s[ns]), Dl, Dr, Du, Dd, ev.dn(y), ev.ba(y), ev.bb(y), X1, X2, Ry);
    const int cnt = ev.ua(y) * Dl * ev.ba(y);
    const int e = pow2_exponent((double)block_absmax(Ry, 1, cnt, cnt, red));
    scale_pow2(Ry, cnt, e);
    if (tid == 0) dex[y] = e;
    __syncthreads();
  }
  if (tid == 0) Lf[0] = T(1);
  __syncthreads();
  for (int y = 0; y < Ly; ++y) {
    const int n1 = x * Ly + y;
    const int nw = (kind == 0) ? 2 : 1;
    const bool propose = (kind == 0) ? (y < Ly - 1) && (s[n1] != s[n1 + 1]) : true;
    if (propose) {
      const int move = (kind == 0) ? x * (2 * Ly - 1) + y : n1;
      T val[2];
      for (int which = 0; which < 2; ++which) {  // 0: current, 1: proposed
        const T* cur = Lf;
        T* nxt = Lt;
        for (int j = 0; j < nw; ++j) {
          const int nn = n1 + j;
          int p = s[nn];
          if (which == 1) p = (kind == 0) ? s[n1 + (1 - j)] : 1 - s[nn];
          int dl, dr, du, dd;
          legs_of(tab, L, nn, dl, dr, du, dd);
          left(cur, y + j, tens(nn, p), dl, dr, du, dd, nxt);
          scale_pow2(nxt, ev.ub(y + j) * dr * ev.bb(y + j), dex[y + j]);
          __syncthreads();
          cur = nxt;
          nxt = (nxt == Lt) ? Lt2 : Lt;
        }
        const int ye = y + nw - 1;
        const int cnt = ev.ub(ye) * tab[L.off_legs + 4 * (x * Ly + ye) + 1] * ev.bb(ye);
        val[which] = lds_dot(cur, (const T*)(Rt + (size_t)(ye + 1) * box), cnt, red);
      }
      if (smp_decide(move, sweep_ctr, chain, k0, k1, smp_ratio2(val[1], val[0]))) {
        if (tid == 0) {
          if (kind == 0) {
            const uint8_t a = s[n1];
            s[n1] = s[n1 + 1];
            s[n1 + 1] = a;
          } else {
            s[n1] = 1 - s[n1];
          }
          nacc += 1;
        }
      }
      __syncthreads();
    }
    int Dl, Dr, Du, Dd;
    legs_of(tab, L, n1, Dl, Dr, Du, Dd);
    left(Lf, y, tens(n1, s[n1]), Dl, Dr, Du, Dd, Lt);
    {
      const Rl f = (Rl)ldexp(1.0, -dex[y]);
      for (int i = tid; i < ev.ub(y) * Dr * ev.bb(y); i += PEPS_NT) Lf[i] = Lt[i] * f;
    }
    __syncthreads();
  }
  for (int n = tid; n < N; n += PEPS_NT) state[(size_t)chain * N + n] = s[n];
  if (tid == 0) acc[chain] += nacc;
}

// Two-row phase of rows (x, x+1): vertical exchanges left to right.
template <int M, bool GM>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX, SMP_WAVES(M, GM))
k_smp_row2(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
           int n_chains, int x, uint32_t sweep_ctr, uint32_t k0, uint32_t k1,
           uint8_t* __restrict__ state, int* __restrict__ acc,
           const typename ModeT<M>::T* __restrict__ envscr, typename ModeT<M>::T* __restrict__ rt2,
           typename ModeT<M>::T* __restrict__ gws, size_t slab) {
  typedef typename ModeT<M>::T T;
  typedef typename RealOf<T>::type Rl;
  constexpr bool MMP = GM;
  constexpr bool BFP = M == MODE_BF16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int chain = blockIdx.x;
  if (chain >= n_chains) return;
  const int tid = threadIdx.x, Ly = L.Ly, N = L.N;
  const int B = L.bmax, D = L.D;
  const int box2 = B * B * D * D, bd3 = B * D * D * D;
  T* sm = GM ? gws + (size_t)chain * slab : lds;
  T* red = GM ? lds : lds + smp_row2_big(B, D, false);
  // Lf2 | Lu (box2 each) | Y1 | Y2 | Y3 (S2G B D^3 each), or with the
  // matrix-core steps X1 | X2 (B^2 D^3 each)
  T* Lf2 = sm;
  T* Lu = Lf2 + box2;
  T* Y1 = Lu + box2;
  T* Y2 = Y1 + (MMP ? (size_t)box2 * D : (size_t)S2G * bd3);
  T* Y3 = Y2 + S2G * bd3;
  __shared__ uint8_t s[1024];
  __shared__ int dex[32], nacc;
  __shared__ T one[1];
  for (int n = tid; n < N; n += PEPS_NT) s[n] = state[(size_t)chain * N + n];
  if (tid == 0) {
    one[0] = T(1);
    nacc = 0;
  }
  __syncthreads();
  const size_t slot_elems = (size_t)Ly * L.site_box;
  const SmpRowEnv<T> ev(L, tab, envscr + (size_t)chain * L.n_slots * slot_elems, one, x);
  T* Rt2 = rt2 + (size_t)chain * (Ly + 1) * box2;
  auto tens = [&](int n, int p) -> const T* {
    return theta + tab[L.off_param + n] + p * tab[L.off_block + n];
  };
  auto left = [&](int y, const T* A1, int Dl1, int Dr1, int Dd1, const T* A2, int Dl2, int Dr2,
                  int Dd2, T* out) {
    if constexpr (MMP)
      s2_step_left_mm<T, BFP>(Lf2, ev.up(y), ev.ua(y), ev.uk(y), ev.ub(y), A1, Dl1, Dr1, Dd1, A2,
                              Dl2, Dr2, Dd2, ev.dn2(y), ev.ba2(y), ev.bb2(y), Y1, Y2, out);
    else
      s2_step_left<M>(Lf2, ev.up(y), ev.ua(y), ev.uk(y), ev.ub(y), A1, Dl1, Dr1, Dd1, A2, Dl2,
                      Dr2, Dd2, ev.dn2(y), ev.ba2(y), ev.bb2(y), Y1, Y2, Y3, out);
  };
  if (tid == 0) Rt2[(size_t)Ly * box2] = T(1);
  __syncthreads();
  for (int y = Ly - 1; y >= 0; --y) {
    const int n1 = x * Ly + y, n2 = n1 + Ly;
    int Dl1, Dr1, Du1, Dd1, Dl2, Dr2, Du2, Dd2;
    legs_of(tab, L, n1, Dl1, Dr1, Du1, Dd1);
    legs_of(tab, L, n2, Dl2, Dr2, Du2, Dd2);
    T* Ry = Rt2 + (size_t)y * box2;
    if constexpr (MMP)
      s2_step_right_mm<T, BFP>(Rt2 + (size_t)(y + 1) * box2, ev.up(y), ev.ua(y), ev.uk(y),
                               ev.ub(y), tens(n1, s[n1]), Dl1, Dr1, Dd1, tens(n2, s[n2]), Dl2, Dr2,
                               Dd2, ev.dn2(y), ev.ba2(y), ev.bb2(y), Y1, Y2, Ry);
    else
      s2_step_right<M>(Rt2 + (size_t)(y + 1) * box2, ev.up(y), ev.ua(y), ev.uk(y), ev.ub(y),
                       tens(n1, s[n1]), Dl1, Dr1, Dd1, tens(n2, s[n2]), Dl2, Dr2, Dd2, ev.dn2(y),
                       ev.ba2(y), ev.bb2(y), Y1, Y2, Y3, Ry);
    const int cnt = ev.ua(y) * Dl1 * Dl2 * ev.ba2(y);
    const int e = pow2_exponent((double)block_absmax(Ry, 1, cnt, cnt, red));
    scale_pow2(Ry, cnt, e);
    if (tid == 0) dex[y] = e;
    __syncthreads();
  }
  if (tid == 0) Lf2[0] = T(1);
  __syncthreads();
  for (int y = 0; y < Ly; ++y) {
    const int n1 = x * Ly + y, n2 = n1 + Ly;
    int Dl1, Dr1, Du1, Dd1, Dl2, Dr2, Du2, Dd2;
    legs_of(tab, L, n1, Dl1, Dr1, Du1, Dd1);
    legs_of(tab, L, n2, Dl2, Dr2, Du2, Dd2);
    const int cnt = ev.ub(y) * Dr1 * Dr2 * ev.bb2(y);
    if (s[n1] != s[n2]) {
      T val[2];
      for (int which = 0; which < 2; ++which) {
        const int p1 = which ? s[n2] : s[n1];
        const int p2 = which ? s[n1] : s[n2];
        left(y, tens(n1, p1), Dl1, Dr1, Dd1, tens(n2, p2), Dl2, Dr2, Dd2, Lu);
        val[which] = lds_dot(Lu, (const T*)(Rt2 + (size_t)(y + 1) * box2), cnt, red);
      }
      if (smp_decide(x * (2 * Ly - 1) + Ly - 1 + y, sweep_ctr, chain, k0, k1,
                     smp_ratio2(val[1], val[0]))) {
        if (tid == 0) {
          const uint8_t a = s[n1];
          s[n1] = s[n2];
          s[n2] = a;
          nacc += 1;
        }
      }
      __syncthreads();
    }
    left(y, tens(n1, s[n1]), Dl1, Dr1, Dd1, tens(n2, s[n2]), Dl2, Dr2, Dd2, Lu);
    {
      const Rl f = (Rl)ldexp(1.0, -dex[y]);
      for (int i = tid; i < cnt; i += PEPS_NT) Lf2[i] = Lu[i] * f;
    }
    __syncthreads();
  }
  for (int n = tid; n < N; n += PEPS_NT) state[(size_t)chain * N + n] = s[n];
  if (tid == 0) acc[chain] += nacc;
}

// the current states as record rec of every chain
__global__ void k_smp_record(int N, int n_chains, int per_chain, int rec,
                             const uint8_t* __restrict__ state, uint8_t* __restrict__ samples) {
  const int chain = blockIdx.x;
  if (chain >= n_chains) return;
  uint8_t* dst = samples + ((size_t)chain * per_chain + rec) * N;
  for (int n = threadIdx.x; n < N; n += blockDim.x) dst[n] = state[(size_t)chain * N + n];
}

__global__ void k_smp_accepted(int n_chains, const int* __restrict__ acc,
                               int* __restrict__ accepted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_chains) accepted[i] = acc[i];
}

size_t sample_lds_elems(int bmax, int D, int mode) {
  return sample_big(bmax, D, mode, false) + env_small_elems(bmax, D);
}
size_t sample_lds_bytes(int mode, const Lattice& L, bool gm) {
  return (gm ? env_small_elems(L.bmax, L.D) : sample_lds_elems(L.bmax, L.D, mode)) *
         mode_elem_bytes(mode);
}
size_t sample_slab_elems(const Lattice& L, int mode) {
  return (sample_big(L.bmax, L.D, mode, true) + 15) / 16 * 16;
}
size_t sample_state_bytes(const Lattice& L, int n_chains) {
  return ((size_t)n_chains * L.N + 255) / 256 * 256 + (size_t)n_chains * sizeof(int);
}

template <int M, bool GM>
static hipError_t metropolis_impl(const Lattice& L, const int* tab, const void* theta_v, int kind,
                                  int n_chains, int per_chain, int burn_in, int thin,
                                  uint64_t seed, uint64_t offset, uint8_t* samples, int* accepted,
                                  void* envscr, double* logscr, void* rscr, void* rt1, void* rt2,
                                  int jac_sweeps, void* gws, void* state_v, void* dm_slabs,
                                  hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const T* theta = (const T*)theta_v;
  const size_t es = sizeof(T);
  const size_t slab = GM ? sample_slab_elems(L, M) : 0;
  const size_t lds_env =
      (GM ? 0 : env_big_elems(L.bmax, L.D, M)) * es + env_small_elems(L.bmax, L.D) * es;
  const size_t lds_r1 = ((GM ? 0 : smp_row1_big(L.bmax, L.D)) + SMP_RED) * es;
  const size_t lds_r2 = ((GM ? 0 : smp_row2_big(L.bmax, L.D, false)) + SMP_RED) * es;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_smp_env<M, GM>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_env)) !=
      hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_smp_row1<M, GM>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_r1)) !=
      hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_smp_row2<M, GM>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_r2)) !=
      hipSuccess)
    return e;
  uint8_t* state = (uint8_t*)state_v;
  int* acc = (int*)(state + ((size_t)n_chains * L.N + 255) / 256 * 256);
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  T* g = (T*)gws;
  hipLaunchKernelGGL(k_smp_init, dim3(n_chains), dim3(256), 0, st, L.N, kind, n_chains, k0, k1,
                     state, acc);
  // environment phase: the canonical kernel, or the density-matrix one
  auto env_phase = [&](int row) -> hipError_t {
    if (dm_slabs)
      return launch_smp_env_dm(L, tab, M, theta, n_chains, row, state, envscr, logscr, dm_slabs,
                               st);
    hipLaunchKernelGGL((k_smp_env<M, GM>), dim3(n_chains), dim3(env_threads(M)), lds_env, st, L,
                       tab, theta, n_chains, row, (const uint8_t*)state, (T*)envscr, logscr,
                       (T*)rscr, jac_sweeps, g, slab);
    return hipSuccess;
  };
  const int total = burn_in + per_chain * thin;
  int rec = 0;
  for (int sw = 0; sw < total; ++sw) {
    const uint32_t sweep_ctr = (uint32_t)(sw + offset);
    if ((e = env_phase(-1)) != hipSuccess) return e;
    for (int x = 0; x < L.Lx; ++x) {
      hipLaunchKernelGGL((k_smp_row1<M, GM>), dim3(n_chains), dim3(PEPS_BLOCK_MAX), lds_r1, st,
                         L, tab, theta, kind, n_chains, x, sweep_ctr, k0, k1, state, acc,
                         (const T*)envscr, (T*)rt1, g, slab);
      if (kind == 0 && x < L.Lx - 1)
        hipLaunchKernelGGL((k_smp_row2<M, GM>), dim3(n_chains), dim3(PEPS_BLOCK_MAX), lds_r2, st,
                           L, tab, theta, n_chains, x, sweep_ctr, k0, k1, state, acc,
                           (const T*)envscr, (T*)rt2, g, slab);
      if (x < L.Lx - 1 && (e = env_phase(x)) != hipSuccess) return e;
    }
    if (sw >= burn_in && (sw - burn_in) % thin == thin - 1) {
      hipLaunchKernelGGL(k_smp_record, dim3(n_chains), dim3(256), 0, st, L.N, n_chains,
                         per_chain, rec, (const uint8_t*)state, samples);
      ++rec;
    }
  }
  if (accepted)
    hipLaunchKernelGGL(k_smp_accepted, dim3((n_chains + 255) / 256), dim3(256), 0, st, n_chains,
                       (const int*)acc, accepted);
  return hipGetLastError();
}

template <int M>
hipError_t launch_metropolis(const Lattice& L, const int* tab, const void* theta, int kind,
                             int n_chains, int per_chain, int burn_in, int thin, uint64_t seed,
                             uint64_t offset, uint8_t* samples, int* accepted, void* envscr,
                             double* logscr, void* rscr, void* rt1, void* rt2, int jac_sweeps,
                             void* gws, void* state, void* dm_slabs, hipStream_t st) {
  if (gws)
    return metropolis_impl<M, true>(L, tab, theta, kind, n_chains, per_chain, burn_in, thin,
                                    seed, offset, samples, accepted, envscr, logscr, rscr, rt1,
                                    rt2, jac_sweeps, gws, state, dm_slabs, st);
  return metropolis_impl<M, false>(L, tab, theta, kind, n_chains, per_chain, burn_in, thin, seed,
                                   offset, samples, accepted, envscr, logscr, rscr, rt1, rt2,
                                   jac_sweeps, nullptr, state, dm_slabs, st);
}

#define INST(M)                                                                                  \
  template hipError_t launch_metropolis<M>(const Lattice&, const int*, const void*, int, int,   \
                                           int, int, int, uint64_t, uint64_t, uint8_t*, int*,   \
                                           void*, double*, void*, void*, void*, int, void*,     \
                                           void*, void*, hipStream_t);
INST(MODE_F64)
INST(MODE_F32)
INST(MODE_BF16)
INST(MODE_C128)
INST(MODE_C64)
#undef INST

}  // namespace pm
