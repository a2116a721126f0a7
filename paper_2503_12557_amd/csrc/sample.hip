// Local Metropolis sampling of p(S) ~ |Psi(S)|^2 with ratios taken inside
// strips (Sec. "On reusing environments"); the paper names Markov chains
// as the alternative to its direct sampler (Sec. "On Direct Sampling").
//
// One workgroup owns one chain and runs every sweep of it:
//   * rebuild the bottom environments E^l[1..Lx-1] from the current state;
//   * for each row x from the top: propose the horizontal exchanges (x,y) <->
//     (x,y+1) left to right inside the one-row strip between E^u[x-1] and
//     E^l[x+1] (or single-site flips), then the vertical exchanges
//     (x,y) <-> (x+1,y) inside the two-row strip between E^u[x-1] and
//     E^l[x+2], then absorb the updated row x into E^u[x].
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

// Working set of a chain: the matrices of whichever phase runs ("big": in
// LDS, or in a global slab for large shapes) and the vectors and reduction
// scratch ("small": LDS).
__host__ __device__ static size_t sample_big(int bmax, int D, int mode) {
  const size_t BD = (size_t)bmax * D;
  const size_t box = (size_t)bmax * D * bmax;
  const size_t box2 = (size_t)bmax * bmax * D * D;
  const size_t bd3 = (size_t)bmax * D * D * D;
  const size_t one_row = 3 * box + 2 * BD * BD;
  const size_t two_row = 2 * box2 + 3 * S2G * bd3;
  size_t m = env_big_elems(bmax, D, mode);
  m = one_row > m ? one_row : m;
  return two_row > m ? two_row : m;
}

template <int M, bool GM>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_metropolis(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
             int kind, int n_chains, int per_chain, int burn_in, int thin, uint32_t k0, uint32_t k1,
             uint64_t offset, uint8_t* __restrict__ samples, int* __restrict__ accepted,
             typename ModeT<M>::T* __restrict__ envscr, double* __restrict__ logscr,
             typename ModeT<M>::T* __restrict__ rscr, typename ModeT<M>::T* __restrict__ rt1,
             typename ModeT<M>::T* __restrict__ rt2, int jac_sweeps,
             typename ModeT<M>::T* __restrict__ gws, size_t slab) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int chain = blockIdx.x;
  if (chain >= n_chains) return;
  const int tid = threadIdx.x;
  const int Lx = L.Lx, Ly = L.Ly, N = L.N;
  const int B = L.bmax, D = L.D, BD = B * D;
  const int box = B * D * B;
  const int box2 = B * B * D * D;
  const int bd3 = B * D * D * D;
  T* sm = GM ? gws + (size_t)chain * slab : lds;
  T* small = GM ? lds : lds + sample_big(B, D, M);
  const EnvSmem<T> sh(sm, small, L, tsqr_path(M, L.bmax, L.D) && PEPS_NT == 256);
  // strip buffers alias the environment buffers (used in different phases)
  // one-row pass: Lf | Lt | Lt2 (box each) | X1 | X2 (BD^2 each)
  T* Lf = sm;
  T* Lt = Lf + box;
  T* Lt2 = Lt + box;
  T* X1 = Lt2 + box;
  T* X2 = X1 + BD * BD;
  T* red = small;
  // two-row pass: Lf2 | Lu (box2 each) | Y1 | Y2 | Y3 (B D^3 each)
  T* Lf2 = sm;
  T* Lu = Lf2 + box2;
  T* Y1 = Lu + box2;
  T* Y2 = Y1 + S2G * bd3;
  T* Y3 = Y2 + S2G * bd3;
  T* red2 = small;
  __shared__ uint8_t s[1024];
  __shared__ int sflag[2], fl, acc;
  __shared__ int sel[256];
  __shared__ T one[1];
  __shared__ uint32_t keys[1024];
  __shared__ int dex[32];  // powers of two of the strip's right partials
  typedef typename RealOf<T>::type Rl;

  const size_t slot_elems = (size_t)Ly * L.site_box;
  T* envs = envscr + (size_t)chain * L.n_slots * slot_elems;
  double* lg = logscr + (size_t)chain * L.n_slots;
  T* R = rscr + (size_t)chain * Ly * BD * BD;
  T* Rt = rt1 + (size_t)chain * (Ly + 1) * box;
  T* Rt2 = rt2 + (size_t)chain * (Ly + 1) * box2;
  const int* ed = tab + L.off_env;

  // initial state
  for (int n = tid; n < N; n += PEPS_NT) {
    u4 c;
    c.x = (uint32_t)n;
    c.y = 0u;
    c.z = (uint32_t)chain;
    c.w = TAG_INIT;
    keys[n] = philox(c, k0, k1).x;
  }
  if (tid == 0) {
    fl = 0;
    acc = 0;
    one[0] = T(1);
  }
  __syncthreads();
  for (int n = tid; n < N; n += PEPS_NT) {
    if (kind == 0) {
      int rk = 0;
      const uint32_t kn = keys[n];
      for (int m = 0; m < N; ++m) rk += (keys[m] < kn) || (keys[m] == kn && m < n);
      s[n] = rk < N / 2 ? 0 : 1;
    } else {
      s[n] = (uint8_t)(keys[n] & 1u);
    }
  }
  __syncthreads();

  auto tens = [&](int n, int p) -> const T* {
    return theta + tab[L.off_param + n] + p * tab[L.off_block + n];
  };
  // accept iff u < |R|^2
  auto decide = [&](int move, uint32_t sweep, double r2) -> bool {
    u4 c;
    c.x = (uint32_t)move;
    c.y = sweep;
    c.z = (uint32_t)chain;
    c.w = TAG_MOVE;
    const u4 o = philox(c, k0, k1);
    const double u = philox_uniform(o.x, o.y);
    return u < r2;
  };
  auto ratio2 = [&](const T& num, const T& den) -> double {
    if constexpr (IsCplx<T>::value) {
      return (double)abs2x(num) / (double)abs2x(den);
    } else {
      const double ratio = (double)num / (double)den;
      return ratio * ratio;
    }
  };

  const int total = burn_in + per_chain * thin;
  int rec = 0;
  for (int sw = 0; sw < total; ++sw) {
    const uint32_t sweep_ctr = (uint32_t)(sw + offset);
    // bottom environments of the current state
    env_first_row<M>(L, tab, theta, s, true, envs, lg, sh, &fl);
    for (int t = 1; t <= Lx - 2; ++t)
      env_absorb_row<M>(L, tab, theta, s, true, t, envs, lg, R, sh, sel, sflag, &fl, jac_sweeps);
    for (int x = 0; x < Lx; ++x) {
      const bool has_up = x > 0, has_dn = x < Lx - 1;
      const int su = has_up ? slot_top(L, x - 1) : -1;
      const int sd = has_dn ? slot_bottom(L, x + 1) : -1;
      auto upT = [&](int y) -> const T* { return has_up ? env_site(envs, L, su, y) : one; };
      auto dnT = [&](int y) -> const T* { return has_dn ? env_site(envs, L, sd, y) : one; };
      auto ua_ = [&](int y) { return has_up ? ed[(su * Ly + y) * 3 + 0] : 1; };
      auto uk_ = [&](int y) { return has_up ? ed[(su * Ly + y) * 3 + 1] : 1; };
      auto ub_ = [&](int y) { return has_up ? ed[(su * Ly + y) * 3 + 2] : 1; };
      auto ba_ = [&](int y) { return has_dn ? ed[(sd * Ly + y) * 3 + 0] : 1; };
      auto bb_ = [&](int y) { return has_dn ? ed[(sd * Ly + y) * 3 + 2] : 1; };

      // ---- one-row strip: right partials of the current row, each at unit
      // scale (power of two in dex[y], taken out of the left steps too) ----
      if (tid == 0) Rt[(size_t)Ly * box] = T(1);
      __syncthreads();
      for (int y = Ly - 1; y >= 0; --y) {
        const int ns = x * Ly + y;
        int Dl, Dr, Du, Dd;
        legs_of(tab, L, ns, Dl, Dr, Du, Dd);
        T* Ry = Rt + (size_t)y * box;
        s1_step_right<M>(Rt + (size_t)(y + 1) * box, upT(y), ua_(y), ub_(y), tens(ns, s[ns]), Dl,
                         Dr, Du, Dd, dnT(y), ba_(y), bb_(y), X1, X2, Ry);
        const int cnt = ua_(y) * Dl * ba_(y);
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
        bool propose = false;
        if (kind == 0) propose = (y < Ly - 1) && (s[n1] != s[n1 + 1]);
        else propose = true;
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
              s1_step_left<M>(cur, upT(y + j), ua_(y + j), ub_(y + j), tens(nn, p), dl, dr, du,
                              dd, dnT(y + j), ba_(y + j), bb_(y + j), X1, X2, nxt);
              scale_pow2(nxt, ub_(y + j) * dr * bb_(y + j), dex[y + j]);
              __syncthreads();
              cur = nxt;
              nxt = (nxt == Lt) ? Lt2 : Lt;
            }
            const int ye = y + nw - 1;
            const int cnt = ub_(ye) * tab[L.off_legs + 4 * (x * Ly + ye) + 1] * bb_(ye);
            val[which] = lds_dot(cur, (const T*)(Rt + (size_t)(ye + 1) * box), cnt, red);
          }
          if (decide(move, sweep_ctr, ratio2(val[1], val[0]))) {
            if (tid == 0) {
              if (kind == 0) {
                const uint8_t a = s[n1];
                s[n1] = s[n1 + 1];
                s[n1 + 1] = a;
              } else {
                s[n1] = 1 - s[n1];
              }
              acc += 1;
            }
          }
          __syncthreads();
        }
        int Dl, Dr, Du, Dd;
        legs_of(tab, L, n1, Dl, Dr, Du, Dd);
        s1_step_left<M>(Lf, upT(y), ua_(y), ub_(y), tens(n1, s[n1]), Dl, Dr, Du, Dd, dnT(y),
                        ba_(y), bb_(y), X1, X2, Lt);
        {
          const Rl f = (Rl)ldexp(1.0, -dex[y]);
          for (int i = tid; i < ub_(y) * Dr * bb_(y); i += PEPS_NT) Lf[i] = Lt[i] * f;
        }
        __syncthreads();
      }

      // ---- two-row strip: vertical exchanges between rows x and x+1 ----
      if (kind == 0 && x < Lx - 1) {
        const bool has_dn2 = x + 1 < Lx - 1;
        const int sd2 = has_dn2 ? slot_bottom(L, x + 2) : -1;
        auto dn2 = [&](int y) -> const T* { return has_dn2 ? env_site(envs, L, sd2, y) : one; };
        auto ba2 = [&](int y) { return has_dn2 ? ed[(sd2 * Ly + y) * 3 + 0] : 1; };
        auto bb2 = [&](int y) { return has_dn2 ? ed[(sd2 * Ly + y) * 3 + 2] : 1; };
        if (tid == 0) Rt2[(size_t)Ly * box2] = T(1);
        __syncthreads();
        for (int y = Ly - 1; y >= 0; --y) {
          const int n1 = x * Ly + y, n2 = n1 + Ly;
          int Dl1, Dr1, Du1, Dd1, Dl2, Dr2, Du2, Dd2;
          legs_of(tab, L, n1, Dl1, Dr1, Du1, Dd1);
          legs_of(tab, L, n2, Dl2, Dr2, Du2, Dd2);
          T* Ry = Rt2 + (size_t)y * box2;
          s2_step_right<M>(Rt2 + (size_t)(y + 1) * box2, upT(y), ua_(y), uk_(y), ub_(y),
                           tens(n1, s[n1]), Dl1, Dr1, Dd1, tens(n2, s[n2]), Dl2, Dr2, Dd2, dn2(y),
                           ba2(y), bb2(y), Y1, Y2, Y3, Ry);
          const int cnt = ua_(y) * Dl1 * Dl2 * ba2(y);
          const int e = pow2_exponent((double)block_absmax(Ry, 1, cnt, cnt, red2));
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
          if (s[n1] != s[n2]) {
            T val[2];
            for (int which = 0; which < 2; ++which) {
              const int p1 = which ? s[n2] : s[n1];
              const int p2 = which ? s[n1] : s[n2];
              s2_step_left<M>(Lf2, upT(y), ua_(y), uk_(y), ub_(y), tens(n1, p1), Dl1, Dr1, Dd1,
                              tens(n2, p2), Dl2, Dr2, Dd2, dn2(y), ba2(y), bb2(y), Y1, Y2, Y3, Lu);
              const int cnt = ub_(y) * Dr1 * Dr2 * bb2(y);
              val[which] = lds_dot(Lu, (const T*)(Rt2 + (size_t)(y + 1) * box2), cnt, red2);
            }
            if (decide(x * (2 * Ly - 1) + Ly - 1 + y, sweep_ctr, ratio2(val[1], val[0]))) {
              if (tid == 0) {
                const uint8_t a = s[n1];
                s[n1] = s[n2];
                s[n2] = a;
                acc += 1;
              }
            }
            __syncthreads();
          }
          s2_step_left<M>(Lf2, upT(y), ua_(y), uk_(y), ub_(y), tens(n1, s[n1]), Dl1, Dr1, Dd1,
                          tens(n2, s[n2]), Dl2, Dr2, Dd2, dn2(y), ba2(y), bb2(y), Y1, Y2, Y3, Lu);
          const int cnt = ub_(y) * Dr1 * Dr2 * bb2(y);
          {
            const Rl f = (Rl)ldexp(1.0, -dex[y]);
            for (int i = tid; i < cnt; i += PEPS_NT) Lf2[i] = Lu[i] * f;
          }
          __syncthreads();
        }
      }

      // ---- absorb the updated row into the top environment ----
      if (x == 0) env_first_row<M>(L, tab, theta, s, false, envs, lg, sh, &fl);
      else if (x < Lx - 1)
        env_absorb_row<M>(L, tab, theta, s, false, x, envs, lg, R, sh, sel, sflag, &fl,
                          jac_sweeps);
    }
    if (sw >= burn_in && (sw - burn_in) % thin == thin - 1) {
      uint8_t* dst = samples + ((size_t)chain * per_chain + rec) * N;
      for (int n = tid; n < N; n += PEPS_NT) dst[n] = s[n];
      ++rec;
    }
    __syncthreads();
  }
  if (tid == 0 && accepted) accepted[chain] = acc;
}

size_t sample_lds_elems(int bmax, int D, int mode) {
  return sample_big(bmax, D, mode) + env_small_elems(bmax, D);
}
size_t sample_lds_bytes(int mode, const Lattice& L, bool gm) {
  return (gm ? env_small_elems(L.bmax, L.D) : sample_lds_elems(L.bmax, L.D, mode)) *
         mode_elem_bytes(mode);
}
size_t sample_slab_elems(const Lattice& L, int mode) {
  return (sample_big(L.bmax, L.D, mode) + 15) / 16 * 16;
}

template <int M>
hipError_t launch_metropolis(const Lattice& L, const int* tab, const void* theta, int kind,
                             int n_chains, int per_chain, int burn_in, int thin, uint64_t seed,
                             uint64_t offset, uint8_t* samples, int* accepted, void* envscr,
                             double* logscr, void* rscr, void* rt1, void* rt2, int jac_sweeps,
                             void* gws, hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const bool gm = gws != nullptr;
  const size_t lds = sample_lds_bytes(M, L, gm);
  const void* fn = gm ? (const void*)k_metropolis<M, true> : (const void*)k_metropolis<M, false>;
  hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  if (gm)
    hipLaunchKernelGGL((k_metropolis<M, true>), dim3(n_chains), dim3(env_threads(M)), lds, st, L,
                       tab, (const T*)theta, kind, n_chains, per_chain, burn_in, thin, k0, k1,
                       offset, samples, accepted, (T*)envscr, logscr, (T*)rscr, (T*)rt1, (T*)rt2,
                       jac_sweeps, (T*)gws, sample_slab_elems(L, M));
  else
    hipLaunchKernelGGL((k_metropolis<M, false>), dim3(n_chains), dim3(env_threads(M)), lds, st, L,
                       tab, (const T*)theta, kind, n_chains, per_chain, burn_in, thin, k0, k1,
                       offset, samples, accepted, (T*)envscr, logscr, (T*)rscr, (T*)rt1, (T*)rt2,
                       jac_sweeps, (T*)nullptr, (size_t)0);
  return hipGetLastError();
}

#define INST(M)                                                                                  \
  template hipError_t launch_metropolis<M>(const Lattice&, const int*, const void*, int, int,   \
                                           int, int, int, uint64_t, uint64_t, uint8_t*, int*,   \
                                           void*, double*, void*, void*, void*, int, void*,     \
                                           hipStream_t);
INST(MODE_F64)
INST(MODE_F32)
INST(MODE_BF16)
INST(MODE_C128)
INST(MODE_C64)
#undef INST

}  // namespace pm
