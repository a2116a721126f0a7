// Direct sampling of configurations (Sec. "On Direct Sampling"; App. "Direct
// sampling of PEPS", Eq. prob_from_cond_prob): rows are drawn from the top,
// each from its conditional density matrix
//   T^u_{S<i}[i] . D^l[i+1] . (T^u_{S<i}[i])^*,
// where T^u is the top boundary MPS E^u[i-1] of the rows already drawn times
// the open row i, and D^l[i+1] the boundary MPS of the double-layer network
// of the rows below (bond chi_d, computed once per tensor set by the
// environment kernel on the double-layer tensors built here).
//
// Per row and sample one workgroup forms the right environments of the row
// (physical legs traced), then walks the sites from the left: for p = 0, 1 it
// contracts the left environment with the column of site y at p and closes
// with the right environment, q_p; s_y = 0 iff u < q_0 / (q_0 + q_1), u from
// Philox4x32-10. Between rows the top environment absorbs the drawn row (one
// step of the environment sweep, the same code as the amplitude path).
//
// The column contractions are generic loops over output elements (one thread
// per element, the summed legs inside): they run in a per-sample global slab.
#include "common.h"
#include "env_dev.h"
#include "kernels.h"

namespace pm {

#define DIRECT_TAG 0x44495243u

// Double-layer parameters: slice p of site n of the D^2 lattice holds
// sum_q T[q] x conj(T[q]) with legs fused ket-major, (l l', r r', u u', d d')
// (both slices alike; the double-layer sweep reads slice 0). theta and dst
// are FP64, or interleaved FP64 pairs when cplx is set.
__global__ void k_double_theta(Lattice L, const int* __restrict__ tab, Lattice L2,
                               const int* __restrict__ tab2, const double* __restrict__ theta,
                               double* __restrict__ dst, int cplx_) {
  const int n = blockIdx.x;
  if (n >= L.N) return;
  const int* lg = tab + L.off_legs + 4 * n;
  const int Dl = lg[0], Dr = lg[1], Du = lg[2], Dd = lg[3];
  const int blk = tab[L.off_block + n], off = tab[L.off_param + n];
  const int blk2 = tab2[L2.off_block + n], off2 = tab2[L2.off_param + n];
  const int cnt = blk * blk;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    // i = ((((l l') r r') u u') d d') in the fused C order
    int q = i;
    const int d2 = q % Dd; q /= Dd;
    const int d1 = q % Dd; q /= Dd;
    const int u2 = q % Du; q /= Du;
    const int u1 = q % Du; q /= Du;
    const int r2 = q % Dr; q /= Dr;
    const int r1 = q % Dr; q /= Dr;
    const int l2 = q % Dl; q /= Dl;
    const int l1 = q;
    const int a = ((l1 * Dr + r1) * Du + u1) * Dd + d1;
    const int b = ((l2 * Dr + r2) * Du + u2) * Dd + d2;
    double re = 0.0, im = 0.0;
    for (int p = 0; p < 2; ++p) {
      if (cplx_) {
        const double ar = theta[2 * (off + p * blk + a)], ai = theta[2 * (off + p * blk + a) + 1];
        const double br = theta[2 * (off + p * blk + b)], bi = theta[2 * (off + p * blk + b) + 1];
        re += ar * br + ai * bi;  // a conj(b)
        im += ai * br - ar * bi;
      } else {
        re += theta[off + p * blk + a] * theta[off + p * blk + b];
      }
    }
    for (int p = 0; p < 2; ++p) {
      if (cplx_) {
        dst[2 * (off2 + p * blk2 + i)] = re;
        dst[2 * (off2 + p * blk2 + i) + 1] = im;
      } else {
        dst[off2 + p * blk2 + i] = re;
      }
    }
  }
}

// One step t of the top environment sweep (t = 0: the first row) for every
// sample: the rows above t are final, row t has just been drawn.
template <int M, bool GM>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_env_top_step(Lattice L, const int* __restrict__ tab,
               const typename ModeT<M>::T* __restrict__ theta, const uint8_t* __restrict__ samples,
               typename ModeT<M>::T* __restrict__ env, double* __restrict__ logs,
               typename ModeT<M>::T* __restrict__ rscr, int* __restrict__ flags, int n, int t,
               int jac_sweeps, typename ModeT<M>::T* __restrict__ gws, size_t slab) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int smp = blockIdx.x;
  if (smp >= n) return;
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* big = GM ? gws + (size_t)smp * slab : lds;
  T* small = GM ? lds : lds + env_big_elems(L.bmax, L.D, M);
  const EnvSmem<T> sh(big, small, L, tsqr_path(M, L.bmax, L.D) && PEPS_NT == 256);
  const int BD = L.bmax * L.D;
  __shared__ int sflag[2], fl;
  __shared__ int sel[256];
  if (threadIdx.x == 0) fl = 0;
  __syncthreads();
  const uint8_t* s = samples + (size_t)smp * L.N;
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  T* envs = env + (size_t)smp * L.n_slots * slot_elems;
  double* lg = logs + (size_t)smp * L.n_slots;
  T* R = rscr + (size_t)smp * (size_t)L.Ly * BD * BD;
  if (t == 0)
    env_first_row<M>(L, tab, theta, s, false, envs, lg, sh, &fl);
  else
    env_absorb_row<M>(L, tab, theta, s, false, t, envs, lg, R, sh, sel, sflag, &fl, jac_sweeps);
  if (threadIdx.x == 0 && fl && flags) atomicOr(flags + smp, fl);
}

// Per-sample slab of the row kernel, in elements: right environments of the
// Ly + 1 column boundaries, the left environment and the two candidates,
// and two ping-pong buffers for the intermediate tensors.
__host__ __device__ inline size_t direct_env_elems(int B, int D, int Bd) {
  return (size_t)B * D * Bd * D * B;
}
__host__ __device__ inline size_t direct_tmp_elems(int B, int D, int Bd) {
  return (size_t)2 * B * B * D * D * D * Bd;
}
size_t direct_slab_elems(const Lattice& L, const Lattice& L2) {
  const size_t RS = direct_env_elems(L.bmax, L.D, L2.bmax);
  const size_t TM = direct_tmp_elems(L.bmax, L.D, L2.bmax);
  return ((L.Ly + 4) * RS + 2 * TM + 15) / 16 * 16;
}

template <int M>
__device__ __forceinline__ typename ModeT<M>::T dld(const typename ModeT<M>::T* p, size_t i) {
  return opnd<M>(p[i]);
}

// Draw row i of every sample. env: the samples' environment caches (top
// slots 0..i-1 final); env2/L2/tab2: the double-layer environments (one
// sample); logp accumulates ln p(S_i | S_<i).
template <int M>
__global__ void __launch_bounds__(256)
k_direct_row(Lattice L, const int* __restrict__ tab,
             const typename ModeT<M>::T* __restrict__ theta,
             const typename ModeT<M>::T* __restrict__ env, Lattice L2,
             const int* __restrict__ tab2, const typename ModeT<M>::T* __restrict__ env2,
             uint8_t* __restrict__ samples, double* __restrict__ logp, int* __restrict__ flags,
             int n, int i, uint32_t k0, uint32_t k1, uint64_t offset,
             typename ModeT<M>::T* __restrict__ slab, size_t slab_elems) {
  typedef typename ModeT<M>::T T;
  __shared__ T red[8];
  __shared__ double dred[8];
  // the column's small tensors, read in every inner sum, staged in LDS:
  // E (<= B D B), T[0], T[1] (<= D^4 each), D^l (<= Bd D^2 Bd)
  extern __shared__ __align__(16) unsigned char dsm[];
  T* sE = reinterpret_cast<T*>(dsm);
  T* sT0 = sE + L.bmax * L.D * L.bmax;
  T* sT1 = sT0 + L.D * L.D * L.D * L.D;
  T* sG = sT1 + L.D * L.D * L.D * L.D;
  const int smp = blockIdx.x;
  if (smp >= n) return;
  const int tid = threadIdx.x, NT = blockDim.x;
  const int Ly = L.Ly;
  const size_t RS = direct_env_elems(L.bmax, L.D, L2.bmax);
  const size_t TM = direct_tmp_elems(L.bmax, L.D, L2.bmax);
  T* base = slab + (size_t)smp * slab_elems;
  T* Rb = base;                      // (Ly + 1) x RS
  T* Lc = Rb + (size_t)(Ly + 1) * RS;
  T* Cp[2] = {Lc + RS, Lc + 2 * RS};
  T* Ta = Lc + 3 * RS;
  T* Tb = Ta + TM;
  uint8_t* s = samples + (size_t)smp * L.N;
  const size_t slot_elems = (size_t)Ly * L.site_box;
  const T* envs = env + (size_t)smp * L.n_slots * slot_elems;
  const int* ed = tab + L.off_env;
  const size_t slot2_elems = (size_t)Ly * L2.site_box;
  const int* ed2 = tab2 + L2.off_env;
  const int su = i - 1;               // top slot of E^u[i-1]
  const int sb2 = L2.Lx - 1 + i;      // bottom slot of D^l[i+1] (= slot_bottom(i + 1))
  const bool has_e = i > 0, has_d = i < L.Lx - 1;
  const T one = T(1);
  int fl = 0;
  double lp = 0.0;

  // dims and pointers of the column at site y
  struct Col {
    int ea, eu, eb, Dl, Dr, Du, Dd, ga, gb;
    const T* E;
    const T* Tp0;
    const T* Tp1;
    const T* G;
  };
  auto col = [&](int y) {
    Col c;
    const int nsite = i * Ly + y;
    const int* lg = tab + L.off_legs + 4 * nsite;
    c.Dl = lg[0]; c.Dr = lg[1]; c.Du = lg[2]; c.Dd = lg[3];
    const T* tp = theta + tab[L.off_param + nsite];
    c.Tp0 = tp;
    c.Tp1 = tp + tab[L.off_block + nsite];
    if (has_e) {
      c.E = envs + (size_t)su * slot_elems + (size_t)y * L.site_box;
      c.ea = ed[(su * Ly + y) * 3 + 0];
      c.eu = ed[(su * Ly + y) * 3 + 1];
      c.eb = ed[(su * Ly + y) * 3 + 2];
    } else {
      c.E = &one; c.ea = 1; c.eu = 1; c.eb = 1;
    }
    if (has_d) {
      c.G = env2 + (size_t)sb2 * slot2_elems + (size_t)y * L2.site_box;
      c.ga = ed2[(sb2 * Ly + y) * 3 + 0];
      c.gb = ed2[(sb2 * Ly + y) * 3 + 2];
    } else {
      c.G = &one; c.ga = 1; c.gb = 1;
    }
    return c;
  };
  // copy the column's tensors to LDS and point the column at the copies
  // (callers have passed a barrier since the previous column's last read)
  auto stage = [&](Col& c) {
    const int ne = c.ea * c.eu * c.eb, nt = c.Dl * c.Dr * c.Du * c.Dd;
    const int ng = c.ga * c.Dd * c.Dd * c.gb;
    for (int q = tid; q < ne; q += NT) sE[q] = c.E[q];
    for (int q = tid; q < nt; q += NT) {
      sT0[q] = c.Tp0[q];
      sT1[q] = c.Tp1[q];
    }
    for (int q = tid; q < ng; q += NT) sG[q] = c.G[q];
    __syncthreads();
    c.E = sE;
    c.Tp0 = sT0;
    c.Tp1 = sT1;
    c.G = sG;
  };

  // ---- right environments R_y (sites y.. with their physical legs traced)
  if (tid == 0) Rb[(size_t)Ly * RS] = T(1);
  __syncthreads();
  for (int y = Ly - 1; y >= 0; --y) {
    Col c = col(y);
    stage(c);
    const int ea = c.ea, eu = c.eu, eb = c.eb, Dl = c.Dl, Dr = c.Dr, Du = c.Du, Dd = c.Dd;
    const int ga = c.ga, gb = c.gb;
    const T* R1 = Rb + (size_t)(y + 1) * RS;
    T* Ry = Rb + (size_t)y * RS;
    // Y1[e,u,r,g,s,k] = sum_f E[e,u,f] R1[f,r,g,s,k]
    {
      const int n1 = ea * Du * Dr * gb * Dr * eb;
      const int tail = Dr * gb * Dr * eb;
      for (int o = tid; o < n1; o += NT) {
        const int e = o / (Du * tail), rem = o - e * (Du * tail);
        const int u = rem / tail, rk = rem - u * tail;
        T acc = 0;
        for (int f = 0; f < eb; ++f)
          acc += dld<M>(c.E, (size_t)(e * eu + u) * eb + f) * dld<M>(R1, (size_t)f * tail + rk);
        Ta[o] = acc;
      }
    }
    __syncthreads();
    // Y2[e,l,d,p,g,s,k] = sum_{u,r} T[p,l,r,u,d] Y1[e,u,r,g,s,k]
    {
      const int gsk = gb * Dr * eb;
      const int n2 = ea * Dl * Dd * 2 * gsk;
      for (int o = tid; o < n2; o += NT) {
        int q = o;
        const int x = q % gsk; q /= gsk;
        const int p = q % 2; q /= 2;
        const int d = q % Dd; q /= Dd;
        const int l = q % Dl; q /= Dl;
        const int e = q;
        const T* tp = p ? c.Tp1 : c.Tp0;
        T acc = 0;
        for (int u = 0; u < Du; ++u)
          for (int r = 0; r < Dr; ++r)
            acc += dld<M>(tp, (size_t)((l * Dr + r) * Du + u) * Dd + d) *
                   dld<M>(Ta, ((size_t)(e * Du + u) * Dr + r) * gsk + x);
        Tb[o] = acc;
      }
    }
    __syncthreads();
    // Y3[e,l,p,b,w,s,k] = sum_{d,g} G[b,(d,w),g] Y2[e,l,d,p,g,s,k]
    {
      const int sk = Dr * eb;
      const int n3 = ea * Dl * 2 * ga * Dd * sk;
      const int gk = Dd * Dd;
      for (int o = tid; o < n3; o += NT) {
        int q = o;
        const int x = q % sk; q /= sk;
        const int w = q % Dd; q /= Dd;
        const int b = q % ga; q /= ga;
        const int p = q % 2; q /= 2;
        const int el = q;  // e * Dl + l
        T acc = 0;
        for (int d = 0; d < Dd; ++d)
          for (int g = 0; g < gb; ++g)
            acc += dld<M>(c.G, (size_t)(b * gk + d * Dd + w) * gb + g) *
                   dld<M>(Tb, ((((size_t)el * Dd + d) * 2 + p) * gb + g) * sk + x);
        Ta[o] = acc;
      }
    }
    __syncthreads();
    // Y4[e,l,b,m,v,k] = sum_{p,w,s} conj T[p,m,s,v,w] Y3[e,l,p,b,w,s,k]
    {
      const int n4 = ea * Dl * ga * Dl * Du * eb;
      for (int o = tid; o < n4; o += NT) {
        int q = o;
        const int k = q % eb; q /= eb;
        const int v = q % Du; q /= Du;
        const int m = q % Dl; q /= Dl;
        const int b = q % ga; q /= ga;
        const int el = q;
        T acc = 0;
        for (int p = 0; p < 2; ++p) {
          const T* tp = p ? c.Tp1 : c.Tp0;
          for (int w = 0; w < Dd; ++w)
            for (int ss = 0; ss < Dr; ++ss)
              acc += conjx(dld<M>(tp, (size_t)((m * Dr + ss) * Du + v) * Dd + w)) *
                     dld<M>(Ta, (((((size_t)el * 2 + p) * ga + b) * Dd + w) * Dr + ss) * eb + k);
        }
        Tb[o] = acc;
      }
    }
    __syncthreads();
    // R_y[e,l,b,m,h] = sum_{v,k} conj E[h,v,k] Y4[e,l,b,m,v,k]
    {
      const int n5 = ea * Dl * ga * Dl * ea;
      for (int o = tid; o < n5; o += NT) {
        const int h = o % ea, elbm = o / ea;
        T acc = 0;
        for (int v = 0; v < Du; ++v)
          for (int k = 0; k < eb; ++k)
            acc += conjx(dld<M>(c.E, (size_t)(h * eu + v) * eb + k)) *
                   dld<M>(Tb, ((size_t)elbm * Du + v) * eb + k);
        Ry[o] = acc;
      }
      __syncthreads();
      const int ex = pow2_exponent((double)block_absmax(Ry, 1, n5, n5, red));
      scale_pow2(Ry, n5, ex);
      __syncthreads();
    }
  }

  // ---- left to right: draw the sites
  if (tid == 0) Lc[0] = T(1);
  __syncthreads();
  for (int y = 0; y < Ly; ++y) {
    Col c = col(y);
    stage(c);
    const int ea = c.ea, eu = c.eu, eb = c.eb, Dl = c.Dl, Dr = c.Dr, Du = c.Du, Dd = c.Dd;
    const int ga = c.ga, gb = c.gb;
    const T* R1 = Rb + (size_t)(y + 1) * RS;
    // X1[l,b,m,h,u,f] = sum_e Lc[e,l,b,m,h] E[e,u,f]  (common to both p)
    const int lbmh = Dl * ga * Dl * ea;
    {
      const int n1 = lbmh * Du * eb;
      for (int o = tid; o < n1; o += NT) {
        const int uf = o % (Du * eb), x = o / (Du * eb);
        T acc = 0;
        for (int e = 0; e < ea; ++e)
          acc += dld<M>(Lc, (size_t)e * lbmh + x) * dld<M>(c.E, (size_t)e * eu * eb + uf);
        Ta[o] = acc;
      }
    }
    __syncthreads();
    double q[2];
    const int nc = eb * Dr * gb * Dr * eb;
    for (int p = 0; p < 2; ++p) {
      const T* tp = p ? c.Tp1 : c.Tp0;
      T* X2 = Tb;
      T* X3 = Tb + TM / 2;
      // X2[b,m,h,f,r,d] = sum_{l,u} X1[l,b,m,h,u,f] T[p,l,r,u,d]
      {
        const int bmh = ga * Dl * ea;
        const int n2 = bmh * eb * Dr * Dd;
        for (int o = tid; o < n2; o += NT) {
          int qq = o;
          const int d = qq % Dd; qq /= Dd;
          const int r = qq % Dr; qq /= Dr;
          const int f = qq % eb; qq /= eb;
          const int x = qq;  // (b, m, h)
          T acc = 0;
          for (int l = 0; l < Dl; ++l)
            for (int u = 0; u < Du; ++u)
              acc += dld<M>(Ta, (((size_t)l * bmh + x) * Du + u) * eb + f) *
                     dld<M>(tp, (size_t)((l * Dr + r) * Du + u) * Dd + d);
          X2[o] = acc;
        }
      }
      __syncthreads();
      // X3[m,h,f,r,g,w] = sum_{b,d} X2[b,m,h,f,r,d] G[b,(d,w),g]
      {
        const int mhfr = Dl * ea * eb * Dr;
        const int n3 = mhfr * gb * Dd;
        const int gk = Dd * Dd;
        for (int o = tid; o < n3; o += NT) {
          const int w = o % Dd, g = (o / Dd) % gb, x = o / (Dd * gb);
          T acc = 0;
          for (int b = 0; b < ga; ++b)
            for (int d = 0; d < Dd; ++d)
              acc += dld<M>(X2, ((size_t)b * mhfr + x) * Dd + d) *
                     dld<M>(c.G, (size_t)(b * gk + d * Dd + w) * gb + g);
          X3[o] = acc;
        }
      }
      __syncthreads();
      // X4[h,f,r,g,s,v] = sum_{m,w} X3[m,h,f,r,g,w] conj T[p,m,s,v,w]
      T* X4 = X2;
      {
        const int hfrg = ea * eb * Dr * gb;
        const int n4 = hfrg * Dr * Du;
        for (int o = tid; o < n4; o += NT) {
          const int v = o % Du, ss = (o / Du) % Dr, x = o / (Du * Dr);
          T acc = 0;
          for (int m = 0; m < Dl; ++m)
            for (int w = 0; w < Dd; ++w)
              acc += dld<M>(X3, ((size_t)m * hfrg + x) * Dd + w) *
                     conjx(dld<M>(tp, (size_t)((m * Dr + ss) * Du + v) * Dd + w));
          X4[o] = acc;
        }
      }
      __syncthreads();
      // C_p[f,r,g,s,k] = sum_{h,v} X4[h,f,r,g,s,v] conj E[h,v,k]; q_p = C_p . R_{y+1}
      {
        const int frgs = eb * Dr * gb * Dr;
        double part = 0.0;
        for (int o = tid; o < nc; o += NT) {
          const int k = o % eb, x = o / eb;
          T acc = 0;
          for (int h = 0; h < ea; ++h)
            for (int v = 0; v < Du; ++v)
              acc += dld<M>(X4, ((size_t)h * frgs + x) * Du + v) *
                     conjx(dld<M>(c.E, (size_t)(h * eu + v) * eb + k));
          Cp[p][o] = acc;
          part += (double)realx(acc * R1[o]);
        }
        q[p] = block_sum(part, dred);
      }
      __syncthreads();
    }
    // conditional of site y and the draw
    const int nsite = i * Ly + y;
    const uint64_t j = offset + (uint64_t)smp;
    const u4 ctr = {(uint32_t)nsite, (uint32_t)j, (uint32_t)(j >> 32), DIRECT_TAG};
    const u4 rr = philox(ctr, k0, k1);
    const double u = philox_uniform(rr.x, rr.y);
    const double q0 = q[0] > 0.0 ? q[0] : 0.0, q1 = q[1] > 0.0 ? q[1] : 0.0;
    const double tot = q0 + q1;
    if (!(isfinite(q[0]) && isfinite(q[1]))) fl |= 2;
    else if (!(tot > 0.0)) fl |= 1;
    const double p0 = (tot > 0.0 && isfinite(tot)) ? q0 / tot : 0.5;
    const int bsel = u < p0 ? 0 : 1;
    const double pb = bsel == 0 ? p0 : 1.0 - p0;
    lp += log(pb);
    if (tid == 0) s[nsite] = (uint8_t)bsel;
    // the left environment moves past site y with the drawn value
    {
      const T* src = Cp[bsel];
      for (int o = tid; o < nc; o += NT) Lc[o] = src[o];
      __syncthreads();
      const int ex = pow2_exponent((double)block_absmax(Lc, 1, nc, nc, red));
      scale_pow2(Lc, nc, ex);
      __syncthreads();
    }
  }
  if (tid == 0) {
    logp[smp] += lp;
    if (fl && flags) flags[smp] |= fl;
  }
}

// ln w = ln|Psi(S)|^2 - ln p(S) (unnormalised importance weight); the
// amplitude's flags are ORed into the sample's.
__global__ void k_direct_logw(int n, const double* __restrict__ lpsi,
                              const double* __restrict__ logp, const int* __restrict__ afl,
                              double* __restrict__ logw, int* __restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (logw) logw[i] = 2.0 * lpsi[2 * i] - logp[i];
  if (flags) flags[i] |= afl[i];
}

hipError_t launch_direct_logw(int n, const double* lpsi, const double* logp, const int* afl,
                              double* logw, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_direct_logw, dim3((n + 255) / 256), dim3(256), 0, st, n, lpsi, logp, afl,
                     logw, flags);
  return hipGetLastError();
}

template <int M>
hipError_t launch_direct_row(const Lattice& L, const int* tab, const void* theta, const void* env,
                             const Lattice& L2, const int* tab2, const void* env2,
                             uint8_t* samples, double* logp, int* flags, int n, int i,
                             uint64_t seed, uint64_t offset, void* slab, hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const size_t D4 = (size_t)L.D * L.D * L.D * L.D;
  const size_t lds = ((size_t)L.bmax * L.D * L.bmax + 2 * D4 +
                      (size_t)L2.bmax * L.D * L.D * L2.bmax) * sizeof(T);
  const hipError_t e = hipFuncSetAttribute((const void*)k_direct_row<M>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_direct_row<M>, dim3(n), dim3(256), lds, st, L, tab, (const T*)theta,
                     (const T*)env, L2, tab2, (const T*)env2, samples, logp, flags, n, i, k0, k1,
                     offset, (T*)slab, direct_slab_elems(L, L2));
  return hipGetLastError();
}

template <int M>
hipError_t launch_env_top_step(const Lattice& L, const int* tab, const void* theta,
                               const uint8_t* samples, void* env, double* logs, void* rscr,
                               int* flags, int n, int t, int jac_sweeps, void* gws,
                               hipStream_t st) {
  typedef typename ModeT<M>::T T;
  if (gws) {
    const size_t lds = env_lds_bytes(M, L, true);
    hipFuncSetAttribute((const void*)k_env_top_step<M, true>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_env_top_step<M, true>), dim3(n), dim3(env_threads(M)), lds, st, L,
                       tab, (const T*)theta, samples, (T*)env, logs, (T*)rscr, flags, n, t,
                       jac_sweeps, (T*)gws, env_slab_elems(L, M));
  } else {
    const size_t lds = env_lds_bytes(M, L, false);
    hipFuncSetAttribute((const void*)k_env_top_step<M, false>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_env_top_step<M, false>), dim3(n), dim3(env_threads(M)), lds, st, L,
                       tab, (const T*)theta, samples, (T*)env, logs, (T*)rscr, flags, n, t,
                       jac_sweeps, (T*)nullptr, (size_t)0);
  }
  return hipGetLastError();
}

hipError_t launch_double_theta(const Lattice& L, const int* tab, const Lattice& L2,
                               const int* tab2, const double* theta, double* dst, bool cplx_,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_double_theta, dim3(L.N), dim3(256), 0, st, L, tab, L2, tab2, theta, dst,
                     cplx_ ? 1 : 0);
  return hipGetLastError();
}

#define INST(M)                                                                                  \
  template hipError_t launch_direct_row<M>(const Lattice&, const int*, const void*, const void*, \
                                           const Lattice&, const int*, const void*, uint8_t*,    \
                                           double*, int*, int, int, uint64_t, uint64_t, void*,   \
                                           hipStream_t);                                         \
  template hipError_t launch_env_top_step<M>(const Lattice&, const int*, const void*,            \
                                             const uint8_t*, void*, double*, void*, int*, int,   \
                                             int, int, void*, hipStream_t);
INST(MODE_F64)
INST(MODE_F32)
INST(MODE_BF16)
INST(MODE_C128)
INST(MODE_C64)
#undef INST

}  // namespace pm
