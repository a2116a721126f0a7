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
// Complex parameters (complex modes) take the same steps with the Hermitian
// forms: a_s = sum_k O_sk conj(m_k), G = O O^H, T = L L^H and
// dtheta = Obar^H y; the scalar type S is double or cplx<double>.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace pm {

// FP64 scalar of the solve for an O element type
template <typename TO> struct SolveT { typedef double type; };
template <typename R> struct SolveT<cplx<R>> { typedef cplx<double> type; };

__device__ __forceinline__ double to_s(float v) { return (double)v; }
__device__ __forceinline__ double to_s(double v) { return v; }
template <typename R>
__device__ __forceinline__ cplx<double> to_s(cplx<R> v) {
  return cplx<double>((double)v.re, (double)v.im);
}

// dtheta / mean entries are (re, im) pairs for complex parameters
__device__ __forceinline__ void put(double* out, size_t k, double v) { out[k] = v; }
__device__ __forceinline__ void put(double* out, size_t k, cplx<double> v) {
  out[2 * k] = v.re;
  out[2 * k + 1] = v.im;
}

// m_k for every parameter k; one thread per compact index.
template <typename TO>
__global__ void k_colmean(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
                          const uint8_t* __restrict__ samples, int n,
                          typename SolveT<TO>::type* __restrict__ mean) {
  typedef typename SolveT<TO>::type S;
  const int jc = blockIdx.x * blockDim.x + threadIdx.x;
  if (jc >= L.n_compact) return;
  const int site = tab[L.off_csite + jc];
  const int j = jc - tab[L.off_compact + site];
  S acc0 = 0.0, acc1 = 0.0;
  for (int s = 0; s < n; ++s) {
    const S v = to_s(O[(size_t)s * L.n_compact + jc]);
    if (pbit(samples[(size_t)s * L.N + site])) acc1 += v;
    else acc0 += v;
  }
  const int off = tab[L.off_param + site], blk = tab[L.off_block + site];
  mean[off + j] = acc0 / (double)n;
  mean[off + blk + j] = acc1 / (double)n;
}

// a_s = sum_k O_sk conj(m_k) (block per sample); slot n holds |m|^2 (block n).
template <typename TO>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_proj_mean(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
            const uint8_t* __restrict__ samples, int n,
            const typename SolveT<TO>::type* __restrict__ mean,
            typename SolveT<TO>::type* __restrict__ a) {
  typedef typename SolveT<TO>::type S;
  __shared__ S red[8];
  const int s = blockIdx.x;
  S acc = 0.0;
  if (s < n) {
    for (int jc = threadIdx.x; jc < L.n_compact; jc += PEPS_NT) {
      const int site = tab[L.off_csite + jc];
      const int j = jc - tab[L.off_compact + site];
      const int p = pbit(samples[(size_t)s * L.N + site]);
      acc += to_s(O[(size_t)s * L.n_compact + jc]) *
             conjx(mean[tab[L.off_param + site] + p * tab[L.off_block + site] + j]);
    }
  } else {
    for (int k = threadIdx.x; k < L.n_params; k += PEPS_NT) acc += S(abs2x(mean[k]));
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) a[s] = acc;
}

// E statistics: ws[0] = mean Re E, ws[8] = mean Im E (complex parameters
// only; real ones use Re E), ws[1] = mean |E - <E>|^2.
template <bool CPLX>
__global__ void k_estats(const double* __restrict__ eloc, int n, double* __restrict__ ws,
                         int* __restrict__ bad) {
  __shared__ double red[8];
  double s = 0.0, si = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) {
    const double v = eloc[2 * i];
    if (!isfinite(v) || !isfinite(eloc[2 * i + 1])) atomicOr(bad, 1);
    s += v;
    if (CPLX) si += eloc[2 * i + 1];
  }
  s = block_sum(s, red);
  const double mu = s / n;
  double mi = 0.0;
  if (CPLX) mi = block_sum(si, red) / n;
  double q = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) {
    const double v = eloc[2 * i] - mu;
    q += v * v;
    if (CPLX) {
      const double w = eloc[2 * i + 1] - mi;
      q += w * w;
    }
  }
  q = block_sum(q, red);
  if (threadIdx.x == 0) {
    ws[0] = mu;
    ws[1] = q / n;
    ws[8] = mi;
  }
}

// ---- FP64 matrix-core tiles of the Hermitian products --------------------
// A workgroup of four waves forms one 64 x 64 tile of C = A B^H, where the
// rows of A and B are samples (the Gram) or rows of the Cholesky panel (the
// trailing update); each wave owns a 32 x 32 block of 2 x 2 MFMA tiles.
// Operands pass through LDS in chunks of HKC columns stored k-major,
// [k][row], the layout in which 16 consecutive lanes read 16 rows of one k.
// A complex product takes three real ones: with B' = conj(B),
// P1 = Re A Re B', P2 = Im A Im B', P3 = (Re A + Im A)(Re B' + Im B'),
// Re C = P1 - P2 and Im C = P3 - P1 - P2.
#define HT 64
#define HKC 16
#define HLS (HT + 2)

template <bool CX> struct HStage {
  static constexpr int NP = CX ? 3 : 1;
  double a[NP][HKC][HLS];
  double b[NP][HKC][HLS];
};

// Partial products of one wave: p[component][row tile][column tile]
template <bool CX> struct HPart {
  static constexpr int NP = CX ? 3 : 1;
  mf64x4 p[NP][2][2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) p[c][i][j] = mf64x4{0.0, 0.0, 0.0, 0.0};
  }
};

// element (k, r) of the staged A (isb = false) or of conj(B) (isb = true)
template <bool CX>
__device__ __forceinline__ void hput(HStage<CX>& sh, bool isb, int k, int r, double re,
                                     double im) {
  double (*d)[HKC][HLS] = isb ? sh.b : sh.a;
  d[0][k][r] = re;
  if constexpr (CX) {
    if (isb) im = -im;
    d[1][k][r] = im;
    d[2][k][r] = re + im;
  }
}

// accumulate kc4 (a multiple of 4) staged columns into the wave's partials
template <bool CX>
__device__ __forceinline__ void hchunk(const HStage<CX>& sh, HPart<CX>& acc, int kc4, int lane,
                                       int wr, int wc) {
  constexpr int NP = HStage<CX>::NP;
  const int lr = lane & 15, lk = lane >> 4;
  for (int kq = 0; kq < kc4; kq += 4) {
    double av[NP][2], bv[NP][2];
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[c][t] = sh.a[c][kq + lk][32 * wr + 16 * t + lr];
        bv[c][t] = sh.b[c][kq + lk][32 * wc + 16 * t + lr];
      }
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc.p[c][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[c][i], bv[c][j],
                                                                acc.p[c][i][j], 0, 0, 0);
  }
}

// value v (0..3) of tile (i, j) of the wave's partials as the scalar S
template <typename S, bool CX>
__device__ __forceinline__ S hval(const HPart<CX>& acc, int i, int j, int v) {
  if constexpr (CX) {
    const double p1 = acc.p[0][i][j][v], p2 = acc.p[1][i][j][v], p3 = acc.p[2][i][j][v];
    return S(p1 - p2, p3 - p1 - p2);
  } else {
    return acc.p[0][i][j][v];
  }
}

// lower-triangle tile t -> (bi, bj), bj <= bi; blocks are dealt out so that
// each XCD (blocks b, b + 8, ...) takes a contiguous range of tiles, which
// share operand rows in its L2
__device__ __forceinline__ bool tri_tile(int ntiles, int& bi, int& bj) {
  const int per = gridDim.x >> 3;
  const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (t >= ntiles) return false;
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  bi = i;
  bj = t - i * (i + 1) / 2;
  return true;
}

static unsigned tri_grid(int nt) {
  const unsigned ntiles = (unsigned)nt * (unsigned)(nt + 1) / 2;
  return (ntiles + 7u) & ~7u;
}

// Masked Gram G[s,s'] = sum_k O_sk conj(O_s'k) over compact columns: the
// parameters of site (x, y) are shared by two samples only when their
// physical indices there agree, so each site's columns are accumulated
// apart and added where the two bits agree (the bits of the tile's 64 rows
// at every site are packed into one 64-bit word per site in LDS). Chunks of
// HKC columns of one site are double-buffered in LDS, holding (Re, Im) of A
// and of conj(B); the next chunk is loaded into registers before the
// current one is multiplied, so one barrier per chunk remains. Written with
// the centring and eps already applied:
// T = (G - a_s - conj(a_s') + |m|^2)/n + eps delta, both triangles.
template <bool CX> struct GStage {
  static constexpr int NC = CX ? 2 : 1;
  double v[2][2][NC][HKC][HLS];  // [buffer][A, conj B][Re, Im][k][row]
};

template <typename TO>
__global__ void __launch_bounds__(256)
k_gram(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
       const uint8_t* __restrict__ samples, int n, const typename SolveT<TO>::type* __restrict__ a,
       double eps, typename SolveT<TO>::type* __restrict__ Tm, int ntiles,
       const int* __restrict__ run_if) {
  typedef typename SolveT<TO>::type S;
  constexpr bool CX = IsCplx<TO>::value;
  constexpr int NP = CX ? 3 : 1, NE = HT * HKC / 256;
  if (run_if && !*run_if) return;
  __shared__ GStage<CX> sh;
  extern __shared__ unsigned long long bits[];  // [site][A rows, B rows]
  int bi, bj;
  if (!tri_tile(ntiles, bi, bj)) return;
  const int s0 = bi * HT, t0 = bj * HT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const size_t nc = (size_t)L.n_compact;
  // physical bits of the 64 A rows and 64 B rows at every site
  for (int site = w; site < L.N; site += 4) {
    const int ra = s0 + lane, rb = t0 + lane;
    const int ba = ra < n ? pbit(samples[(size_t)ra * L.N + site]) : 0;
    const int bb = rb < n ? pbit(samples[(size_t)rb * L.N + site]) : 0;
    const unsigned long long ma = __ballot(ba), mb = __ballot(bb);
    if (lane == 0) {
      bits[2 * site] = ma;
      bits[2 * site + 1] = mb;
    }
  }
  // chunk loader: element u of this thread is (row e / HKC, column e % HKC)
  TO ra[NE], rb[NE];
  auto load = [&](int site, int k0) {
    const int c0 = tab[L.off_compact + site], kc = min(HKC, tab[L.off_block + site] - k0);
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + 256 * u, r = e / HKC, k = e - r * HKC;
      const size_t col = (size_t)c0 + k0 + k;
      ra[u] = (k < kc && s0 + r < n) ? O[(size_t)(s0 + r) * nc + col] : TO(0);
      rb[u] = (k < kc && t0 + r < n) ? O[(size_t)(t0 + r) * nc + col] : TO(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + 256 * u, r = e / HKC, k = e - r * HKC;
      double re, im;
      split(to_s(ra[u]), re, im);
      sh.v[buf][0][0][k][r] = re;
      if constexpr (CX) sh.v[buf][0][1][k][r] = im;
      split(to_s(rb[u]), re, im);
      sh.v[buf][1][0][k][r] = re;
      if constexpr (CX) sh.v[buf][1][1][k][r] = -im;
    }
  };
  mf64x4 tot[2][2][CX ? 2 : 1];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int c = 0; c < (CX ? 2 : 1); ++c) tot[i][j][c] = mf64x4{0.0, 0.0, 0.0, 0.0};
  HPart<CX> cur;
  cur.zero();
  int site = 0, k0 = 0;
  load(0, 0);
  store(0);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int buf = 0;; buf ^= 1) {
    const int nbk = tab[L.off_block + site];
    const int kc4 = (min(HKC, nbk - k0) + 3) & ~3;
    // the chunk after this one
    int nsite = site, nk0 = k0 + HKC;
    if (nk0 >= nbk) {
      ++nsite;
      nk0 = 0;
    }
    const bool more = nsite < L.N;
    if (more) load(nsite, nk0);
    for (int kq = 0; kq < kc4; kq += 4) {
      double av[NP][2], bv[NP][2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[0][t] = sh.v[buf][0][0][kq + lk][32 * wr + 16 * t + lr];
        bv[0][t] = sh.v[buf][1][0][kq + lk][32 * wc + 16 * t + lr];
        if constexpr (CX) {
          av[1][t] = sh.v[buf][0][1][kq + lk][32 * wr + 16 * t + lr];
          bv[1][t] = sh.v[buf][1][1][kq + lk][32 * wc + 16 * t + lr];
          av[2][t] = av[0][t] + av[1][t];
          bv[2][t] = bv[0][t] + bv[1][t];
        }
      }
#pragma unroll
      for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            cur.p[c][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[c][i], bv[c][j],
                                                                  cur.p[c][i][j], 0, 0, 0);
    }
    if (nsite != site) {
      // add this site's products where the two samples share its parameters
      const unsigned long long ma = bits[2 * site], mb = bits[2 * site + 1];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = 32 * wc + 16 * j + lr;
          const int pb = (int)((mb >> col) & 1ull);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 32 * wr + 16 * i + 4 * v + lk;
            if ((int)((ma >> row) & 1ull) == pb) {
              double gr, gi;
              split(hval<S, CX>(cur, i, j, v), gr, gi);
              tot[i][j][0][v] += gr;
              if constexpr (CX) tot[i][j][1][v] += gi;
            }
          }
        }
      cur.zero();
    }
    if (!more) break;
    store(buf ^ 1);
    __syncthreads();
    site = nsite;
    k0 = nk0;
  }
  const S m2 = a[n];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int t = t0 + 32 * wc + 16 * j + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int s = s0 + 32 * wr + 16 * i + 4 * v + lk;
        if (s < n && t < n && t <= s) {
          S g;
          if constexpr (CX) g = S(tot[i][j][0][v], tot[i][j][1][v]);
          else g = tot[i][j][0][v];
          S val = (g - a[s] - conjx(a[t]) + m2) / (double)n;
          if (s == t) {
            val += S(eps);
            if constexpr (IsCplx<S>::value) val.im = 0.0;  // Hermitian diagonal
          }
          Tm[(size_t)s * n + t] = val;
          Tm[(size_t)t * n + s] = conjx(val);
        }
      }
    }
}

// trace of T (before eps) into ws[2]
template <typename S>
__global__ void k_trace(const S* __restrict__ Tm, int n, double eps, double* __restrict__ ws) {
  __shared__ double red[8];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) s += realx(Tm[(size_t)i * n + i]) - eps;
  s = block_sum(s, red);
  if (threadIdx.x == 0) ws[2] = s;
}

// ---- blocked Cholesky T = L L^H, lower, in place on the full matrix ----
#define CB 64
// factor the diagonal block kb (one block of 256 threads, in LDS)
template <typename S>
__global__ void __launch_bounds__(256) k_chol_diag(S* __restrict__ A, int n, int kb,
                                                   double* __restrict__ ws) {
  __shared__ S Sd[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = (n - k0) < CB ? (n - k0) : CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    Sd[i][j] = A[(size_t)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    __shared__ double piv;
    if (tid == 0) {
      double d = realx(Sd[j][j]);
      if (!(d > 0.0)) {
        ws[4] = 1.0;  // not positive definite
        d = 1e-300;
      }
      piv = sqrt(d);
      if (piv < ws[5]) ws[5] = piv;
      Sd[j][j] = S(piv);
    }
    __syncthreads();
    const double ip = 1.0 / piv;
    for (int i = j + 1 + tid; i < nb; i += 256) {
      if constexpr (IsCplx<S>::value) Sd[i][j] = Sd[i][j] * ip;
      else Sd[i][j] /= piv;
    }
    __syncthreads();
    const int rem = nb - j - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int i = j + 1 + e / rem, c = j + 1 + e % rem;
      if (c <= i) Sd[i][c] -= Sd[i][j] * conjx(Sd[c][j]);
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    A[(size_t)(k0 + i) * n + k0 + j] = (j <= i) ? Sd[i][j] : S(0.0);
  }
}

// rows below the diagonal block: X L_kk^H = A_ik. NQ lanes share a row
// (4 real, 8 complex), lane q holding the columns j = NQ u + q; column j is
// finished by its owner and passed to the other lanes of the row.
template <typename S> constexpr int trsm_lanes() { return IsCplx<S>::value ? 8 : 4; }

template <typename S>
__global__ void __launch_bounds__(256) k_chol_trsm(S* __restrict__ A, int n, int kb) {
  constexpr int NQ = trsm_lanes<S>(), NU = CB / NQ;
  __shared__ S Lk[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = (n - k0) < CB ? (n - k0) : CB;
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    Lk[i][j] = conjx(A[(size_t)(k0 + i) * n + k0 + j]);
  }
  __syncthreads();
  const int tid = threadIdx.x, q = tid % NQ, lane = tid & 63;
  const int row = k0 + nb + blockIdx.x * (256 / NQ) + tid / NQ;
  const bool live = row < n;
  S* a = A + (size_t)(live ? row : 0) * n + k0;
  S x[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int j = NQ * u + q;
    x[u] = (live && j < nb) ? a[j] : S(0.0);
  }
#pragma clang loop unroll(full)
  for (int j = 0; j < CB; ++j) {
    if (j < nb) {
      S xj = x[j / NQ] * (1.0 / realx(Lk[j][j]));
      if (q == j % NQ) x[j / NQ] = xj;
      const int src = (lane & ~(NQ - 1)) | (j % NQ);
      if constexpr (IsCplx<S>::value) xj = S(__shfl(xj.re, src, 64), __shfl(xj.im, src, 64));
      else xj = __shfl(xj, src, 64);
#pragma unroll
      for (int u = j / NQ; u < NU; ++u) {
        const int i = NQ * u + q;
        if (i > j && i < nb) x[u] -= xj * Lk[i][j];
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int j = NQ * u + q;
    if (j < nb) a[j] = x[u];
  }
}

// trailing update A_ij -= L_ik L_jk^H of the lower triangle on the matrix
// cores, 64 x 64 tiles (rows i, j beyond block kb; k over block kb)
template <typename S>
__global__ void __launch_bounds__(256) k_chol_syrk(S* __restrict__ A, int n, int kb,
                                                   int ntiles) {
  constexpr bool CX = IsCplx<S>::value;
  __shared__ HStage<CX> sh;
  int bi, bj;
  if (!tri_tile(ntiles, bi, bj)) return;
  const int k0 = kb * CB;
  const int base = k0 + CB;
  const int i0 = base + bi * HT, j0 = base + bj * HT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  HPart<CX> acc;
  acc.zero();
  for (int kk = 0; kk < CB; kk += HKC) {
    if (kk > 0) __syncthreads();
    for (int e = tid; e < HT * HKC; e += 256) {
      const int r = e / HKC, k = e - r * HKC;
      double re = 0.0, im = 0.0, re2 = 0.0, im2 = 0.0;
      if (i0 + r < n) split(A[(size_t)(i0 + r) * n + k0 + kk + k], re, im);
      if (j0 + r < n) split(A[(size_t)(j0 + r) * n + k0 + kk + k], re2, im2);
      hput<CX>(sh, false, k, r, re, im);
      hput<CX>(sh, true, k, r, re2, im2);
    }
    __syncthreads();
    hchunk<CX>(sh, acc, HKC, lane, wr, wc);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = j0 + 32 * wc + 16 * j + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = i0 + 32 * wr + 16 * i + 4 * v + (lane >> 4);
        if (r < n && c < n && c <= r) A[(size_t)r * n + c] -= hval<S, CX>(acc, i, j, v);
      }
    }
}

// ebar = (E - <E>)/sqrt(n) (Re E for real parameters) into y
template <typename S>
__global__ void k_ebar(const double* __restrict__ eloc, int n, const double* __restrict__ ws,
                       S* __restrict__ y, const int* __restrict__ run_if) {
  if (run_if && !*run_if) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double isn = 1.0 / sqrt((double)n);
  if constexpr (IsCplx<S>::value)
    y[i] = S((eloc[2 * i] - ws[0]) * isn, (eloc[2 * i + 1] - ws[8]) * isn);
  else
    y[i] = (eloc[2 * i] - ws[0]) * isn;
}

// Blocked triangular solves of y = L^-H L^-1 y over 64-row blocks, one
// launch per block. Forward (L z = b): workgroup g subtracts the solved
// block ub from the rows of block ub + 1 + g; workgroup 0, which holds
// block ub + 1 = sb, then solves it in one wave (lane i owns row i; the
// diagonal block sits transposed in LDS so that a column is a contiguous
// read). ub < 0: no update.
template <typename S>
__global__ void __launch_bounds__(256) k_trsv_fwd(const S* __restrict__ Lm, int n, int ub,
                                                  int sb, S* __restrict__ y) {
  __shared__ S Lt[CB][CB + 1];
  __shared__ S xs[CB], zs[CB];
  const int tid = threadIdx.x, lane = tid & 63;
  const int rb = (ub >= 0 ? ub + 1 : sb) + blockIdx.x;  // row block of this workgroup
  const int r0 = rb * CB;
  if (ub >= 0) {
    const int k0 = ub * CB;
    if (tid < CB) xs[tid] = y[k0 + tid];  // block ub is full: only the last can be short
    __syncthreads();
    const int r = tid >> 2, q = tid & 3, row = r0 + r;
    S acc = S(0.0);
    if (row < n) {
      const S* l = Lm + (size_t)row * n + k0 + 16 * q;
#pragma unroll
      for (int j = 0; j < 16; ++j) acc += l[j] * xs[16 * q + j];
    }
    acc += shfl_xor_x(acc, 1);
    acc += shfl_xor_x(acc, 2);
    if (q == 0 && row < n) {
      const S v = y[row] - acc;
      y[row] = v;
      zs[r] = v;
    }
  } else if (tid < CB) {
    zs[tid] = (r0 + tid < n) ? y[r0 + tid] : S(0.0);
  }
  if (blockIdx.x != 0 || sb < 0) return;
  const int k1 = sb * CB, nb = (n - k1) < CB ? (n - k1) : CB;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    if (j <= i) Lt[j][i] = Lm[(size_t)(k1 + i) * n + k1 + j];
  }
  __syncthreads();
  if (tid >= 64) return;
  S b = zs[lane];
  for (int j = 0; j < nb; ++j) {
    S bj;
    if constexpr (IsCplx<S>::value) bj = S(__shfl(b.re, j, 64), __shfl(b.im, j, 64));
    else bj = __shfl(b, j, 64);
    const S xj = bj * (1.0 / realx(Lt[j][j]));
    if (lane == j) b = xj;
    else if (lane > j && lane < nb) b -= Lt[j][lane] * xj;
  }
  if (lane < nb) y[k1 + lane] = b;
}

// Backward (L^H x = z): workgroup g subtracts the solved block ub from the
// rows of block g (g < ub); the last workgroup, which holds block sb =
// ub - 1, then solves it in one wave. ub = number of blocks: no update,
// one workgroup solving block sb.
template <typename S>
__global__ void __launch_bounds__(256) k_trsv_bwd(const S* __restrict__ Lm, int n, int ub,
                                                  int sb, int nblk, S* __restrict__ y) {
  __shared__ S Lr[CB][CB + 1];
  __shared__ S xs[CB], part[4][CB], zs[CB];
  const int tid = threadIdx.x, lane = tid & 63;
  const int rb = (ub < nblk) ? (int)blockIdx.x : sb;
  const int r0 = rb * CB;
  if (ub < nblk) {
    const int k0 = ub * CB, nbu = (n - k0) < CB ? (n - k0) : CB;
    if (tid < CB) xs[tid] = (tid < nbu) ? y[k0 + tid] : S(0.0);
    __syncthreads();
    const int r = lane, q = tid >> 6;
    S acc = S(0.0);
#pragma unroll 4
    for (int j = 16 * q; j < 16 * q + 16; ++j)
      if (j < nbu) acc += conjx(Lm[(size_t)(k0 + j) * n + r0 + r]) * xs[j];
    part[q][r] = acc;
    __syncthreads();
    if (tid < CB) {
      const S v = y[r0 + tid] - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
      y[r0 + tid] = v;
      zs[tid] = v;
    }
  } else if (tid < CB) {
    zs[tid] = (r0 + tid < n) ? y[r0 + tid] : S(0.0);
  }
  if (rb != sb) return;
  const int k1 = sb * CB, nb = (n - k1) < CB ? (n - k1) : CB;
  for (int e = tid; e < nb * nb; e += 256) {
    const int j = e / nb, i = e - j * nb;
    if (i <= j) Lr[j][i] = Lm[(size_t)(k1 + j) * n + k1 + i];
  }
  __syncthreads();
  if (tid >= 64) return;
  S b = zs[lane];
  for (int j = nb - 1; j >= 0; --j) {
    S bj;
    if constexpr (IsCplx<S>::value) bj = S(__shfl(b.re, j, 64), __shfl(b.im, j, 64));
    else bj = __shfl(b, j, 64);
    const S xj = bj * (1.0 / realx(Lr[j][j]));
    if (lane == j) b = xj;
    else if (lane < j) b -= conjx(Lr[j][lane]) * xj;
  }
  if (lane < nb) y[k1 + lane] = b;
}

// dtheta_k = (sum_s conj(O_sk) y_s - conj(m_k) sum_s y_s)/sqrt(n);
// certificate failure -> NaN
template <typename TO>
__global__ void k_dtheta(Lattice L, const int* __restrict__ tab, const TO* __restrict__ O,
                         const uint8_t* __restrict__ samples, int n,
                         const typename SolveT<TO>::type* __restrict__ y,
                         const typename SolveT<TO>::type* __restrict__ mean,
                         const typename SolveT<TO>::type* __restrict__ sy_p,
                         const double* __restrict__ ws, double* __restrict__ dth) {
  typedef typename SolveT<TO>::type S;
  const int jc = blockIdx.x * blockDim.x + threadIdx.x;
  if (jc >= L.n_compact) return;
  const int site = tab[L.off_csite + jc];
  const int j = jc - tab[L.off_compact + site];
  const int off = tab[L.off_param + site], blk = tab[L.off_block + site];
  const bool fail = ws[6] != 0.0;
  S acc0 = 0.0, acc1 = 0.0;
  for (int s = 0; s < n; ++s) {
    const S v = conjx(to_s(O[(size_t)s * L.n_compact + jc])) * y[s];
    if (pbit(samples[(size_t)s * L.N + site])) acc1 += v;
    else acc0 += v;
  }
  const S sy = *sy_p;
  const double isn = 1.0 / sqrt((double)n);
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  const S d0 = (acc0 - conjx(mean[off + j]) * sy) * isn;
  const S d1 = (acc1 - conjx(mean[off + blk + j]) * sy) * isn;
  put(dth, off + j, fail ? S(nan) : d0);
  put(dth, off + blk + j, fail ? S(nan) : d1);
}

template <typename S>
__global__ void k_sum_y(const S* __restrict__ y, int n, S* __restrict__ out) {
  __shared__ S red[8];
  S s = 0.0;
  for (int i = threadIdx.x; i < n; i += PEPS_NT) s += y[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

// certificate: no eigenvalue of T + eps I is dropped if trace(T) + eps <= eps / rcond
// (a non-finite local energy, flagged by k_estats, fails it too: diag[3] = 2).
// on = 1 runs the eigendecomposition solve: always with the eigh solver,
// after a failed certificate with the automatic one (never for a
// non-finite energy).
__global__ void k_certify(int n, double eps, double rcond, double* __restrict__ ws,
                          const int* __restrict__ bad, double* __restrict__ diag, int solver,
                          int* __restrict__ on) {
  if (threadIdx.x != 0) return;
  const double bound = ws[2] + eps;
  const bool ok = (eps > 0.0) && (bound * rcond <= eps);
  ws[6] = ok ? 0.0 : 1.0;
  if (ws[4] != 0.0) ws[6] = 1.0;
  if (*bad) ws[6] = 1.0;
  diag[0] = bound;
  diag[1] = eps;
  diag[2] = 0.0;
  diag[3] = *bad ? 2.0 : ws[6];
  diag[4] = ws[0];
  diag[5] = ws[1];
  diag[6] = (double)n;
  diag[7] = ws[5];
  *on = (*bad == 0) && (solver == MINSR_EIGH || (solver == MINSR_AUTO && ws[6] != 0.0));
}

// fresh state of a call: a kernel rather than a memset, so the whole step
// can be recorded into a graph and the workspace can be shared memory
__global__ void k_init_ws(double* ws, int* bad) {
  if (threadIdx.x == 0) {
    ws[4] = 0.0;
    ws[5] = 1e300;
    ws[6] = 0.0;
    bad[0] = 0;
    bad[1] = 0;
  }
}

template <typename TO>
static hipError_t minsr_impl(const Lattice& L, const int* tab, const TO* O, const uint8_t* samples,
                             int n, const double* eloc, double eps, double rcond, double* dtheta,
                             double* diag, void* mean_v, void* Tm_v, void* vec_v, int solver,
                             void* eig_ws, hipStream_t st) {
  typedef typename SolveT<TO>::type S;
  S* mean = (S*)mean_v;
  S* Tm = (S*)Tm_v;
  // vec layout: a[n+1] | y[n] | sum y | ws[16] (FP64) | bad, on (int)
  S* a = (S*)vec_v;
  S* y = a + n + 1;
  S* sy = y + n;
  double* ws = (double*)(sy + 1);
  int* bad = (int*)(ws + 16);
  int* on = bad + 1;
  hipLaunchKernelGGL(k_init_ws, dim3(1), dim3(64), 0, st, ws, bad);
  const int cb = (L.n_compact + 255) / 256;
  hipLaunchKernelGGL(k_colmean<TO>, dim3(cb), dim3(256), 0, st, L, tab, O, samples, n, mean);
  hipLaunchKernelGGL(k_proj_mean<TO>, dim3(n + 1), dim3(256), 0, st, L, tab, O, samples, n,
                     (const S*)mean, a);
  hipLaunchKernelGGL(k_estats<IsCplx<S>::value>, dim3(1), dim3(256), 0, st, eloc, n, ws, bad);
  const int nt = (n + HT - 1) / HT;
  hipLaunchKernelGGL(k_gram<TO>, dim3(tri_grid(nt)), dim3(256), 2 * L.N * sizeof(uint64_t), st,
                     L, tab, O, samples, n, (const S*)a, eps, Tm, nt * (nt + 1) / 2,
                     (const int*)nullptr);
  hipLaunchKernelGGL(k_trace<S>, dim3(1), dim3(256), 0, st, (const S*)Tm, n, eps, ws);
  const int nkb = (n + CB - 1) / CB;
  if (solver != MINSR_EIGH) {
    for (int kb = 0; kb < nkb; ++kb) {
      hipLaunchKernelGGL(k_chol_diag<S>, dim3(1), dim3(256), 0, st, Tm, n, kb, ws);
      const int rest = n - (kb + 1) * CB;
      if (rest > 0) {
        hipLaunchKernelGGL(k_chol_trsm<S>,
                           dim3((rest + 256 / trsm_lanes<S>() - 1) / (256 / trsm_lanes<S>())),
                           dim3(256), 0, st, Tm, n, kb);
        const int nr = (rest + HT - 1) / HT;
        hipLaunchKernelGGL(k_chol_syrk<S>, dim3(tri_grid(nr)), dim3(256), 0, st, Tm, n, kb,
                           nr * (nr + 1) / 2);
      }
    }
  }
  hipLaunchKernelGGL(k_certify, dim3(1), dim3(64), 0, st, n, eps, rcond, ws, (const int*)bad,
                     diag, solver, on);
  hipLaunchKernelGGL(k_ebar<S>, dim3((n + 255) / 256), dim3(256), 0, st, eloc, n,
                     (const double*)ws, y, (const int*)nullptr);
  if (solver != MINSR_EIGH) {
    hipLaunchKernelGGL(k_trsv_fwd<S>, dim3(1), dim3(256), 0, st, (const S*)Tm, n, -1, 0, y);
    for (int kb = 0; kb + 1 < nkb; ++kb)
      hipLaunchKernelGGL(k_trsv_fwd<S>, dim3(nkb - 1 - kb), dim3(256), 0, st, (const S*)Tm, n,
                         kb, kb + 1, y);
    hipLaunchKernelGGL(k_trsv_bwd<S>, dim3(1), dim3(256), 0, st, (const S*)Tm, n, nkb, nkb - 1,
                       nkb, y);
    for (int kb = nkb - 1; kb >= 1; --kb)
      hipLaunchKernelGGL(k_trsv_bwd<S>, dim3(kb), dim3(256), 0, st, (const S*)Tm, n, kb, kb - 1,
                         nkb, y);
  }
  if (solver != MINSR_CHOLESKY && n <= MINSR_EIG_MAX) {
    if (solver == MINSR_AUTO) {
      // the factorisation overwrote T and y: form both again if the path runs
      hipLaunchKernelGGL(k_gram<TO>, dim3(tri_grid(nt)), dim3(256), 2 * L.N * sizeof(uint64_t),
                         st, L, tab, O, samples, n, (const S*)a, eps, Tm, nt * (nt + 1) / 2,
                         (const int*)on);
      hipLaunchKernelGGL(k_ebar<S>, dim3((n + 255) / 256), dim3(256), 0, st, eloc, n,
                         (const double*)ws, y, (const int*)on);
    }
    const hipError_t e = launch_eigh_solve(IsCplx<S>::value, Tm, n, rcond, on, ws, diag, y,
                                           eig_ws, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sum_y<S>, dim3(1), dim3(256), 0, st, (const S*)y, n, sy);
  hipLaunchKernelGGL(k_dtheta<TO>, dim3(cb), dim3(256), 0, st, L, tab, O, samples, n,
                     (const S*)y, (const S*)mean, (const S*)sy, (const double*)ws, dtheta);
  return hipGetLastError();
}

// bytes of the minSR workspaces: mean [N_p], T [n][n], vec
void minsr_ws_bytes(const Lattice& L, int mode, int n, size_t* mean, size_t* T, size_t* vec) {
  const size_t es = (mode == MODE_C128 || mode == MODE_C64) ? 16 : 8;
  *mean = (size_t)L.n_params * es;
  *T = (size_t)n * n * es;
  *vec = ((size_t)2 * n + 2) * es + 16 * sizeof(double) + 16;
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

// Complex parameters: the gradient of sum_s g_s ln|Psi(S_s)| with respect to
// (Re theta_k, Im theta_k) as the pair d/dRe + i d/dIm = sum_s g_s conj(O_sk)
// (ln|Psi| = Re ln Psi and ln Psi is holomorphic with derivative O_k).
template <typename R>
__global__ void k_vjp_c(Lattice L, const int* __restrict__ tab, const cplx<R>* __restrict__ O,
                        const uint8_t* __restrict__ samples, int n, const double* __restrict__ g,
                        double* __restrict__ out) {
  const int jc = blockIdx.x * blockDim.x + threadIdx.x;
  if (jc >= L.n_compact) return;
  const int site = tab[L.off_csite + jc];
  const int j = jc - tab[L.off_compact + site];
  const int off = tab[L.off_param + site], blk = tab[L.off_block + site];
  cplx<double> acc0(0.0, 0.0), acc1(0.0, 0.0);
  for (int s = 0; s < n; ++s) {
    const cplx<R> o = O[(size_t)s * L.n_compact + jc];
    const cplx<double> v((double)o.re * g[s], -(double)o.im * g[s]);
    if (pbit(samples[(size_t)s * L.N + site])) acc1 += v;
    else acc0 += v;
  }
  put(out, off + j, acc0);
  put(out, off + blk + j, acc1);
}

hipError_t launch_vjp(const Lattice& L, const int* tab, int mode, const void* O,
                      const uint8_t* samples, int n, const double* g, double* out,
                      hipStream_t st) {
  const int cb = (L.n_compact + 255) / 256;
  if (mode == MODE_F64)
    hipLaunchKernelGGL(k_vjp<double>, dim3(cb), dim3(256), 0, st, L, tab, (const double*)O,
                       samples, n, g, out);
  else if (mode == MODE_C128)
    hipLaunchKernelGGL(k_vjp_c<double>, dim3(cb), dim3(256), 0, st, L, tab,
                       (const cplx<double>*)O, samples, n, g, out);
  else if (mode == MODE_C64)
    hipLaunchKernelGGL(k_vjp_c<float>, dim3(cb), dim3(256), 0, st, L, tab,
                       (const cplx<float>*)O, samples, n, g, out);
  else
    hipLaunchKernelGGL(k_vjp<float>, dim3(cb), dim3(256), 0, st, L, tab, (const float*)O,
                       samples, n, g, out);
  return hipGetLastError();
}

// Parameter update of the optimisation loop (Eq. tdvp): theta moves by
// -tau dtheta, element by element over the real (or interleaved complex)
// FP64 parameters; a step whose certificate failed leaves theta unchanged.
__global__ void k_theta_update(double* __restrict__ theta, const double* __restrict__ dtheta,
                               const double* __restrict__ diag, double tau, size_t m) {
  if (diag[3] != 0.0) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (size_t)gridDim.x * blockDim.x)
    theta[i] = fma(-tau, dtheta[i], theta[i]);
}

hipError_t launch_theta_update(double* theta, const double* dtheta, const double* diag,
                               double tau, size_t m, hipStream_t st) {
  const size_t blocks = (m + 255) / 256 < 1024 ? (m + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_theta_update, dim3(blocks > 0 ? (unsigned)blocks : 1u), dim3(256), 0, st,
                     theta, dtheta, diag, tau, m);
  return hipGetLastError();
}

hipError_t launch_minsr(const Lattice& L, const int* tab, int mode, const void* O,
                        const uint8_t* samples, int n, const double* eloc, double eps,
                        double rcond, double* dtheta, double* diag, void* ws_mean, void* ws_T,
                        void* ws_vec, int solver, void* eig_ws, hipStream_t st) {
  switch (mode) {
    case MODE_F64:
      return minsr_impl<double>(L, tab, (const double*)O, samples, n, eloc, eps, rcond, dtheta,
                                diag, ws_mean, ws_T, ws_vec, solver, eig_ws, st);
    case MODE_C128:
      return minsr_impl<cplx<double>>(L, tab, (const cplx<double>*)O, samples, n, eloc, eps,
                                      rcond, dtheta, diag, ws_mean, ws_T, ws_vec, solver, eig_ws, st);
    case MODE_C64:
      return minsr_impl<cplx<float>>(L, tab, (const cplx<float>*)O, samples, n, eloc, eps, rcond,
                                     dtheta, diag, ws_mean, ws_T, ws_vec, solver, eig_ws, st);
    default:
      return minsr_impl<float>(L, tab, (const float*)O, samples, n, eloc, eps, rcond, dtheta,
                               diag, ws_mean, ws_T, ws_vec, solver, eig_ws, st);
  }
}

}  // namespace pm
