// Learned proposal: a masked autoregressive network over the sites in
// raster order (one hidden ReLU layer), trained on configurations drawn by
// the PEPS sampler, and the independence Metropolis-Hastings step that keeps
// the PEPS as the arbiter: accept S' with probability
// min(1, |Psi(S')|^2 q(S) / (|Psi(S)|^2 q(S'))).
//
// Masks: hidden degree m(k) = (k mod (N-1)) + 1, input mask [m(k) >= n+1],
// output mask [n+1 > m(k)]. Parameters (FP32 master copy): W1 [H][N],
// b1 [H], W2 [N][H], b2 [N]. With bf16 != 0 the weights are rounded to
// bfloat16 where they enter a product (accumulation stays FP32).
// Sites are forced once the S^z = 0 budget of zeros (n_up) or ones is used up;
// forced sites add nothing to log q or to the loss.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace pm {

#define TAG_MADE 0x4D414445u
#define TAG_IMH 0x494D4821u

__device__ __forceinline__ bool mask_in(int k, int n, int N) { return (k % (N - 1)) + 1 >= n + 1; }
__device__ __forceinline__ bool mask_out(int n, int k, int N) { return n + 1 > (k % (N - 1)) + 1; }
__device__ __forceinline__ float wround(float w, int bf16) { return bf16 ? bf16_round(w) : w; }

// Tiled GEMM C[i][j] = sum_k A(i,k) B(k,j) on the FP32 matrix cores: 64 x 64
// tiles, 16-deep k chunks staged in LDS, each of the four waves a 32 x 32
// sub-tile of 2 x 2 MFMA 16x16x4 tiles (FP32 products, FP32 accumulation;
// bf16-rounded weights are exact FP32 values). A, B and the epilogue are
// functors so the masks, the ReLU and the biases are applied on the fly.
template <class LA, class LB, class EP>
__global__ void __launch_bounds__(256) k_gemm(int M, int Nn, int K, LA la, LB lb, EP ep) {
  __shared__ float As[16][68], Bs[16][68];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = (wv >> 1) * 32, wj = (wv & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef Mfma<float> F;
  F::acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e >> 6, r = e & 63;
      const bool kin = k0 + kk < K;
      As[kk][r] = (kin && i0 + r < M) ? la(i0 + r, k0 + kk) : 0.f;
      Bs[kk][r] = (kin && j0 + r < Nn) ? lb(k0 + kk, j0 + r) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = 4 * s + lk;
      const float a0 = As[kk][wi + li], a1 = As[kk][wi + 16 + li];
      const float b0 = Bs[kk][wj + li], b1 = Bs[kk][wj + 16 + li];
      acc[0][0] = F::mac(a0, b0, acc[0][0]);
      acc[0][1] = F::mac(a0, b1, acc[0][1]);
      acc[1][0] = F::mac(a1, b0, acc[1][0]);
      acc[1][1] = F::mac(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = i0 + wi + 16 * a + F::row(lane, v), c = j0 + wj + 16 * b + li;
        if (r < M && c < Nn) ep(r, c, acc[a][b][v]);
      }
}

struct MadeP {
  int N, H, n_up, bf16;
  const float* W1;
  const float* b1;
  const float* W2;
  const float* b2;
};

// ---- forward ----
struct LX {  // x[b][n] as float
  const uint8_t* x;
  int N;
  __device__ float operator()(int b, int n) const { return (float)pbit(x[(size_t)b * N + n]); }
};
struct LW1T {  // (W1 * M1)^T [n][k]
  MadeP p;
  __device__ float operator()(int n, int k) const {
    return mask_in(k, n, p.N) ? wround(p.W1[(size_t)k * p.N + n], p.bf16) : 0.f;
  }
};
struct EHid {  // a[b][k] = acc + b1[k]
  float* a;
  MadeP p;
  __device__ void operator()(int b, int k, float v) const { a[(size_t)b * p.H + k] = v + p.b1[k]; }
};
struct LRelu {  // relu(a[b][k])
  const float* a;
  int H;
  __device__ float operator()(int b, int k) const {
    const float v = a[(size_t)b * H + k];
    return v > 0.f ? v : 0.f;
  }
};
struct LW2T {  // (W2 * M2)^T [k][n]
  MadeP p;
  __device__ float operator()(int k, int n) const {
    return mask_out(n, k, p.N) ? wround(p.W2[(size_t)n * p.H + k], p.bf16) : 0.f;
  }
};
struct ELogit {
  float* lg;
  MadeP p;
  __device__ void operator()(int b, int n, float v) const { lg[(size_t)b * p.N + n] = v + p.b2[n]; }
};

// ---- backward ----
struct LDlgT {  // dlg^T [n][b]
  const float* d;
  int N;
  __device__ float operator()(int n, int b) const { return d[(size_t)b * N + n]; }
};
struct EgW2 {
  float* g;
  MadeP p;
  __device__ void operator()(int n, int k, float v) const {
    g[(size_t)n * p.H + k] = mask_out(n, k, p.N) ? v : 0.f;
  }
};
struct LDlg {  // dlg [b][n]
  const float* d;
  int N;
  __device__ float operator()(int b, int n) const { return d[(size_t)b * N + n]; }
};
struct LW2 {  // (W2 * M2) [n][k]
  MadeP p;
  __device__ float operator()(int n, int k) const {
    return mask_out(n, k, p.N) ? wround(p.W2[(size_t)n * p.H + k], p.bf16) : 0.f;
  }
};
struct EdA {  // da[b][k] = acc * [a > 0]
  float* da;
  const float* a;
  int H;
  __device__ void operator()(int b, int k, float v) const {
    da[(size_t)b * H + k] = a[(size_t)b * H + k] > 0.f ? v : 0.f;
  }
};
struct LDaT {  // da^T [k][b]
  const float* da;
  int H;
  __device__ float operator()(int k, int b) const { return da[(size_t)b * H + k]; }
};
struct EgW1 {
  float* g;
  MadeP p;
  __device__ void operator()(int k, int n, float v) const {
    g[(size_t)k * p.N + n] = mask_in(k, n, p.N) ? v : 0.f;
  }
};

// per-sample log q, dloss/dlogit = free * (sigmoid - x) / B (one thread per sample)
__global__ void k_made_head(int B, MadeP p, const uint8_t* __restrict__ x,
                            const float* __restrict__ lg, float* __restrict__ dlg,
                            double* __restrict__ logq) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  int zeros = 0, ones = 0;
  double lq = 0.0;
  const int n_dn = p.N - p.n_up;
  for (int n = 0; n < p.N; ++n) {
    const int s = pbit(x[(size_t)b * p.N + n]);
    const bool forced = p.n_up >= 0 && (zeros >= p.n_up || ones >= n_dn);
    const float l = lg[(size_t)b * p.N + n];
    if (!forced) {
      // log sigmoid(+-l) in double
      const double z = s ? (double)l : -(double)l;
      lq += z >= 0 ? -log1p(exp(-z)) : z - log1p(exp(z));
    }
    if (dlg) {
      const float sg = 1.f / (1.f + expf(-l));
      dlg[(size_t)b * p.N + n] = forced ? 0.f : (sg - (float)s) / (float)B;
    }
    zeros += s == 0;
    ones += s == 1;
  }
  logq[b] = lq;
}

// column sums: out[j] = sum_b in[b][j] (bias gradients), one thread per column
__global__ void k_colsum(int B, int C, const float* __restrict__ in, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= C) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += in[(size_t)b * C + j];
  out[j] = s;
}

// loss = -mean(logq), deterministic single-block reduction
__global__ void k_made_loss(int B, const double* __restrict__ logq, double* __restrict__ loss) {
  __shared__ double red[8];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += PEPS_NT) s += logq[b];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *loss = -s / B;
}

__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Autoregressive sampling: one wave per sample, hidden pre-activations kept
// in registers and updated as each site is drawn (O(N H) per sample).
__global__ void __launch_bounds__(256) k_made_sample(MadeP p, int n, uint32_t k0, uint32_t k1,
                                                    uint32_t off, uint8_t* __restrict__ out,
                                                    double* __restrict__ logq) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int smp = blockIdx.x * 4 + w;
  if (smp >= n) return;
  float h[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = lane + 64 * i;
    h[i] = k < p.H ? p.b1[k] : 0.f;
  }
  int zeros = 0, ones = 0;
  double lq = 0.0;
  const int n_dn = p.N - p.n_up;
  for (int nn = 0; nn < p.N; ++nn) {
    float part = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = lane + 64 * i;
      if (k < p.H && mask_out(nn, k, p.N)) {
        const float hv = h[i] > 0.f ? h[i] : 0.f;
        part += wround(p.W2[(size_t)nn * p.H + k], p.bf16) * hv;
      }
    }
    part = wave_sum(part);
    const float l = part + p.b2[nn];
    int bit;
    if (p.n_up >= 0 && zeros >= p.n_up) bit = 1;
    else if (p.n_up >= 0 && ones >= n_dn) bit = 0;
    else {
      u4 c;
      c.x = (uint32_t)nn;
      c.y = (uint32_t)smp;
      c.z = off;
      c.w = TAG_MADE;
      const u4 o = philox(c, k0, k1);
      const double u = philox_uniform(o.x, o.y);
      const double p1 = 1.0 / (1.0 + exp(-(double)l));
      bit = u < p1 ? 1 : 0;
      const double z = bit ? (double)l : -(double)l;
      lq += z >= 0 ? -log1p(exp(-z)) : z - log1p(exp(z));
    }
    if (lane == 0) out[(size_t)smp * p.N + nn] = (uint8_t)bit;
    zeros += bit == 0;
    ones += bit == 1;
    if (bit) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = lane + 64 * i;
        if (k < p.H && mask_in(k, nn, p.N)) h[i] += wround(p.W1[(size_t)k * p.N + nn], p.bf16);
      }
    }
  }
  if (lane == 0) logq[smp] = lq;
}

// Independence MH step per chain: accept the proposal iff
// ln u < 2 (ln|Psi'| - ln|Psi|) + ln q(S) - ln q(S').
__global__ void k_imh(int n_chains, int N, uint8_t* __restrict__ state,
                      double* __restrict__ st_lp, double* __restrict__ st_lq,
                      const uint8_t* __restrict__ prop, const double* __restrict__ pr_lp,
                      const double* __restrict__ pr_lq, uint32_t k0, uint32_t k1, uint32_t step,
                      int* __restrict__ accepted) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_chains) return;
  u4 ctr;
  ctr.x = (uint32_t)c;
  ctr.y = step;
  ctr.z = 0u;
  ctr.w = TAG_IMH;
  const u4 o = philox(ctr, k0, k1);
  const double u = philox_uniform(o.x, o.y);
  const double lr = 2.0 * (pr_lp[2 * c] - st_lp[2 * c]) + st_lq[c] - pr_lq[c];
  if (u > 0.0 && log(u) < lr) {
    for (int i = 0; i < N; ++i) state[(size_t)c * N + i] = prop[(size_t)c * N + i];
    st_lp[2 * c] = pr_lp[2 * c];
    st_lp[2 * c + 1] = pr_lp[2 * c + 1];
    st_lq[c] = pr_lq[c];
    if (accepted) accepted[c] += 1;
  }
}

// Mini-batch gather: row b of the batch is data row (a_e r + c_e) mod M for
// position g = base + b of the epoch sequence, e = g / M, r = g mod M; a_e is
// coprime with M, so each epoch visits every row once in a permuted order.
__global__ void k_gather_batch(const uint8_t* __restrict__ data, int M, int N, int B, long long base,
                               const unsigned long long* __restrict__ tab,
                               uint8_t* __restrict__ out) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const long long g = base + b;
  const long long e = g / M, r = g - e * M;
  const unsigned long long a = tab[2 * e], c = tab[2 * e + 1];
  const long long row = (long long)((a * (unsigned long long)r + c) % (unsigned long long)M);
  for (int n = threadIdx.x; n < N; n += blockDim.x)
    out[(size_t)b * N + n] = data[(size_t)row * N + n];
}

hipError_t launch_made_gather(const uint8_t* data, int M, int N, int B, long long base,
                              const unsigned long long* tab, uint8_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_batch, dim3(B), dim3(64), 0, st, data, M, N, B, base, tab, out);
  return hipGetLastError();
}

// Chain c's state (and ln Psi) into row c * per_chain + j of the output.
__global__ void k_imh_record(int n_chains, int N, const uint8_t* __restrict__ state,
                             const double* __restrict__ st_lp, int per_chain, int j,
                             uint8_t* __restrict__ out, double* __restrict__ out_lp) {
  const int c = blockIdx.x;
  if (c >= n_chains) return;
  const size_t row = (size_t)c * per_chain + j;
  for (int i = threadIdx.x; i < N; i += blockDim.x) out[row * N + i] = state[(size_t)c * N + i];
  if (out_lp && threadIdx.x == 0) {
    out_lp[2 * row] = st_lp[2 * c];
    out_lp[2 * row + 1] = st_lp[2 * c + 1];
  }
}

hipError_t launch_imh_record(int n_chains, int N, const uint8_t* state, const double* st_lp,
                             int per_chain, int j, uint8_t* out, double* out_lp, hipStream_t st) {
  hipLaunchKernelGGL(k_imh_record, dim3(n_chains), dim3(64), 0, st, n_chains, N, state, st_lp,
                     per_chain, j, out, out_lp);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Integrated autocorrelation time of a scalar series on n_chains chains of
// length T (Sokal's automatic window, c), the autocorrelation averaged over
// chains and centred on the mean over all chains (the chains start
// stationary). ranked: the series is first replaced by the normal scores
// Phi^-1((r - 3/8) / (S + 1/4)) of its pooled ranks r (average rank for
// ties; Blom's offsets), as in the rank-normalised effective sample size of
// Vehtari et al. (2021). One workgroup; work: S + T doubles.
// ---------------------------------------------------------------------------
// Phi^-1(p) for 0 < p < 1: Acklam's rational approximation (relative error
// below 1.2e-9) refined by one Halley step on Phi(x) = erfc(-x / sqrt 2) / 2.
__device__ double inv_normal_cdf(double p) {
  const double a[6] = {-3.969683028665376e+01, 2.209460984245205e+02, -2.759285104469687e+02,
                       1.383577518672690e+02, -3.066479806614716e+01, 2.506628277459239e+00};
  const double b[5] = {-5.447609879822406e+01, 1.615858368580409e+02, -1.556989798598866e+02,
                       6.680131188771972e+01, -1.328068155288572e+01};
  const double c[6] = {-7.784894002430293e-03, -3.223964580411365e-01, -2.400758277161838e+00,
                       -2.549732539343734e+00, 4.374664141464968e+00, 2.938163982698783e+00};
  const double d[4] = {7.784695709041462e-03, 3.224671290700398e-01, 2.445134137142996e+00,
                       3.754408661907416e+00};
  const double plow = 0.02425;
  double x;
  if (p < plow) {
    const double q = sqrt(-2.0 * log(p));
    x = (((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
        ((((d[0] * q + d[1]) * q + d[2]) * q + d[3]) * q + 1.0);
  } else if (p <= 1.0 - plow) {
    const double q = p - 0.5, r = q * q;
    x = (((((a[0] * r + a[1]) * r + a[2]) * r + a[3]) * r + a[4]) * r + a[5]) * q /
        (((((b[0] * r + b[1]) * r + b[2]) * r + b[3]) * r + b[4]) * r + 1.0);
  } else {
    const double q = sqrt(-2.0 * log(1.0 - p));
    x = -(((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
        ((((d[0] * q + d[1]) * q + d[2]) * q + d[3]) * q + 1.0);
  }
  const double e = 0.5 * erfc(-x * 0.70710678118654752440) - p;
  const double u = e * 2.50662827463100050242 * exp(0.5 * x * x);
  return x - u / (1.0 + 0.5 * x * u);
}

__global__ void __launch_bounds__(1024) k_tau_int(const double* __restrict__ series, int nc, int T,
                                                  int ranked, double cwin,
                                                  double* __restrict__ work,
                                                  double* __restrict__ out) {
  __shared__ double red[16];
  __shared__ double sv[2];
  const int S = nc * T, tid = threadIdx.x, NT = blockDim.x;
  const double* x = series;
  double* z = work;
  double* ac = work + S;
  if (ranked) {
    for (int i = tid; i < S; i += NT) {
      const double xi = series[i];
      long long less = 0, eq = 0;
      for (int j = 0; j < S; ++j) {
        const double xj = series[j];
        less += xj < xi;
        eq += xj == xi;
      }
      const double r = (double)less + 0.5 * (double)(eq + 1);
      z[i] = inv_normal_cdf((r - 0.375) / ((double)S + 0.25));
    }
    __syncthreads();
    x = z;
  }
  double sm = 0;
  for (int i = tid; i < S; i += NT) sm += x[i];
  sm = block_sum(sm, red);
  const double mu = sm / S;
  for (int t = tid; t < T; t += NT) {
    double a = 0;
    for (int cc = 0; cc < nc; ++cc) {
      const double* row = x + (size_t)cc * T;
      for (int i = 0; i + t < T; ++i) a += (row[i] - mu) * (row[i + t] - mu);
    }
    ac[t] = a / ((double)nc * (double)(T - t));
  }
  __syncthreads();
  if (tid == 0) {
    double tau = 1.0;
    if (ac[0] > 0.0 && T >= 2) {
      double s = 0.0;
      for (int W = 1; W < T; ++W) {
        s += ac[W] / ac[0];
        tau = 1.0 + 2.0 * s;
        if (W >= cwin * tau) break;
      }
    }
    if (tau < 1.0) tau = 1.0;
    sv[0] = tau;
    out[0] = tau;
    out[1] = (double)S / tau;
  }
}

hipError_t launch_tau_int(const double* series, int nc, int T, int ranked, double c,
                          double* work, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_tau_int, dim3(1), dim3(1024), 0, st, series, nc, T, ranked, c, work, out);
  return hipGetLastError();
}

static MadeP made_params(int N, int H, int n_up, int bf16, const float* P) {
  MadeP p;
  p.N = N;
  p.H = H;
  p.n_up = n_up;
  p.bf16 = bf16;
  p.W1 = P;
  p.b1 = P + (size_t)H * N;
  p.W2 = p.b1 + H;
  p.b2 = p.W2 + (size_t)N * H;
  return p;
}

static dim3 grid2(int M, int Nn) { return dim3((Nn + 63) / 64, (M + 63) / 64); }

hipError_t launch_made_forward(int N, int H, int n_up, int bf16, const float* P,
                               const uint8_t* x, int B, float* a, float* lg, hipStream_t st) {
  const MadeP p = made_params(N, H, n_up, bf16, P);
  hipLaunchKernelGGL((k_gemm<LX, LW1T, EHid>), grid2(B, H), dim3(256), 0, st, B, H, N, LX{x, N},
                     LW1T{p}, EHid{a, p});
  hipLaunchKernelGGL((k_gemm<LRelu, LW2T, ELogit>), grid2(B, N), dim3(256), 0, st, B, N, H,
                     LRelu{a, H}, LW2T{p}, ELogit{lg, p});
  return hipGetLastError();
}

hipError_t launch_made_head(int N, int H, int n_up, const uint8_t* x, int B, const float* lg,
                            float* dlg, double* logq, hipStream_t st) {
  MadeP p = made_params(N, H, n_up, 0, nullptr);
  hipLaunchKernelGGL(k_made_head, dim3((B + 127) / 128), dim3(128), 0, st, B, p, x, lg, dlg, logq);
  return hipGetLastError();
}

hipError_t launch_made_backward(int N, int H, int n_up, int bf16, const float* P,
                                const uint8_t* x, int B, const float* a, const float* dlg,
                                float* da, float* G, const double* logq, double* loss,
                                hipStream_t st) {
  const MadeP p = made_params(N, H, n_up, bf16, P);
  float* gW1 = G;
  float* gb1 = G + (size_t)H * N;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (size_t)N * H;
  // dW2[n][k] = sum_b dlg[b][n] relu(a[b][k])
  hipLaunchKernelGGL((k_gemm<LDlgT, LRelu, EgW2>), grid2(N, H), dim3(256), 0, st, N, H, B,
                     LDlgT{dlg, N}, LRelu{a, H}, EgW2{gW2, p});
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, st, B, N, dlg, gb2);
  // da[b][k] = (sum_n dlg[b][n] W2m[n][k]) [a > 0]
  hipLaunchKernelGGL((k_gemm<LDlg, LW2, EdA>), grid2(B, H), dim3(256), 0, st, B, H, N,
                     LDlg{dlg, N}, LW2{p}, EdA{da, a, H});
  // dW1[k][n] = sum_b da[b][k] x[b][n]
  hipLaunchKernelGGL((k_gemm<LDaT, LX, EgW1>), grid2(H, N), dim3(256), 0, st, H, N, B,
                     LDaT{da, H}, LX{x, N}, EgW1{gW1, p});
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, st, B, H, da, gb1);
  hipLaunchKernelGGL(k_made_loss, dim3(1), dim3(256), 0, st, B, logq, loss);
  return hipGetLastError();
}

hipError_t launch_made_adam(int n, float* P, const float* G, float* m, float* v, int t, float lr,
                            float b1, float b2, float eps, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  const int blocks = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, st, n, P, G, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_made_sample(int N, int H, int n_up, int bf16, const float* P, int n,
                              uint64_t seed, uint64_t offset, uint8_t* out, double* logq,
                              hipStream_t st) {
  const MadeP p = made_params(N, H, n_up, bf16, P);
  hipLaunchKernelGGL(k_made_sample, dim3((n + 3) / 4), dim3(256), 0, st, p, n,
                     (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), (uint32_t)offset, out,
                     logq);
  return hipGetLastError();
}

hipError_t launch_imh(int n_chains, int N, uint8_t* state, double* st_lp, double* st_lq,
                      const uint8_t* prop, const double* pr_lp, const double* pr_lq, uint64_t seed,
                      uint64_t step, int* accepted, hipStream_t st) {
  hipLaunchKernelGGL(k_imh, dim3((n_chains + 127) / 128), dim3(128), 0, st, n_chains, N, state,
                     st_lp, st_lq, prop, pr_lp, pr_lq, (uint32_t)(seed & 0xffffffffu),
                     (uint32_t)(seed >> 32), (uint32_t)step, accepted);
  return hipGetLastError();
}

}  // namespace pm
