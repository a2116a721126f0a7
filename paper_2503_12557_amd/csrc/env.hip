// Boundary-MPS environments (Sec. "On the boundary MPS method") and the
// amplitude at the middle cut (Eq. boundary_MPS_approx).
//
// One workgroup owns one (sample, direction) pair and walks the whole sweep:
// the first row read as an MPS, then each further row absorbed and the
// product truncated back to chi. The truncation is the canonical two-sweep
// one written so that no orthogonal factor is ever stored:
//   left to right : R_y = R factor of (R_{y-1} P_y), by Householder QR of the
//                   stacked [R_acc; R_{y-1} P_y[:, k, :]] blocks, one physical
//                   index k at a time;
//   right to left : Z_y = P_y W_{y+1}, C_y = R_{y-1} Z_y, one-sided Jacobi on
//                   the rows of C_y gives its right singular vectors; the chi
//                   dominant ones are the new tensor B_y and W_y = Z_y B_y^T.
// R_{y-1} Z_y is the centre matrix of the canonical form (its Gram is the
// left environment of the density-matrix algorithm), so the truncated state
// is the one both of those algorithms produce.
#include "common.h"
#include "env_dev.h"
#include "kernels.h"

namespace pm {

size_t env_lds_elems(int bmax, int D, int mode) { return env_lds_elems_(bmax, D, mode); }

// GM: the matrices live in a per-workgroup slab of gws (slab elements each)
// instead of LDS, for shapes whose working set exceeds the on-chip memory.
template <int M, bool GM>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_env_sweep(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
            const uint8_t* __restrict__ samples, typename ModeT<M>::T* __restrict__ env,
            double* __restrict__ logs, typename ModeT<M>::T* __restrict__ rscr,
            int* __restrict__ flags, int n, int jac_sweeps, typename ModeT<M>::T* __restrict__ gws,
            size_t slab, int dir0) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int smp = blockIdx.x;
  const int dir = (int)blockIdx.y + dir0;  // 0: from the top, 1: from the bottom
  const bool bottom = dir == 1;
  if (smp >= n) return;
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* big = GM ? gws + ((size_t)smp * 2 + dir) * slab : lds;
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
  T* R = rscr + ((size_t)smp * 2 + (bottom ? 1 : 0)) * (size_t)L.Ly * BD * BD;
  env_first_row<M>(L, tab, theta, s, bottom, envs, lg, sh, &fl);
  for (int t = 1; t <= L.Lx - 2; ++t)
    env_absorb_row<M>(L, tab, theta, s, bottom, t, envs, lg, R, sh, sel, sflag, &fl, jac_sweeps);
  if (threadIdx.x == 0 && fl && flags) atomicOr(flags + smp, fl);
}

// ln(E^u[i] . E^l[i+1]) + scales for one sample per workgroup.
template <int M>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_overlap(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ env,
          const double* __restrict__ logs, int icut, double* __restrict__ logpsi,
          int* __restrict__ flags, int n) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int smp = blockIdx.x;
  if (smp >= n) return;
  const int tid = threadIdx.x;
  const int B = L.bmax, D = L.D;
  T* Lm = sm;               // B x B
  T* X = Lm + B * B;        // B x D x B
  const size_t slot_elems = (size_t)L.Ly * L.site_box;
  const T* envs = env + (size_t)smp * L.n_slots * slot_elems;
  const int su = slot_top(L, icut), sb = slot_bottom(L, icut + 1);
  const int* ed = tab + L.off_env;
  if (tid == 0) Lm[0] = T(1);
  __syncthreads();
  int da = 1, dc = 1;
  int esum = 0;  // powers of two taken out of the transfer matrix
  for (int y = 0; y < L.Ly; ++y) {
    const T* U = envs + (size_t)su * slot_elems + (size_t)y * L.site_box;
    const T* Bt = envs + (size_t)sb * slot_elems + (size_t)y * L.site_box;
    const int ua = ed[(su * L.Ly + y) * 3 + 0], uk = ed[(su * L.Ly + y) * 3 + 1],
              ub = ed[(su * L.Ly + y) * 3 + 2];
    const int bc = ed[(sb * L.Ly + y) * 3 + 0], bd = ed[(sb * L.Ly + y) * 3 + 2];
    // X[c,k,b] = sum_a L[a,c] U[a,k,b]
    gemm<M>(dc, uk * ub, da, Lm, 1, dc, U, uk * ub, 1, X, uk * ub, 1, false);
    __syncthreads();
    // L'[b,d] = sum_{c,k} X[(c,k), b] B[(c,k), d]
    gemm<M>(ub, bd, bc * uk, X, 1, ub, Bt, bd, 1, Lm, bd, 1, false);
    __syncthreads();
    if (y + 1 < L.Ly) {
      // unit scale between columns (the FP32 range is exceeded otherwise)
      const int e = pow2_exponent((double)block_absmax(Lm, ub, bd, bd, X));
      scale_pow2(Lm, ub * bd, e);
      esum += e;
      __syncthreads();
    }
    da = ub;
    dc = bd;
  }
  if (tid == 0) {
    const double* lg = logs + (size_t)smp * L.n_slots;
    const double sc = lg[su] + lg[sb] + esum * 0.69314718055994530942;
    int f = 0;
    if constexpr (IsCplx<T>::value) {
      const double vr = (double)Lm[0].re, vi = (double)Lm[0].im;
      if (vr == 0.0 && vi == 0.0) f |= 1;
      if (!isfinite(vr) || !isfinite(vi)) f |= 2;
      logpsi[2 * smp] = log(hypot(vr, vi)) + sc;
      logpsi[2 * smp + 1] = atan2(vi, vr);
    } else {
      const double v = (double)Lm[0];
      if (v == 0.0) f |= 1;
      if (!isfinite(v)) f |= 2;
      logpsi[2 * smp] = log(fabs(v)) + sc;
      logpsi[2 * smp + 1] = v < 0 ? 3.14159265358979323846 : 0.0;
    }
    if (f && flags) atomicOr(flags + smp, f);
  }
}

// theta (FP64, or interleaved FP64 pairs for complex modes) to the compute type
template <typename T>
__global__ void k_convert_theta(const double* __restrict__ src, T* __restrict__ dst, int n,
                                int* __restrict__ bad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if constexpr (IsCplx<T>::value) {
      typedef typename RealOf<T>::type R;
      const double a = src[2 * i], b = src[2 * i + 1];
      if (!isfinite(a) || !isfinite(b)) atomicOr(bad, 1);
      dst[i] = T((R)a, (R)b);
    } else {
      const double v = src[i];
      if (!isfinite(v)) atomicOr(bad, 1);
      dst[i] = (T)v;
    }
  }
}

// every sample's flags get bit 1 (non-finite) when theta held a non-finite value
__global__ void k_flag_bad(int* __restrict__ flags, int n, const int* __restrict__ bad) {
  if (*bad == 0) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    flags[i] |= 2;
}

hipError_t launch_flag_bad(int* flags, int n, const int* bad, hipStream_t st) {
  const int blocks = (n + 255) / 256 < 256 ? (n + 255) / 256 : 256;
  hipLaunchKernelGGL(k_flag_bad, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, flags, n, bad);
  return hipGetLastError();
}

// ---- host launchers ----
size_t env_lds_bytes(int mode, const Lattice& L, bool gm) {
  const size_t es = mode_elem_bytes(mode);
  return (gm ? env_small_elems(L.bmax, L.D) : env_lds_elems_(L.bmax, L.D, mode)) * es;
}
size_t env_slab_elems(const Lattice& L, int mode) {
  return (env_big_elems(L.bmax, L.D, mode) + 15) / 16 * 16;
}

template <int M>
hipError_t launch_env_sweep(const Lattice& L, const int* tab, const void* theta,
                            const uint8_t* samples, void* env, double* logs, void* rscr,
                            int* flags, int n, int jac_sweeps, void* gws, hipStream_t st,
                            bool bottom_only) {
  typedef typename ModeT<M>::T T;
  const dim3 grid(n, bottom_only ? 1 : 2);
  const int dir0 = bottom_only ? 1 : 0;
  if (gws) {
    const size_t lds = env_lds_bytes(M, L, true);
    hipFuncSetAttribute((const void*)k_env_sweep<M, true>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_env_sweep<M, true>), grid, dim3(env_threads(M)), lds, st, L, tab,
                       (const T*)theta, samples, (T*)env, logs, (T*)rscr, flags, n, jac_sweeps,
                       (T*)gws, env_slab_elems(L, M), dir0);
  } else {
    const size_t lds = env_lds_bytes(M, L, false);
    hipFuncSetAttribute((const void*)k_env_sweep<M, false>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_env_sweep<M, false>), grid, dim3(env_threads(M)), lds, st, L, tab,
                       (const T*)theta, samples, (T*)env, logs, (T*)rscr, flags, n, jac_sweeps,
                       (T*)nullptr, (size_t)0, dir0);
  }
  return hipGetLastError();
}

template <int M>
hipError_t launch_overlap(const Lattice& L, const int* tab, const void* env, const double* logs,
                          int icut, double* logpsi, int* flags, int n, hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const size_t lds = (size_t)(L.bmax * L.bmax + L.bmax * L.D * L.bmax) * sizeof(T);
  hipFuncSetAttribute((const void*)k_overlap<M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  hipLaunchKernelGGL(k_overlap<M>, dim3(n), dim3(256), lds, st, L, tab, (const T*)env,
                     logs, icut, logpsi, flags, n);
  return hipGetLastError();
}

hipError_t launch_convert_theta(int mode, const double* src, void* dst, int n, int* bad,
                                hipStream_t st) {
  const int blocks = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
  const dim3 g(blocks > 0 ? blocks : 1);
  if (mode == MODE_F64)
    hipLaunchKernelGGL(k_convert_theta<double>, g, dim3(256), 0, st, src, (double*)dst, n, bad);
  else if (mode == MODE_C128)
    hipLaunchKernelGGL(k_convert_theta<cplx<double>>, g, dim3(256), 0, st, src,
                       (cplx<double>*)dst, n, bad);
  else if (mode == MODE_C64)
    hipLaunchKernelGGL(k_convert_theta<cplx<float>>, g, dim3(256), 0, st, src,
                       (cplx<float>*)dst, n, bad);
  else
    hipLaunchKernelGGL(k_convert_theta<float>, g, dim3(256), 0, st, src, (float*)dst, n, bad);
  return hipGetLastError();
}

#define INST(M)                                                                                 \
  template hipError_t launch_env_sweep<M>(const Lattice&, const int*, const void*,             \
                                          const uint8_t*, void*, double*, void*, int*, int, int, \
                                          void*, hipStream_t, bool);                            \
  template hipError_t launch_overlap<M>(const Lattice&, const int*, const void*, const double*, \
                                        int, double*, int*, int, hipStream_t);
INST(MODE_F64)
INST(MODE_F32)
INST(MODE_BF16)
INST(MODE_C128)
INST(MODE_C64)
#undef INST

}  // namespace pm
