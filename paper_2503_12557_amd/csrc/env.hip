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

size_t env_lds_elems(int bmax, int D) { return env_lds_elems_(bmax, D); }

template <int M>
__global__ void __launch_bounds__(PEPS_BLOCK_MAX)
k_env_sweep(Lattice L, const int* __restrict__ tab, const typename ModeT<M>::T* __restrict__ theta,
            const uint8_t* __restrict__ samples, typename ModeT<M>::T* __restrict__ env,
            double* __restrict__ logs, typename ModeT<M>::T* __restrict__ rscr,
            int* __restrict__ flags, int n, int jac_sweeps) {
  typedef typename ModeT<M>::T T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int smp = blockIdx.x;
  const bool bottom = blockIdx.y == 1;
  if (smp >= n) return;
  const EnvSmem<T> sh(reinterpret_cast<T*>(smem_raw), L);
  const int BD = L.bmax * L.D;
  __shared__ int sflag, fl;
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
    env_absorb_row<M>(L, tab, theta, s, bottom, t, envs, lg, R, sh, sel, &sflag, &fl, jac_sweeps);
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
    da = ub;
    dc = bd;
  }
  if (tid == 0) {
    const double v = (double)Lm[0];
    const double* lg = logs + (size_t)smp * L.n_slots;
    const double sc = lg[su] + lg[sb];
    int f = 0;
    if (v == 0.0) f |= 1;
    if (!isfinite(v)) f |= 2;
    logpsi[2 * smp] = log(fabs(v)) + sc;
    logpsi[2 * smp + 1] = v < 0 ? 3.14159265358979323846 : 0.0;
    if (f && flags) atomicOr(flags + smp, f);
  }
}

template <typename T>
__global__ void k_convert_theta(const double* __restrict__ src, T* __restrict__ dst, int n,
                                int* __restrict__ bad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double v = src[i];
    if (!isfinite(v)) atomicOr(bad, 1);
    dst[i] = (T)v;
  }
}

// ---- host launchers ----
template <int M>
hipError_t launch_env_sweep(const Lattice& L, const int* tab, const void* theta,
                            const uint8_t* samples, void* env, double* logs, void* rscr,
                            int* flags, int n, int jac_sweeps, hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const size_t lds = env_lds_elems(L.bmax, L.D) * sizeof(T);
  hipFuncSetAttribute((const void*)k_env_sweep<M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  dim3 grid(n, 2);
  hipLaunchKernelGGL(k_env_sweep<M>, grid, dim3(env_threads(M)), lds, st, L, tab, (const T*)theta,
                     samples, (T*)env, logs, (T*)rscr, flags, n, jac_sweeps);
  return hipGetLastError();
}

template <int M>
hipError_t launch_overlap(const Lattice& L, const int* tab, const void* env, const double* logs,
                          int icut, double* logpsi, int* flags, int n, hipStream_t st) {
  typedef typename ModeT<M>::T T;
  const size_t lds = (size_t)(L.bmax * L.bmax + L.bmax * L.D * L.bmax) * sizeof(T);
  hipLaunchKernelGGL(k_overlap<M>, dim3(n), dim3(256), lds, st, L, tab, (const T*)env,
                     logs, icut, logpsi, flags, n);
  return hipGetLastError();
}

hipError_t launch_convert_theta(int mode, const double* src, void* dst, int n, int* bad,
                                hipStream_t st) {
  const int blocks = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
  if (mode == MODE_F64)
    hipLaunchKernelGGL(k_convert_theta<double>, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st,
                       src, (double*)dst, n, bad);
  else
    hipLaunchKernelGGL(k_convert_theta<float>, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st,
                       src, (float*)dst, n, bad);
  return hipGetLastError();
}

template hipError_t launch_env_sweep<MODE_F64>(const Lattice&, const int*, const void*,
                                               const uint8_t*, void*, double*, void*, int*, int,
                                               int, hipStream_t);
template hipError_t launch_env_sweep<MODE_F32>(const Lattice&, const int*, const void*,
                                               const uint8_t*, void*, double*, void*, int*, int,
                                               int, hipStream_t);
template hipError_t launch_env_sweep<MODE_BF16>(const Lattice&, const int*, const void*,
                                                const uint8_t*, void*, double*, void*, int*, int,
                                                int, hipStream_t);
template hipError_t launch_overlap<MODE_F64>(const Lattice&, const int*, const void*,
                                             const double*, int, double*, int*, int, hipStream_t);
template hipError_t launch_overlap<MODE_F32>(const Lattice&, const int*, const void*,
                                             const double*, int, double*, int*, int, hipStream_t);
template hipError_t launch_overlap<MODE_BF16>(const Lattice&, const int*, const void*,
                                              const double*, int, double*, int*, int, hipStream_t);

}  // namespace pm
