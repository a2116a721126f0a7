// Global single-site basis rotation of the PEPS parameters (Sec. "On reusing
// environments and the convenient treatment of long-range interactions"):
// the tensors of U^(x N) Psi are T'[s] = sum_p U[s, p] T[p] on every site's
// physical index, with U the Hadamard H (X -> Z) or H S^dagger (Y -> Z,
// S = diag(1, i)). One workgroup per site; each thread reads both physical
// slices of its elements before writing them, so the call may run in place.
#include "common.h"
#include "kernels.h"

namespace pm {

__global__ void __launch_bounds__(256)
k_rotate_basis(Lattice L, const int* __restrict__ tab, int basis, int cplx,
               const double* in, double* out) {
  const int n = blockIdx.x;
  const int off = tab[L.off_param + n], blk = tab[L.off_block + n];
  const double h = 0.70710678118654752440;  // 1 / sqrt(2)
  for (int e = threadIdx.x; e < blk; e += blockDim.x) {
    if (!cplx) {
      const double a = in[off + e], b = in[off + blk + e];
      out[off + e] = h * a + h * b;
      out[off + blk + e] = h * a - h * b;
      continue;
    }
    const size_t i0 = 2 * ((size_t)off + e), i1 = 2 * ((size_t)off + blk + e);
    const double ar = in[i0], ai = in[i0 + 1], br = in[i1], bi = in[i1 + 1];
    if (basis == ROT_X) {
      // (a + b) / sqrt 2, (a - b) / sqrt 2
      out[i0] = h * ar + h * br;
      out[i0 + 1] = h * ai + h * bi;
      out[i1] = h * ar - h * br;
      out[i1 + 1] = h * ai - h * bi;
    } else {
      // (a - i b) / sqrt 2, (a + i b) / sqrt 2
      out[i0] = h * ar + h * bi;
      out[i0 + 1] = h * ai - h * br;
      out[i1] = h * ar - h * bi;
      out[i1 + 1] = h * ai + h * br;
    }
  }
}

hipError_t launch_rotate_basis(const Lattice& L, const int* tab, int basis, bool cplx,
                               const double* in, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_rotate_basis, dim3(L.N), dim3(256), 0, st, L, tab, basis, cplx ? 1 : 0,
                     in, out);
  return hipGetLastError();
}

}  // namespace pm
