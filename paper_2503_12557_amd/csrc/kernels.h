// Host-side launchers of the device kernels (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace pm {

// Hamiltonian tables on the device (built by the host term compiler).
//   mstart[n_strips+1] : CSR of the moves of each strip (one-row strips
//                        x = 0..Lx-1, then two-row strips x = 0..Lx-2), moves
//                        of a strip sorted by their first column
//   moves[8*m]          : y0, y1, nsites, site0, site1, site2, cstart, ccount
//   contrib[2*c]        : term, flip mask (bit j = j-th site of the term, MSB first)
//   terms[4*t]          : nsites, site0, site1, site2
//   mats[t][64][2]      : <c|h_t|c'> as (re, im)
struct HamDev {
  int n_strips;
  int n_terms;
  int n_pairs;
  const int* mstart;
  const int* moves;
  const int* contrib;
  const int* terms;
  const double* mats;
  const int* pair_ij;
  const double* pair_v;
  const double* onsite;  // [N][2] or null
};

// Per-workgroup working sets. Each kernel keeps its matrices in LDS when
// they fit ("_lds_bytes" with gm = false); otherwise the host passes a
// global working-set buffer gws of one slab ("_slab_elems" elements of the
// compute type) per workgroup of the grid, and only the small vectors stay
// in LDS (gm = true; the two-row strips in the FP32 modes also keep chunks
// of their steps' first and last intermediates there).
size_t env_lds_elems(int bmax, int D, int mode);
size_t strip1_lds_elems(int bmax, int D);
size_t strip2_lds_elems(int bmax, int D);
size_t env_lds_bytes(int mode, const Lattice& L, bool gm);
size_t strip1_lds_bytes(int mode, const Lattice& L, bool gm);
size_t strip2_lds_bytes(int mode, const Lattice& L, bool gm);
size_t sample_lds_bytes(int mode, const Lattice& L, bool gm);
size_t env_slab_elems(const Lattice& L, int mode);
size_t strip1_slab_elems(const Lattice& L);
size_t strip2_slab_elems(const Lattice& L, int mode);
size_t sample_slab_elems(const Lattice& L, int mode);

template <int M>
hipError_t launch_env_sweep(const Lattice& L, const int* tab, const void* theta,
                            const uint8_t* samples, void* env, double* logs, void* rscr,
                            int* flags, int n, int jac_sweeps, void* gws, hipStream_t st,
                            bool bottom_only = false);
// density-matrix environments on the matrix cores (env_dm.hip): one
// persistent grid of `grid` workgroups, each with a slab of
// env_dm_slab_elems elements of the compute type
size_t env_dm_slab_elems(const Lattice& L, int mode);
size_t env_dm_lds_bytes(const Lattice& L, int mode);
int env_dm_grid(const Lattice& L, int mode, int tasks);
template <int M>
hipError_t launch_env_dm(const Lattice& L, const int* tab, const void* theta,
                         const uint8_t* samples, void* env, double* logs, int* flags, int n,
                         void* slabs, int grid, hipStream_t st, bool bottom_only = false);
template <int M>
hipError_t launch_overlap(const Lattice& L, const int* tab, const void* env, const double* logs,
                          int icut, double* logpsi, int* flags, int n, hipStream_t st);
hipError_t launch_convert_theta(int mode, const double* src, void* dst, int n, int* bad,
                                hipStream_t st);
hipError_t launch_flag_bad(int* flags, int n, const int* bad, hipStream_t st);

template <int M>
hipError_t launch_strip1(const Lattice& L, const int* tab, const void* theta,
                         const uint8_t* samples, const void* env, const HamDev& H, void* rt,
                         double* epart, void* O, int* flags, int n, bool want_e, bool want_o,
                         void* gws, hipStream_t st);
template <int M>
hipError_t launch_strip2(const Lattice& L, const int* tab, const void* theta,
                         const uint8_t* samples, const void* env, const HamDev& H, void* rt,
                         double* epart, int* flags, int n, void* gws, hipStream_t st);
hipError_t launch_energy_diag_sum(const Lattice& L, const HamDev& H, const uint8_t* samples,
                                  const double* epart, int nparts, double* eloc, int n,
                                  hipStream_t st);

// strict local energy: neighbour counts and offsets (off[n+1], starting at
// n), the batch [samples | neighbours] with coefficients, the combination
hipError_t launch_strict_count(const Lattice& L, const HamDev& H, int n_moves,
                               const uint8_t* samples, int n, int* cnt, int* off,
                               hipStream_t st);
hipError_t launch_strict_expand(const Lattice& L, const HamDev& H, int n_moves,
                                const uint8_t* samples, int n, const int* off, uint8_t* batch,
                                double* coef, hipStream_t st);
hipError_t launch_strict_combine(int n, const int* off, const double* coef, const double* lp,
                                 const int* bfl, double* eloc, int* flags, hipStream_t st);

// direct sampler: double-layer parameters, one top-environment step for a
// batch, one row drawn for a batch, the importance weights
size_t direct_slab_elems(const Lattice& L, const Lattice& L2);
hipError_t launch_double_theta(const Lattice& L, const int* tab, const Lattice& L2,
                               const int* tab2, const double* theta, double* dst, bool cplx_,
                               hipStream_t st);
template <int M>
hipError_t launch_env_top_step(const Lattice& L, const int* tab, const void* theta,
                               const uint8_t* samples, void* env, double* logs, void* rscr,
                               int* flags, int n, int t, int jac_sweeps, void* gws,
                               hipStream_t st);
template <int M>
hipError_t launch_direct_row(const Lattice& L, const int* tab, const void* theta, const void* env,
                             const Lattice& L2, const int* tab2, const void* env2,
                             uint8_t* samples, double* logp, int* flags, int n, int i,
                             uint64_t seed, uint64_t offset, void* slab, hipStream_t st);
hipError_t launch_direct_logw(int n, const double* lpsi, const double* logp, const int* afl,
                              double* logw, int* flags, hipStream_t st);

// Metropolis sampler; state: sample_state_bytes of chain states and counts;
// dm_slabs (chains x env_dm_slab_elems) selects the density-matrix
// truncation for the environments, nullptr the canonical one
size_t sample_lds_elems(int bmax, int D, int mode);
size_t sample_state_bytes(const Lattice& L, int n_chains);
template <int M>
hipError_t launch_metropolis(const Lattice& L, const int* tab, const void* theta, int kind,
                             int n_chains, int per_chain, int burn_in, int thin, uint64_t seed,
                             uint64_t offset, uint8_t* samples, int* accepted, void* envscr,
                             double* logscr, void* rscr, void* rt1, void* rt2, int jac_sweeps,
                             void* gws, void* state, void* dm_slabs, hipStream_t st);
// the sampler's environment phase by the density-matrix truncation
hipError_t launch_smp_env_dm(const Lattice& L, const int* tab, int mode, const void* theta,
                             int n_chains, int row, const uint8_t* state, void* env, double* logs,
                             void* slabs, hipStream_t st);

// learned proposal
hipError_t launch_made_forward(int N, int H, int n_up, int bf16, const float* P,
                               const uint8_t* x, int B, float* a, float* lg, hipStream_t st);
hipError_t launch_made_head(int N, int H, int n_up, const uint8_t* x, int B, const float* lg,
                            float* dlg, double* logq, hipStream_t st);
hipError_t launch_made_backward(int N, int H, int n_up, int bf16, const float* P,
                                const uint8_t* x, int B, const float* a, const float* dlg,
                                float* da, float* G, const double* logq, double* loss,
                                hipStream_t st);
hipError_t launch_made_gather(const uint8_t* data, int M, int N, int B, long long base,
                              const unsigned long long* tab, uint8_t* out, hipStream_t st);
hipError_t launch_imh_record(int n_chains, int N, const uint8_t* state, const double* st_lp,
                             int per_chain, int j, uint8_t* out, double* out_lp, hipStream_t st);
hipError_t launch_tau_int(const double* series, int nc, int T, int ranked, double c,
                          double* work, double* out, hipStream_t st);
hipError_t launch_made_adam(int n, float* P, const float* G, float* m, float* v, int t, float lr,
                            float b1, float b2, float eps, hipStream_t st);
hipError_t launch_made_sample(int N, int H, int n_up, int bf16, const float* P, int n,
                              uint64_t seed, uint64_t offset, uint8_t* out, double* logq,
                              hipStream_t st);
hipError_t launch_imh(int n_chains, int N, uint8_t* state, double* st_lp, double* st_lq,
                      const uint8_t* prop, const double* pr_lp, const double* pr_lq, uint64_t seed,
                      uint64_t step, int* accepted, hipStream_t st);

// global basis rotation of FP64 parameters (real, or interleaved complex):
// ROT_X multiplies every physical index by the Hadamard matrix, ROT_Y by
// H S^dagger (complex parameters only); in and out may alias
#define ROT_X 1
#define ROT_Y 2
hipError_t launch_rotate_basis(const Lattice& L, const int* tab, int basis, bool cplx,
                               const double* in, double* out, hipStream_t st);

hipError_t launch_vjp(const Lattice& L, const int* tab, int mode, const void* O,
                      const uint8_t* samples, int n, const double* g, double* out,
                      hipStream_t st);

// minSR
// mode: MODE_F64 / MODE_F32 (FP64 solve of real parameters) or MODE_C128 /
// MODE_C64 (complex FP64 solve); workspaces sized by minsr_ws_bytes.
// solver: certified Cholesky, eigendecomposition, or Cholesky with the
// eigendecomposition after a failed certificate (n <= MINSR_EIG_MAX for the
// latter two; eig_ws of eigh_ws_bytes(n, complex) bytes, else unused).
#define MINSR_CHOLESKY 0
#define MINSR_EIGH 1
#define MINSR_AUTO 2
#define MINSR_EIG_MAX 3072
void minsr_ws_bytes(const Lattice& L, int mode, int n, size_t* mean, size_t* T, size_t* vec);
hipError_t launch_minsr(const Lattice& L, const int* tab, int mode, const void* O,
                        const uint8_t* samples, int n, const double* eloc, double eps,
                        double rcond, double* dtheta, double* diag, void* ws_mean, void* ws_T,
                        void* ws_vec, int solver, void* eig_ws, hipStream_t st);
// eigendecomposition solve of T y = ebar in place of y (runs when *on)
size_t eigh_ws_bytes(int n, bool cplx);
hipError_t launch_eigh_solve(bool cplx, void* Tm, int n, double rcond, const int* on, double* ws,
                             double* diag, void* y, void* eig_ws, hipStream_t st);
// theta[i] -= tau * dtheta[i] for i < m, skipped when diag[3] (failed
// pseudo-inverse certificate) is set
hipError_t launch_theta_update(double* theta, const double* dtheta, const double* diag,
                               double tau, size_t m, hipStream_t st);

}  // namespace pm
