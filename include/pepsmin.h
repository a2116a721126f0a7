/*
 * pepsmin — sampled finite-PEPS amplitudes, local energies, log-derivatives
 * and the minimum-step stochastic-reconfiguration (minSR) update on AMD
 * Instinct MI355X (gfx950).
 *
 * The calls follow the operations a sampling-based PEPS optimisation needs
 * (arXiv 2503.12557, Sec. "Finite PEPS and Sampling"): samples from
 * p(S) = |Psi(S)|^2/<Psi|Psi>, the amplitudes Psi(S), the local estimator
 * O_loc(S) = sum_S' <S|O|S'> Psi(S')/Psi(S) (Eq. local_estimator), the
 * log-derivatives O_{S,i} = (dPsi(S)/dtheta_i)/Psi(S) (Eq. tdvp) and the
 * minSR solution dtheta = O^dagger (O O^dagger)^-1 E_loc (Eq. tdvp_fast).
 *
 * Conventions shared by every call
 *  - Lattice: open Lx x Ly square lattice, rows x = 0..Lx-1 from the top,
 *    columns y = 0..Ly-1, site n = x*Ly + y. Physical dimension d = 2.
 *  - Parameters theta: the entries of the site tensors T[x,y] of shape
 *    (d, Dl, Dr, Du, Dd) in C order, sites concatenated in row-major order;
 *    virtual legs on an open edge have dimension 1. theta is FP64 [N_p]
 *    (real modes) or interleaved (re, im) FP64 pairs [N_p][2] (complex
 *    modes), converted to the compute precision inside the call.
 *  - Samples: uint8 [n][Lx*Ly], one physical index per site (0 = spin up /
 *    atom in |g>, 1 = spin down / atom in |r>).
 *  - Amplitudes are contracted with boundary MPS of bond chi (Sec. "On the
 *    boundary MPS method"): rows are absorbed from the top and from the
 *    bottom, each MPS-MPO product is truncated to chi by a left QR sweep and
 *    a right SVD sweep (the same truncated state as the density-matrix
 *    algorithm) and every tensor is divided by its largest modulus with the
 *    logarithms accumulated in FP64 (Sec. "On Numerical Stability").
 *  - Every pointer passed to a compute call is caller-owned DEVICE memory
 *    unless stated otherwise; the library reads and writes it only from
 *    work enqueued on the given stream, keeps no reference after the call
 *    and frees nothing it did not allocate. The context owns only its own
 *    workspace, grown on demand with hipMalloc.
 *  - Every call returns a peps_status; no exception crosses the ABI. On an
 *    error nothing is enqueued and peps_last_error() describes it.
 *  - Calls enqueue work on `stream` and return; results are valid after the
 *    stream is synchronised. One context per host thread at a time.
 */
#ifndef PEPSMIN_H
#define PEPSMIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PEPS_OK = 0,
  PEPS_ERR_ARG = 1,          /* bad shape, null pointer, out-of-range value */
  PEPS_ERR_UNSUPPORTED = 2,  /* valid request outside what is implemented */
  PEPS_ERR_HIP = 3,          /* a HIP runtime call failed */
  PEPS_ERR_OOM = 4,          /* device workspace could not be allocated */
  PEPS_ERR_NONFINITE = 5     /* non-finite input (theta, E_loc) */
} peps_status;

/* Asynchrony. peps_amplitude, peps_local_energy, peps_logderiv,
 * peps_evaluate and minsr_step_noalloc enqueue their work on the stream and
 * return without waiting for the device: a non-finite theta is then not a
 * return code but bit PEPS_FLAG_NONFINITE in every sample's flags (when
 * flags are requested; the outputs are non-finite too). minsr_step checks
 * E_loc on the host first (one synchronisation); the samplers, the
 * optimisation step and the strict energy synchronise where they need a
 * count or a decision from the device. */

/* Compute precision of the contractions (Sec. "On Numerical Stability"
 * discusses reduced precision). Log scales, local energies and the minSR
 * solve are always FP64 (complex FP64 for complex parameters). */
typedef enum {
  PEPS_F64 = 0,   /* real tensors, FP64 everywhere */
  PEPS_F32 = 1,   /* real tensors, FP32 contractions, QR and SVD */
  PEPS_BF16 = 2,  /* real tensors, BF16 contraction operands with FP32
                     accumulation; QR/SVD in FP32 */
  PEPS_C128 = 3,  /* complex tensors, complex128 contractions, QR and SVD */
  PEPS_C64 = 4    /* complex tensors, complex64 contractions, QR and SVD */
} peps_dtype;

/* Per-sample flags (bit set = condition seen for that sample). */
enum {
  PEPS_FLAG_ZERO = 1,        /* Psi(S) = 0 exactly */
  PEPS_FLAG_NONFINITE = 2,   /* a non-finite value appeared */
  PEPS_FLAG_NOCONV = 4,      /* a Jacobi SVD hit its sweep limit */
  PEPS_FLAG_DEGENERATE = 8   /* relative gap at a truncation cut below 1e-8, or a
                                cutoff decision within its margin */
};

/* Sampler kinds for peps_sample. */
enum { PEPS_SAMPLE_EXCHANGE = 0, PEPS_SAMPLE_FLIP = 1 };

typedef struct {
  int Lx, Ly;   /* lattice size, 2 <= Lx, Ly <= 32 */
  int d;        /* physical dimension, must be 2 */
  int D;        /* virtual bond dimension, >= 1 */
  int chi;      /* boundary-MPS bond dimension D_c, >= 1 */
  int dtype;    /* peps_dtype */
} peps_geom;

typedef struct peps_ctx peps_ctx;

/* Create a context for one geometry and precision; *out receives it.
 * Kernels whose per-workgroup matrices do not fit in LDS keep them in a
 * global-memory slab per workgroup instead (slower, same results).
 * PEPS_ERR_UNSUPPORTED if max(chi, D) * D > 256 or D > 16. */
peps_status peps_create(const peps_geom* geom, peps_ctx** out);
void peps_destroy(peps_ctx* ctx);

/* Thread-local description of the last error; valid until the next call. */
const char* peps_last_error(void);

/* Number of parameters N_p; the compact log-derivative row has N_p/d. */
size_t peps_num_params(const peps_ctx* ctx);

/* Bytes of the environment cache for n samples: every top environment
 * E^u[0..Lx-2] and bottom environment E^l[1..Lx-1] of every sample, each site
 * tensor padded to chi*D*chi entries of the compute type (complex entries
 * for complex modes), plus the FP64 log scales. */
size_t peps_env_cache_bytes(const peps_ctx* ctx, int n);

/* Hamiltonian H = sum_t h_t + sum_(i<j) V_ij n_i n_j + sum_i onsite[i][s_i].
 * HOST pointers. Term t acts on term_nsites[t] (1..3) sites listed in
 * term_sites[3*t + j] and has the 2^k x 2^k complex matrix
 * term_mats[t][c][c'] = <c|h_t|c'> stored as interleaved (re, im) FP64 pairs
 * in blocks of 64 complex entries per term (8 x 8, row-major, only the
 * leading 2^k x 2^k used); the first listed site is the most significant
 * bit of c. Diagonal pairs: pair_ij[2p], pair_ij[2p+1], value pair_v[p].
 * onsite: [N][2] FP64 or NULL. The local energy of S is
 * E_loc(S) = sum_t sum_S' <S|h_t|S'> Psi(S')/Psi(S) + diagonal parts
 * (Eq. local_obs with the element read as <S|H|S'>); every ratio is taken
 * inside the one-row or two-row strip that holds the changed sites, reusing
 * the environments outside it (Sec. "On reusing environments"); diagonal
 * terms of any range need no amplitude.
 * PEPS_ERR_UNSUPPORTED if an off-diagonal term changes sites on more than
 * two adjacent rows. */
peps_status peps_set_hamiltonian(peps_ctx* ctx, int n_terms, const int* term_nsites,
                                 const int* term_sites, const double* term_mats,
                                 int n_pairs, const int* pair_ij, const double* pair_v,
                                 const double* onsite);

/* Direct sampling (Sec. "On Direct Sampling"; App. "Direct sampling of
 * PEPS", Eq. prob_from_cond_prob): n independent configurations drawn row by
 * row from the top. Row i comes from the conditional density matrix
 * T^u . D^l[i+1] . T^u*, where T^u is the top environment E^u[i-1] of the
 * drawn rows (bond chi, truncated as in peps_amplitude) times the open row
 * i (its bond chi*D is not truncated further), and D^l[i+1] the boundary
 * MPS from the bottom of the double-layer network (site tensors
 * sum_p T[p] x conj(T[p]), bond D^2) with bond chi_double. refresh != 0
 * builds D^l from theta; refresh = 0 reuses the D^l of the context's last
 * refresh (same chi_double, else PEPS_ERR_ARG), possibly of older tensors:
 * the paper's stale double-layer environments, which leave the importance
 * weights exact because ln p is the sampler's own. n = 0 with refresh != 0
 * only builds D^l. Sites are drawn from the left: s = 0 iff u < q_0 / (q_0 + q_1) with
 * u from Philox4x32-10 (key = seed; counter (site, j mod 2^32, j >> 32,
 * 0x44495243), j = offset + index); a negative q counts as 0.
 * samples: device uint8 [n][N] (written); logp: device FP64 [n], ln p(S)
 * of the sampler (written); logw: device FP64 [n] or NULL, the unnormalised
 * log importance weight ln|Psi(S)_i*|^2 - ln p(S) (the amplitude of
 * peps_amplitude), which corrects the sampler's bias by reweighting; flags:
 * int32 [n] or NULL (1: both q zero at some site, 2: non-finite value, and
 * the amplitude's flags). Needs D^2 <= 16, max(chi_double, D^2) * D^2 <=
 * 256 and the row kernel's staged column, (max(chi, D)^2 D + 2 D^4 +
 * max(chi_double, D^2)^2 D^2) elements of the compute type, within 150 KiB
 * of LDS (e.g. FP64 at D = 4 allows chi <= 60 with chi_double = 4); any of
 * these fails with PEPS_ERR_UNSUPPORTED before anything is queued. The workspace (double-layer context,
 * per-sample slabs of O(Ly chi^2 D^2 chi_double) elements) is grown on
 * demand; returns with the work queued on the stream. */
peps_status peps_direct_sample(peps_ctx* ctx, const double* theta, int n, int chi_double,
                               int refresh, uint64_t seed, uint64_t offset, uint8_t* samples,
                               double* logp, double* logw, int32_t* flags, void* stream);

/* Truncation rule of every boundary-MPS compression of the context
 * (environments, amplitudes, strips, sampler; Sec. "On the boundary MPS
 * method": the contraction bond chosen dynamically from a maximal truncated
 * weight, 1e-4 in the paper's runs). max_weight = 0 (the default) keeps chi
 * singular values per bond. max_weight in (0, 1): at each bond the fewest
 * r <= chi singular values sigma_k (descending) with
 * sum_{k>=r} sigma_k^2 <= max_weight * sum_k sigma_k^2; chi when chi values
 * discard more. The environments keep their chi-wide layout: the bond
 * directions beyond r are zero. A cut whose kept count lies within a
 * relative margin of the limit (1e-8 in FP64/complex128, 1e-4 in the FP32
 * modes) sets flag 8, like a degenerate cut. Host-side setting, takes effect
 * at the next call. PEPS_ERR_ARG outside [0, 1). */
peps_status peps_set_truncation(peps_ctx* ctx, double max_weight);

/* Truncation algorithm of the context's environment kernels (the amplitude,
 * energy and log-derivative calls and the Metropolis sampler's
 * environments; the direct sampler keeps the canonical one). Both give the
 * same truncated boundary MPS; DENSMAT is the faster one once chi*D exceeds
 * 64 (about 16x at 10x10 D=5 chi=25 in FP32), CANONICAL at chi*D <= 64,
 * where its factorisations stay in registers and LDS:
 *   PEPS_COMPRESS_CANONICAL (default): left-to-right QR, right-to-left SVD
 *     of the centre matrix (Sec. "On the boundary MPS method").
 *   PEPS_COMPRESS_DENSMAT: the density-matrix MPS-MPO algorithm the paper
 *     uses (same section): left Gram environments
 *     G_{y+1} = sum_k P_k^H G_y P_k of the untruncated product, then from
 *     the right the reduced density matrix rho_y = Z_y^H G_y Z_y of each
 *     site and its chi leading eigenvectors (the new tensor) in the compute
 *     precision; the Gram and density products run on the matrix cores.
 * The cut flags (8) and a maximal truncated weight apply to both, the
 * eigenvalues of rho_y being the squared singular values. PEPS_ERR_ARG for
 * an unknown method; PEPS_ERR_UNSUPPORTED for DENSMAT when chi*D rounded
 * up to 32 exceeds 256, chi exceeds 255 or the packed density matrix
 * (n(n+1)/2 elements, n = that padded size) does not fit in LDS (e.g.
 * complex128 at chi*D > 128, FP64 at chi*D > 160). Host-side setting,
 * takes effect at the next call. */
#define PEPS_COMPRESS_CANONICAL 0
#define PEPS_COMPRESS_DENSMAT 1
peps_status peps_set_compression(peps_ctx* ctx, int method);

/* ln Psi(S)_i* = ln(E^u[i*] . E^l[i*+1]) with i* = floor(Lx/2) - 1
 * (Eq. boundary_MPS_approx), as (ln|Psi|, arg Psi) FP64 pairs in
 * logpsi[n][2]. env_cache: device buffer of peps_env_cache_bytes(n) that
 * receives every environment of every sample, or NULL to keep none.
 * flags: int32 [n] or NULL. */
peps_status peps_amplitude(peps_ctx* ctx, const double* theta, const uint8_t* samples,
                           int n, void* env_cache, double* logpsi, int32_t* flags,
                           void* stream);

/* Local energies eloc[n][2] (complex, FP64) of the Hamiltonian set by
 * peps_set_hamiltonian. env_cache must hold the environments written by
 * peps_amplitude for the same theta and samples, or be NULL (then they are
 * rebuilt in the context's workspace). */
peps_status peps_local_energy(peps_ctx* ctx, const double* theta, const uint8_t* samples,
                              int n, const void* env_cache, double* eloc, int32_t* flags,
                              void* stream);

/* Strict local energies (Sec. "On Variational Upper Bound"): eloc[n][2] as
 * for peps_local_energy, except that every amplitude is the full contraction
 * at the one cut i* of peps_amplitude, E_loc(S) = diag(S) +
 * sum_S' <S|H|S'> Psi(S')_i* / Psi(S)_i*. The sampled mean over
 * p(S) ~ |Psi(S)_i*|^2 is then the energy of the single vector
 * S -> Psi(S)_i* and stays above the ground-state energy at any chi; the
 * strip ratios of peps_local_energy carry no such bound when chi truncates.
 * Cost: one amplitude per sample and per move of nonzero <S|H|S'> (moves
 * are the distinct sets of sites that an off-diagonal term changes), held
 * in the context's workspace. flags: int32 [n] or NULL, the OR of the flags
 * of S and of all its neighbours. Needs a Hamiltonian; PEPS_ERR_UNSUPPORTED
 * when n x (1 + moves) exceeds 2^31 - 1. Returns after the neighbour count
 * has been read back; the rest is queued on the stream. */
peps_status peps_local_energy_strict(peps_ctx* ctx, const double* theta,
                                     const uint8_t* samples, int n, double* eloc,
                                     int32_t* flags, void* stream);

/* Rotated-basis estimator (Sec. "On reusing environments and the convenient
 * treatment of long-range interactions"; App. "Sampling-based PEPS schemes
 * can yield a variational upper bound on the energy"): the terms of a
 * Hamiltonian split into sets that are each diagonal in one product basis
 * (a long-range Heisenberg model: the X X, Y Y and Z Z terms). For a set
 * diagonal in the eigenbasis of sigma^b, the PEPS U_b^(x N) Psi is sampled
 * and the set's diagonal form evaluated on its configurations; the sum over
 * the sets estimates <H> with no amplitude ratio.
 *
 * peps_rotate_basis writes the parameters of U_b^(x N) Psi: every site
 * tensor's physical index multiplied by U_b, T'[s] = sum_p U_b[s,p] T[p],
 * with U_x the Hadamard matrix (U_x X U_x^dagger = Z) and U_y = H S^dagger,
 * S = diag(1, i) (U_y Y U_y^dagger = Z); PEPS_BASIS_Z copies. theta and
 * theta_out: FP64 device arrays in the context's parameter layout ([N_p], or
 * [N_p][2] for complex contexts); they may be the same array. PEPS_BASIS_Y
 * needs a complex context (PEPS_ERR_UNSUPPORTED otherwise: the rotated
 * tensors are complex); another basis value is PEPS_ERR_ARG. Queued on
 * stream. */
#define PEPS_BASIS_Z 0
#define PEPS_BASIS_X 1
#define PEPS_BASIS_Y 2
peps_status peps_rotate_basis(peps_ctx* ctx, const double* theta, int basis, double* theta_out,
                              void* stream);

/* The diagonal part of the context's Hamiltonian on each configuration:
 * eloc[n][2] (re, im) FP64 device array, sum_t <S|h_t|S> + the long-range
 * pairs + the on-site table, no amplitude. With a Hamiltonian whose terms are
 * all diagonal (a set of the rotated-basis estimator in its rotated form)
 * this is the set's local energy. Needs a Hamiltonian (PEPS_ERR_ARG
 * otherwise). Queued on stream. */
peps_status peps_energy_diag(peps_ctx* ctx, const uint8_t* samples, int n, double* eloc,
                             void* stream);

/* Log-derivatives O_k(S) = d ln Psi_row(x)(S) / d theta_k for every
 * parameter k of a site (x, y) with physical index s_xy (the hole network
 * of row x between E^u[x-1] and E^l[x+1], divided by that strip's
 * amplitude); parameters with p != s_xy have O = 0 and are not stored.
 * O: compact [n][N_p/d] in FP64 (PEPS_F64), FP32 (PEPS_F32, PEPS_BF16),
 * interleaved FP64 pairs (PEPS_C128) or FP32 pairs (PEPS_C64), site-major
 * with the (l, r, u, d) entries of each site in C order. For complex
 * tensors O is the holomorphic derivative (no conjugation).
 * env_cache as for peps_local_energy. */
peps_status peps_logderiv(peps_ctx* ctx, const double* theta, const uint8_t* samples,
                          int n, const void* env_cache, void* O, void* stream);

/* Vector-Jacobian product of ln|Psi| over a batch (the backward pass of the
 * log-amplitude, Sec. "Finite PEPS and Sampling": dPsi/dT as a hole
 * network): grad_theta[k] = sum_s g[s] O_k(S_s) with O from peps_logderiv
 * (compact, compute precision) expanded with zeros where p != s_xy.
 * g: FP64 [n]; grad_theta: FP64 [N_p], overwritten. Complex parameters:
 * grad_theta is FP64 pairs [N_p][2] holding d/dRe theta_k + i d/dIm theta_k
 * of sum_s g[s] ln|Psi(S_s)|, which is sum_s g[s] conj(O_k(S_s)) since
 * ln|Psi| = Re ln Psi and ln Psi is holomorphic in theta. */
peps_status peps_logderiv_vjp(peps_ctx* ctx, const void* O, const uint8_t* samples, int n,
                              const double* g, double* grad_theta, void* stream);

/* Fused amplitude + local energy + log-derivatives of one batch, sharing the
 * environments and the one-row strips between the three; outputs as in the
 * three calls above (any of eloc, O may be NULL). */
peps_status peps_evaluate(peps_ctx* ctx, const double* theta, const uint8_t* samples,
                          int n, double* logpsi, double* eloc, void* O, int32_t* flags,
                          void* stream);

/* minSR step (Eqs. tdvp, tdvp_fast). With O the compact log-derivatives of
 * peps_logderiv (expanded with zeros where p != s_xy) and E = eloc:
 *   Obar = (O - <O>)/sqrt(n), ebar = (E - <E>)/sqrt(n),
 *   T = Obar Obar^T (n x n, FP64),
 *   dtheta = Obar^T (T + eps I)^+ ebar,
 * where eigenvalues of T + eps I at or below rcond * (largest) are dropped
 * from the pseudo-inverse. The solver is chosen by peps_set_minsr_solver:
 *   PEPS_MINSR_CHOLESKY (default): a Cholesky factorisation of T + eps I,
 *     which equals the pseudo-inverse whenever no eigenvalue is dropped;
 *     that holds when trace(T) + eps <= eps / rcond, which is checked on
 *     the device. If the check fails diag[3] is set to 1 and dtheta is
 *     filled with NaN.
 *   PEPS_MINSR_EIGH: the eigendecomposition of T + eps I (the paper's
 *     solve): Householder tridiagonalisation, bisection, inverse iteration;
 *     n <= 3072 (PEPS_ERR_UNSUPPORTED above).
 *   PEPS_MINSR_AUTO: Cholesky, and the eigendecomposition when the
 *     certificate fails (n <= 3072; above that as CHOLESKY). Its kernels are
 *     queued every call and return at once when the certificate holds (a
 *     few microseconds each, three per sample row).
 * Real modes use the real part of eloc and give dtheta FP64 [N_p]. Complex
 * modes use the Hermitian forms T = Obar Obar^H,
 * dtheta = Obar^H (T + eps I)^+ ebar with complex ebar, and give dtheta as
 * interleaved FP64 pairs [N_p][2]. dtheta is the direction of Eq. tdvp:
 * theta moves as theta - tau * dtheta. A non-finite local energy is
 * reported on the device (diag[3] = 2, dtheta NaN); the call does not
 * synchronise.
 * diag (device, FP64 [8]): [0] trace(T)+eps (bound on the largest
 * eigenvalue), [1] eps, [2] number of dropped eigenvalues (0 unless the
 * eigendecomposition ran), [3] 1 if no valid step was formed (certificate
 * failed with no eigendecomposition), 2 for a non-finite local energy, 0
 * otherwise, [4] Re <E>, [5] mean |E - <E>|^2 (real modes: of Re E), [6] n,
 * [7] smallest Cholesky pivot (1e300 when no factorisation ran). */
peps_status minsr_step(peps_ctx* ctx, const void* O, const uint8_t* samples, int n,
                       const double* eloc, double eps, double rcond, double* dtheta,
                       double* diag, void* stream);

/* Solver of minsr_step (and of the step inside peps_vmc_step); the
 * eigendecomposition allocates n^2 FP64 of workspace on first use. */
#define PEPS_MINSR_CHOLESKY 0
#define PEPS_MINSR_EIGH 1
#define PEPS_MINSR_AUTO 2
peps_status peps_set_minsr_solver(peps_ctx* ctx, int solver);

/* minsr_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results as minsr_step with the Cholesky solver
 * (PEPS_ERR_UNSUPPORTED when another solver is set), with the workspace (column
 * means [N_p], T [n][n], solve vectors) in a fixed device array of 48 MiB
 * that the library holds on every GPU it runs on until the process ends.
 * Calls no allocator and does not synchronise; the inputs, outputs and
 * errors are those of minsr_step. PEPS_ERR_UNSUPPORTED when the workspace,
 * N_p * e + n * n * e + (2n + 2) * e + 144 bytes with e = 8 (real) or 16
 * (complex) each rounded up to 256, exceeds 48 MiB (e.g. n = 1024 with
 * complex parameters needs 16 MiB plus 16 N_p bytes). Every call on one GPU
 * uses that GPU's one array, which keeps the last call's contents: calls
 * that overlap on one GPU (other streams, other host threads) race. */
peps_status minsr_step_noalloc(peps_ctx* ctx, const void* O, const uint8_t* samples, int n,
                               const double* eloc, double eps, double rcond, double* dtheta,
                               double* diag, void* stream);

/* Sampling of p(S) ~ |Psi(S)|^2 by Markov chains (Sec. "On Direct
 * Sampling" names them as the alternative to direct sampling).
 * kind PEPS_SAMPLE_EXCHANGE: local exchanges of anti-aligned nearest
 * neighbours (S^z conserved, chains start with floor(N/2) up spins);
 * PEPS_SAMPLE_FLIP: single-site flips. A move is accepted iff
 * u < |Psi(S')/Psi(S)|^2 with the ratio taken in the strip holding the move
 * and u from Philox4x32-10 keyed by seed (counter: move id, sweep + offset,
 * chain, tag). A sweep visits every bond (site) once.
 * kind PEPS_SAMPLE_IMH: independence Metropolis-Hastings with the learned
 * proposal q of `proposal` (a made_ctx and its parameters): every step draws
 * one S' ~ q per chain (made_sample, offset + step), evaluates
 * ln Psi(S')_i* (peps_amplitude) and accepts iff
 * ln u < 2 (ln|Psi(S')| - ln|Psi(S)|) + ln q(S) - ln q(S') (imh_step);
 * chains start from proposal->init [n_chains][N] (device, e.g. local
 * samples) or, if NULL, from a draw of q; a "sweep" is one step.
 * Chain c writes samples[c*per_chain + j] = its state after sweep
 * burn_in + (j+1)*thin - 1; logpsi (device FP64 [n][2] or NULL) receives
 * (ln|Psi|, arg Psi) of every written sample (the local kinds evaluate it
 * with peps_amplitude after the chains). accepted: int32 [n_chains]
 * accepted-move counts (or NULL). proposal: required for IMH, ignored
 * otherwise. At most 1024 sites for the local kinds (PEPS_ERR_UNSUPPORTED
 * above). */
typedef struct made_ctx made_ctx;
typedef struct {
  made_ctx* made;          /* the proposal network */
  const float* params;     /* its FP32 parameters (device) */
  const uint8_t* init;     /* initial states [n_chains][N] (device) or NULL */
} peps_proposal;
enum { PEPS_SAMPLE_IMH = 2 };
peps_status peps_sample(peps_ctx* ctx, const double* theta, int kind, int n_chains,
                        int per_chain, int burn_in, int thin, uint64_t seed, uint64_t offset,
                        const peps_proposal* proposal, uint8_t* samples, double* logpsi,
                        int32_t* accepted, void* stream);

/* One step of the optimisation loop (Eq. tdvp iterated, as in the
 * optimisations of Sec. "Results"): n = n_chains * per_chain samples from
 * peps_sample (same arguments), ln Psi, E_loc and O on them as in
 * peps_evaluate, the minSR direction dtheta as in minsr_step (eps, rcond),
 * then theta <- theta - tau * dtheta on the device.
 * theta: device FP64 parameters (interleaved pairs for complex modes),
 *   updated in place; left unchanged, with PEPS_ERR_NONFINITE returned, if
 *   the minSR pseudo-inverse certificate fails.
 * samples: device uint8 [n][N] (written); eloc: device FP64 [n][2]
 *   (written); flags: device int32 [n] or NULL; diag: device FP64 [8] as
 *   in minsr_step ([4] is the batch mean of Re E_loc before the update).
 * The context's workspace holds O and dtheta (grown on demand). Returns
 * after the step has finished on the stream. Needs a Hamiltonian and
 * 2 <= n <= 2^24. */
peps_status peps_vmc_step(peps_ctx* ctx, double* theta, int kind, int n_chains, int per_chain,
                          int burn_in, int thin, uint64_t seed, uint64_t offset, double tau,
                          double eps, double rcond, uint8_t* samples, double* eloc,
                          int32_t* flags, double* diag, void* stream);

/* Kernel timing. With profiling enabled every kernel launch of the context
 * is bracketed by two HIP events on its launch stream. peps_profile_read
 * waits for the recorded events and returns, per kernel kind, the summed
 * milliseconds (ms[PEPS_PROF_KINDS], host FP64) and launch counts
 * (counts[PEPS_PROF_KINDS], host); reset != 0 clears the totals. */
enum {
  PEPS_PROF_ENV = 0,      /* boundary-MPS environments (both directions) */
  PEPS_PROF_OVERLAP = 1,  /* amplitude at the middle cut */
  PEPS_PROF_STRIP1 = 2,   /* one-row strips: ratios and log-derivatives */
  PEPS_PROF_STRIP2 = 3,   /* two-row strips: ratios */
  PEPS_PROF_ESUM = 4,     /* diagonal energy and the per-sample sum */
  PEPS_PROF_MINSR = 5,    /* the whole minSR step */
  PEPS_PROF_SAMPLE = 6,   /* Metropolis sweeps */
  PEPS_PROF_KINDS = 8
};
peps_status peps_profile(peps_ctx* ctx, int enable);
peps_status peps_profile_read(peps_ctx* ctx, double* ms, long* counts, int reset);

/* ------------------------------------------------------------------------
 * Learned proposal for independence Metropolis-Hastings (an extension: the
 * paper corrects approximate samples by importance weights, App. "direct
 * sampling of PEPS"; here the PEPS arbitrates every proposal through the
 * acceptance |Psi(S')|^2 q(S) / (|Psi(S)|^2 q(S'))).
 * q is a masked autoregressive network over the N sites in raster order with
 * one hidden ReLU layer of width H (H <= 256): hidden degrees
 * m(k) = (k mod (N-1)) + 1, input mask [m(k) >= n+1], output mask
 * [n+1 > m(k)], p(s_n = 1 | s_<n) = sigmoid(logit_n). With n_up >= 0 every
 * configuration has exactly n_up zeros: a site is forced once the zeros or
 * the ones are used up and then contributes a factor 1 to q.
 * Parameters: FP32 device vector W1 [H][N], b1 [H], W2 [N][H], b2 [N];
 * with bf16 != 0 the weights are rounded to bfloat16 where they enter a
 * product (FP32 accumulation). Configurations: uint8 [n][N] device.
 * ---------------------------------------------------------------------- */
peps_status made_create(int N, int H, int n_up, int bf16, made_ctx** out);
void made_destroy(made_ctx* m);
size_t made_num_params(const made_ctx* m);
/* loss = -mean_b ln q(x_b) (device FP64 scalar) and its gradient (device
 * FP32, parameter layout) for a batch of B configurations. */
peps_status made_loss_grad(made_ctx* m, const float* params, const uint8_t* x, int B,
                           float* grads, double* loss, void* stream);
/* One Adam step (Kingma and Ba) on params with moments mom, var (device
 * FP32, same layout), step counter t >= 1. */
peps_status made_adam_step(made_ctx* m, float* params, const float* grads, float* mom,
                           float* var, int t, double lr, double beta1, double beta2, double eps,
                           void* stream);
/* `steps` Adam steps of mini-batch training on data (device uint8 [M][N]):
 * step i takes the batch of `batch` rows at positions i*batch ..
 * (i+1)*batch - 1 of a sequence of epochs, epoch e visiting row
 * (a_e r + c_e) mod M at its position r, with (a_e, c_e) drawn from
 * splitmix64 seeded by `seed` (a_e coprime with M: a permutation); then the
 * loss and gradient of made_loss_grad and the Adam update of
 * made_adam_step with step counter t0 + i + 1. losses: device FP64
 * [steps], the batch loss of every step. Queued on the stream; the
 * permutation table is copied from host memory the context keeps. */
peps_status made_train(made_ctx* m, float* params, const uint8_t* data, int M, int steps,
                       int batch, int t0, double lr, double beta1, double beta2, double eps,
                       uint64_t seed, float* mom, float* var, double* losses, void* stream);
/* Draw n configurations from q site by site (uniforms from Philox4x32-10,
 * counter (site, sample, offset, tag)) with their ln q (device FP64 [n]). */
peps_status made_sample(made_ctx* m, const float* params, int n, uint64_t seed, uint64_t offset,
                        uint8_t* out, double* logq, void* stream);
/* ln q of given configurations (device FP64 [n]). */
peps_status made_logq(made_ctx* m, const float* params, const uint8_t* x, int n, double* logq,
                      void* stream);
/* Integrated autocorrelation time and effective sample size of a scalar
 * series observed on n_chains chains of length T (device FP64
 * [n_chains][T], e.g. E_loc along each chain): rho(t) averaged over the
 * chains, centred on the mean over all observations (chains that start
 * stationary), tau(W) = 1 + 2 sum_{t=1..W} rho(t) with Sokal's automatic
 * window (the smallest W >= c tau(W)); ranked != 0 first replaces the
 * values by the normal scores Phi^-1((r - 3/8) / (S + 1/4)) of their pooled
 * ranks (average ranks for ties, S = n_chains T), the rank-normalised form
 * that heavy-tailed local energies need. out: device FP64 [2] = (tau_int,
 * S / tau_int); work: device FP64 [S + T]. At most 2^24 observations
 * (PEPS_ERR_UNSUPPORTED); ranked costs O(S^2) comparisons. */
peps_status peps_tau_int(const double* series, int n_chains, int T, int ranked, double c,
                         double* work, double* out, void* stream);
/* One independence Metropolis-Hastings step for n_chains chains: chain c
 * moves to prop[c] iff ln u < 2 (ln|Psi(prop)| - ln|Psi(state)|)
 * + ln q(state) - ln q(prop), u from Philox (counter: chain, step, 0, tag).
 * state_logpsi / prop_logpsi are [n][2] (ln|Psi|, arg) as from
 * peps_amplitude; accepted[c] is incremented on acceptance (or NULL). */
peps_status imh_step(int n_chains, int N, uint8_t* state, double* state_logpsi,
                     double* state_logq, const uint8_t* prop, const double* prop_logpsi,
                     const double* prop_logq, uint64_t seed, uint64_t step, int32_t* accepted,
                     void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PEPSMIN_H */
