// C-ABI of the library: argument validation, lattice tables, the
// Hamiltonian term compiler, workspace management and stream-ordered
// launches. Declared in include/pepsmin.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pepsmin.h"
#include "common.h"
#include "kernels.h"

using namespace pm;

namespace {

thread_local std::string g_err;

peps_status fail(peps_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(PEPS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

// A device buffer that only grows.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  peps_status ensure(size_t bytes) {
    if (bytes <= cap) return PEPS_OK;
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
      return fail(PEPS_ERR_OOM, "hipMalloc of %zu bytes failed", bytes);
    }
    cap = bytes;
    return PEPS_OK;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

}  // namespace

// Workspace of the allocation-free minSR entry point: one array per GPU,
// held until the process ends. Its name is a host-side stand-in; kernels get
// the device address resolved per device by scratch_ptr().
#define PEPS_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)
__device__ __align__(256) unsigned char scratch[PEPS_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scr_mu;
void* g_scr_ptr[64] = {};

// Device address of `scratch` on the current device, resolved once per
// device with that device current.
peps_status scratch_ptr(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(PEPS_ERR_UNSUPPORTED, "device index %d above 63", dev);
  std::lock_guard<std::mutex> lk(g_scr_mu);
  if (!g_scr_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PEPS_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scr_ptr[dev] = p;
  }
  *out = g_scr_ptr[dev];
  return PEPS_OK;
}

}  // namespace

struct peps_ctx {
  peps_geom g;
  Lattice L;
  std::vector<int> tab;  // host copy
  int* d_tab = nullptr;
  size_t tsize = 8;      // bytes per compute element
  int icut = 0;
  // Hamiltonian
  bool has_ham = false;
  HamDev H{};
  int* d_hint = nullptr;
  double* d_hdbl = nullptr;
  // workspace
  DevBuf theta_c, env_int, rscr, rt1, rt2, epart, bad, mean, Tm, vec, eloc_tmp, logpsi_tmp;
  // optimisation step: O, dtheta and ln Psi of its batch
  DevBuf vmc_O, vmc_dth, vmc_lp;
  // strict local energy: neighbour counts/offsets, the amplitude batch
  // [samples | neighbours], coefficients, ln Psi and flags of the batch
  int n_moves = 0;
  DevBuf str_idx, str_batch, str_coef, str_lp, str_fl;
  // direct sampler: the double-layer context (D^2 lattice, bond chi_d) and
  // its parameters, environments and dummy configuration; the row kernel's
  // slabs, ln Psi and amplitude flags of the drawn batch
  peps_ctx* dbl = nullptr;
  int dbl_chi = 0;
  bool dbl_built = false;  // dir_env2 holds D^l of the last refresh
  // environments from the bottom only (the double-layer context)
  bool bottom_only = false;
  DevBuf dir_th2, dir_zero, dir_env2, dir_lp2, dir_slab, dir_lp, dir_fl;
  // global working sets of the kernels whose matrices do not fit in LDS
  bool env_gm = false, s1_gm = false, s2_gm = false, smp_gm = false;
  // truncation: canonical QR -> SVD (0) or the density-matrix algorithm on
  // the matrix cores (1); dm_ok: the shape fits the density-matrix kernel
  int compress = 0;
  bool dm_ok = false;
  DevBuf gws_dm;
  // minSR solve: certified Cholesky, eigendecomposition, or Cholesky with the
  // eigendecomposition after a failed certificate; its workspace
  int minsr_solver = PEPS_MINSR_CHOLESKY;
  DevBuf eig_ws;
  // independence MH chains: states, proposals, their ln Psi and ln q
  DevBuf imh_st, imh_pr, imh_stlp, imh_stlq, imh_prlp, imh_prlq;
  DevBuf gws_env, gws_s1, gws_s2, gws_smp;
  DevBuf smp_state;  // chain states and acceptance counts between the sampler's phases
  int jac_sweeps = 40;
  // optional per-kernel timing with HIP events on the launch stream
  bool prof = false;
  struct Ev { hipEvent_t a, b; int kind; };
  std::vector<Ev> pending;
  double prof_ms[PEPS_PROF_KINDS] = {};
  long prof_n[PEPS_PROF_KINDS] = {};
  size_t chunk_budget = (size_t)48 << 30;  // bytes of per-chunk scratch
};

struct made_ctx {
  int N, H, n_up, bf16;
  DevBuf a, lg, dlg, da, logq;
  // training: the gathered batch, the gradient and the per-epoch
  // permutations (a, c)
  DevBuf xb, gr, ptab;
  std::vector<unsigned long long> hptab;
};

// Bracket one launch with events when profiling is on.
struct ProfScope {
  peps_ctx* c;
  hipStream_t st;
  int kind;
  hipEvent_t a{}, b{};
  ProfScope(peps_ctx* c_, hipStream_t st_, int kind_) : c(c_), st(st_), kind(kind_) {
    if (c->prof) {
      hipEventCreate(&a);
      hipEventCreate(&b);
      hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (c->prof) {
      hipEventRecord(b, st);
      c->pending.push_back({a, b, kind});
    }
  }
};

static size_t elem_bytes(int dtype) { return mode_elem_bytes(dtype); }
static bool is_complex(int dtype) { return dtype == PEPS_C128 || dtype == PEPS_C64; }
// dynamic LDS a workgroup may request (the static arrays take the rest of 160 KiB)
static const size_t kLdsDyn = 150 * 1024;

static size_t env_tensor_elems_per_sample(const Lattice& L) {
  return (size_t)L.n_slots * L.Ly * L.site_box;
}

static peps_status build_tables(peps_ctx* c) {
  const peps_geom& g = c->g;
  const int Lx = g.Lx, Ly = g.Ly, D = g.D, N = Lx * Ly;
  Lattice& L = c->L;
  L.Lx = Lx;
  L.Ly = Ly;
  L.D = D;
  L.chi = g.chi;
  L.N = N;
  L.trunc_w = 0.0;
  L.bmax = std::max(g.chi, D);
  L.site_box = L.bmax * D * L.bmax;
  L.n_slots = 2 * (Lx - 1);
  std::vector<int> poff(N), blk(N), legs(4 * N), coff(N);
  int off = 0, coffs = 0;
  for (int x = 0; x < Lx; ++x)
    for (int y = 0; y < Ly; ++y) {
      const int n = x * Ly + y;
      const int Dl = y == 0 ? 1 : D, Dr = y == Ly - 1 ? 1 : D;
      const int Du = x == 0 ? 1 : D, Dd = x == Lx - 1 ? 1 : D;
      legs[4 * n] = Dl;
      legs[4 * n + 1] = Dr;
      legs[4 * n + 2] = Du;
      legs[4 * n + 3] = Dd;
      blk[n] = Dl * Dr * Du * Dd;
      poff[n] = off;
      coff[n] = coffs;
      off += g.d * blk[n];
      coffs += blk[n];
    }
  L.n_params = off;
  L.n_compact = coffs;
  std::vector<int> csite(coffs);
  for (int n = 0; n < N; ++n)
    for (int j = 0; j < blk[n]; ++j) csite[coff[n] + j] = n;
  // environment dims: simulate both sweeps
  std::vector<int> ed((size_t)L.n_slots * Ly * 3, 1);
  auto set = [&](int slot, int y, int a, int k, int b) {
    ed[((size_t)slot * Ly + y) * 3 + 0] = a;
    ed[((size_t)slot * Ly + y) * 3 + 1] = k;
    ed[((size_t)slot * Ly + y) * 3 + 2] = b;
  };
  auto get = [&](int slot, int y, int i) { return ed[((size_t)slot * Ly + y) * 3 + i]; };
  for (int dir = 0; dir < 2; ++dir) {
    const int x0 = dir ? Lx - 1 : 0;
    const int s0 = dir ? (Lx - 1) + (Lx - 2) : 0;
    for (int y = 0; y < Ly; ++y) {
      const int n = x0 * Ly + y;
      set(s0, y, legs[4 * n], dir ? legs[4 * n + 2] : legs[4 * n + 3], legs[4 * n + 1]);
    }
    for (int t = 1; t <= Lx - 2; ++t) {
      const int x = dir ? Lx - 1 - t : t;
      const int sp = dir ? (Lx - 1) + (x + 1 - 1) : x - 1;
      const int sn = dir ? (Lx - 1) + (x - 1) : x;
      std::vector<int> kk(Ly, 0);
      int kp = 1;
      for (int y = 0; y < Ly - 1; ++y) {
        const int n = x * Ly + y;
        const int kout = dir ? legs[4 * n + 2] : legs[4 * n + 3];
        const int Pr = get(sp, y, 2) * legs[4 * n + 1];
        kk[y] = std::min(kp * kout, Pr);
        kp = kk[y];
      }
      int nbr = 1;
      for (int y = Ly - 1; y >= 0; --y) {
        const int n = x * Ly + y;
        const int kout = dir ? legs[4 * n + 2] : legs[4 * n + 3];
        const int zc = kout * nbr;
        int r = 1;
        if (y > 0) r = std::min(std::min(g.chi, kk[y - 1]), zc);
        set(sn, y, r, kout, nbr);
        nbr = r;
      }
    }
  }
  // concatenate
  std::vector<int>& tab = c->tab;
  tab.clear();
  L.off_param = (int)tab.size();
  tab.insert(tab.end(), poff.begin(), poff.end());
  L.off_block = (int)tab.size();
  tab.insert(tab.end(), blk.begin(), blk.end());
  L.off_legs = (int)tab.size();
  tab.insert(tab.end(), legs.begin(), legs.end());
  L.off_compact = (int)tab.size();
  tab.insert(tab.end(), coff.begin(), coff.end());
  L.off_env = (int)tab.size();
  tab.insert(tab.end(), ed.begin(), ed.end());
  L.off_csite = (int)tab.size();
  tab.insert(tab.end(), csite.begin(), csite.end());
  HIPCHK(hipMalloc(&c->d_tab, tab.size() * sizeof(int)));
  HIPCHK(hipMemcpy(c->d_tab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
  return PEPS_OK;
}

extern "C" {

const char* peps_last_error(void) { return g_err.c_str(); }

peps_status peps_create(const peps_geom* geom, peps_ctx** out) {
  if (!geom || !out) return fail(PEPS_ERR_ARG, "null geometry or output pointer");
  *out = nullptr;
  const peps_geom& g = *geom;
  if (g.Lx < 2 || g.Ly < 2 || g.Lx > 32 || g.Ly > 32)
    return fail(PEPS_ERR_ARG, "lattice %dx%d outside 2..32", g.Lx, g.Ly);
  if (g.d != 2) return fail(PEPS_ERR_UNSUPPORTED, "physical dimension %d (only d = 2)", g.d);
  if (g.D < 1 || g.chi < 1) return fail(PEPS_ERR_ARG, "D = %d, chi = %d must be >= 1", g.D, g.chi);
  if (g.dtype < PEPS_F64 || g.dtype > PEPS_C64) return fail(PEPS_ERR_ARG, "unknown dtype %d", g.dtype);
  const int bmax = std::max(g.chi, g.D);
  // the Householder and the cut selection index at most 256 columns / rows
  if (bmax * g.D > 256)
    return fail(PEPS_ERR_UNSUPPORTED, "chi*D = %d above the limit 256", bmax * g.D);
  if (g.D > 16) return fail(PEPS_ERR_UNSUPPORTED, "D = %d above 16", g.D);
  const size_t eb = elem_bytes(g.dtype);
  peps_ctx* c = new peps_ctx();
  c->g = g;
  c->tsize = eb;
  c->icut = g.Lx / 2 - 1;
  peps_status st = build_tables(c);
  if (st != PEPS_OK) {
    peps_destroy(c);
    return st;
  }
  c->env_gm = env_lds_bytes(g.dtype, c->L, false) > kLdsDyn;
  c->s1_gm = strip1_lds_bytes(g.dtype, c->L, false) > kLdsDyn;
  c->s2_gm = strip2_lds_bytes(g.dtype, c->L, false) > kLdsDyn;
  c->smp_gm = sample_lds_bytes(g.dtype, c->L, false) > kLdsDyn;
  {
    void* sp = nullptr;
    if ((st = scratch_ptr(&sp)) != PEPS_OK) {
      peps_destroy(c);
      return st;
    }
  }
  c->dm_ok = env_dm_lds_bytes(c->L, g.dtype) <= kLdsDyn && g.chi + 1 <= 256 &&
             ((c->L.bmax * g.D + 31) / 32 * 32) <= 256;
  *out = c;
  return PEPS_OK;
}

void peps_destroy(peps_ctx* c) {
  if (!c) return;
  if (c->d_tab) hipFree(c->d_tab);
  if (c->d_hint) hipFree(c->d_hint);
  if (c->d_hdbl) hipFree(c->d_hdbl);
  DevBuf* bufs[] = {&c->theta_c, &c->env_int,   &c->rscr,       &c->rt1,    &c->rt2,
                    &c->epart,   &c->bad,       &c->mean,       &c->Tm,     &c->vec,
                    &c->eloc_tmp, &c->logpsi_tmp, &c->gws_env,   &c->gws_s1, &c->gws_s2,
                    &c->gws_smp, &c->vmc_O,      &c->vmc_dth,    &c->vmc_lp,
                    &c->str_idx, &c->str_batch,  &c->str_coef,   &c->str_lp, &c->str_fl,
                    &c->dir_th2, &c->dir_zero,   &c->dir_env2,   &c->dir_lp2, &c->dir_slab,
                    &c->dir_lp,  &c->dir_fl,    &c->gws_dm,
                    &c->imh_st,  &c->imh_pr,    &c->imh_stlp,   &c->imh_stlq, &c->imh_prlp,
                    &c->imh_prlq, &c->eig_ws,   &c->smp_state};
  if (c->dbl) peps_destroy(c->dbl);
  for (DevBuf* b : bufs) b->release();
  delete c;
}

size_t peps_num_params(const peps_ctx* c) { return c ? (size_t)c->L.n_params : 0; }

size_t peps_env_cache_bytes(const peps_ctx* c, int n) {
  if (!c || n < 0) return 0;
  return (size_t)n * env_tensor_elems_per_sample(c->L) * c->tsize +
         (size_t)n * c->L.n_slots * sizeof(double);
}

peps_status peps_set_hamiltonian(peps_ctx* c, int n_terms, const int* term_nsites,
                                 const int* term_sites, const double* term_mats, int n_pairs,
                                 const int* pair_ij, const double* pair_v, const double* onsite) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (n_terms < 0 || n_pairs < 0) return fail(PEPS_ERR_ARG, "negative term or pair count");
  if (n_terms > 0 && (!term_nsites || !term_sites || !term_mats))
    return fail(PEPS_ERR_ARG, "null term arrays");
  if (n_pairs > 0 && (!pair_ij || !pair_v)) return fail(PEPS_ERR_ARG, "null pair arrays");
  const Lattice& L = c->L;
  const int Ly = L.Ly, N = L.N;
  struct Move {
    int x, two, y0, y1, ns, site[3];
    std::vector<int> contrib;  // (term, mask) pairs
  };
  std::map<std::vector<int>, int> index;
  std::vector<Move> moves;
  for (int t = 0; t < n_terms; ++t) {
    const int k = term_nsites[t];
    if (k < 1 || k > 3) return fail(PEPS_ERR_ARG, "term %d acts on %d sites (1..3)", t, k);
    for (int j = 0; j < k; ++j) {
      const int sj = term_sites[3 * t + j];
      if (sj < 0 || sj >= N) return fail(PEPS_ERR_ARG, "term %d site %d out of range", t, sj);
      for (int i = 0; i < j; ++i)
        if (term_sites[3 * t + i] == sj) return fail(PEPS_ERR_ARG, "term %d repeats site %d", t, sj);
    }
    const double* h = term_mats + (size_t)t * 128;
    const int dim = 1 << k;
    for (int i = 0; i < 128; ++i)
      if (!std::isfinite(h[i])) return fail(PEPS_ERR_NONFINITE, "term %d matrix not finite", t);
    for (int mask = 1; mask < dim; ++mask) {
      bool nz = false;
      for (int cc = 0; cc < dim && !nz; ++cc) {
        const int c2 = cc ^ mask;
        nz = h[(cc * 8 + c2) * 2] != 0.0 || h[(cc * 8 + c2) * 2 + 1] != 0.0;
      }
      if (!nz) continue;
      std::vector<int> sites;
      for (int j = 0; j < k; ++j)
        if ((mask >> (k - 1 - j)) & 1) sites.push_back(term_sites[3 * t + j]);
      std::sort(sites.begin(), sites.end());
      auto it = index.find(sites);
      int id;
      if (it == index.end()) {
        Move m;
        int xmin = 1 << 30, xmax = -1, ymin = 1 << 30, ymax = -1;
        for (int sidx : sites) {
          xmin = std::min(xmin, sidx / Ly);
          xmax = std::max(xmax, sidx / Ly);
          ymin = std::min(ymin, sidx % Ly);
          ymax = std::max(ymax, sidx % Ly);
        }
        if (xmax - xmin > 1)
          return fail(PEPS_ERR_UNSUPPORTED,
                      "term %d changes sites on rows %d..%d (at most two adjacent rows)", t, xmin,
                      xmax);
        m.x = xmin;
        m.two = xmax > xmin;
        if (m.two && xmin >= L.Lx - 1) return fail(PEPS_ERR_ARG, "bad row pair");
        m.y0 = ymin;
        m.y1 = ymax;
        m.ns = (int)sites.size();
        for (int j = 0; j < 3; ++j) m.site[j] = j < m.ns ? sites[j] : -1;
        id = (int)moves.size();
        moves.push_back(m);
        index[sites] = id;
      } else {
        id = it->second;
      }
      moves[id].contrib.push_back(t);
      moves[id].contrib.push_back(mask);
    }
  }
  // group by strip, sort by first column
  const int n_strips = L.Lx + (L.Lx - 1);
  std::vector<std::vector<int>> by(n_strips);
  for (int i = 0; i < (int)moves.size(); ++i)
    by[moves[i].two ? L.Lx + moves[i].x : moves[i].x].push_back(i);
  std::vector<int> mstart(n_strips + 1, 0), mv, contrib;
  for (int s = 0; s < n_strips; ++s) {
    std::stable_sort(by[s].begin(), by[s].end(),
                     [&](int a, int b) { return moves[a].y0 < moves[b].y0; });
    mstart[s] = (int)(mv.size() / 8);
    for (int i : by[s]) {
      const Move& m = moves[i];
      mv.push_back(m.y0);
      mv.push_back(m.y1);
      mv.push_back(m.ns);
      for (int j = 0; j < 3; ++j) mv.push_back(m.site[j]);
      mv.push_back((int)(contrib.size() / 2));
      mv.push_back((int)(m.contrib.size() / 2));
      contrib.insert(contrib.end(), m.contrib.begin(), m.contrib.end());
    }
  }
  mstart[n_strips] = (int)(mv.size() / 8);
  std::vector<int> terms(4 * (size_t)n_terms, -1);
  for (int t = 0; t < n_terms; ++t) {
    terms[4 * t] = term_nsites[t];
    for (int j = 0; j < term_nsites[t]; ++j) terms[4 * t + 1 + j] = term_sites[3 * t + j];
  }
  std::vector<int> pairs(2 * (size_t)n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    const int i = pair_ij[2 * p], j = pair_ij[2 * p + 1];
    if (i < 0 || j < 0 || i >= N || j >= N) return fail(PEPS_ERR_ARG, "pair %d out of range", p);
    if (!std::isfinite(pair_v[p])) return fail(PEPS_ERR_NONFINITE, "pair %d value not finite", p);
    pairs[2 * p] = i;
    pairs[2 * p + 1] = j;
  }
  // upload: ints = mstart | moves | contrib | terms | pairs; doubles = mats | pair_v | onsite
  std::vector<int> ints;
  const size_t o_ms = 0;
  ints.insert(ints.end(), mstart.begin(), mstart.end());
  const size_t o_mv = ints.size();
  ints.insert(ints.end(), mv.begin(), mv.end());
  const size_t o_ct = ints.size();
  ints.insert(ints.end(), contrib.begin(), contrib.end());
  const size_t o_tm = ints.size();
  ints.insert(ints.end(), terms.begin(), terms.end());
  const size_t o_pr = ints.size();
  ints.insert(ints.end(), pairs.begin(), pairs.end());
  ints.push_back(0);
  std::vector<double> dbl;
  dbl.insert(dbl.end(), term_mats, term_mats + (size_t)n_terms * 128);
  const size_t o_pv = dbl.size();
  dbl.insert(dbl.end(), pair_v, pair_v + n_pairs);
  const size_t o_on = dbl.size();
  if (onsite) {
    for (int i = 0; i < 2 * N; ++i)
      if (!std::isfinite(onsite[i])) return fail(PEPS_ERR_NONFINITE, "onsite not finite");
    dbl.insert(dbl.end(), onsite, onsite + 2 * N);
  }
  dbl.push_back(0.0);
  if (c->d_hint) hipFree(c->d_hint);
  if (c->d_hdbl) hipFree(c->d_hdbl);
  c->d_hint = nullptr;
  c->d_hdbl = nullptr;
  HIPCHK(hipMalloc(&c->d_hint, ints.size() * sizeof(int)));
  HIPCHK(hipMalloc(&c->d_hdbl, dbl.size() * sizeof(double)));
  HIPCHK(hipMemcpy(c->d_hint, ints.data(), ints.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->d_hdbl, dbl.data(), dbl.size() * sizeof(double), hipMemcpyHostToDevice));
  HamDev& H = c->H;
  H.n_strips = n_strips;
  H.n_terms = n_terms;
  H.n_pairs = n_pairs;
  H.mstart = c->d_hint + o_ms;
  H.moves = c->d_hint + o_mv;
  H.contrib = c->d_hint + o_ct;
  H.terms = c->d_hint + o_tm;
  H.pair_ij = c->d_hint + o_pr;
  H.mats = c->d_hdbl;
  H.pair_v = c->d_hdbl + o_pv;
  H.onsite = onsite ? c->d_hdbl + o_on : nullptr;
  c->n_moves = mstart[n_strips];
  c->has_ham = true;
  return PEPS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// internal drivers
// ---------------------------------------------------------------------------
// theta in the compute type. sync: check it on the host (synchronises the
// stream) and fail with PEPS_ERR_NONFINITE; otherwise the non-finite flag
// stays on the device (c->bad) for launch_flag_bad.
static peps_status prepare_theta(peps_ctx* c, const double* theta, hipStream_t st,
                                 bool sync = true) {
  const int np = c->L.n_params;
  peps_status s = c->theta_c.ensure((size_t)np * c->tsize);
  if (s != PEPS_OK) return s;
  s = c->bad.ensure(64);
  if (s != PEPS_OK) return s;
  HIPCHK(hipMemsetAsync(c->bad.p, 0, sizeof(int), st));
  HIPCHK(launch_convert_theta(c->g.dtype == PEPS_BF16 ? MODE_F32 : c->g.dtype, theta,
                              c->theta_c.p, np, (int*)c->bad.p, st));
  if (!sync) return PEPS_OK;
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, c->bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad) return fail(PEPS_ERR_NONFINITE, "theta contains non-finite values");
  return PEPS_OK;
}

// Device bytes one sample needs per evaluation chunk: R factors, strip right
// partials, the global working sets of kernels that do not fit in LDS and,
// when the caller keeps no cache, its environments.
static size_t per_sample_scratch(const peps_ctx* c, bool env_internal) {
  const Lattice& L = c->L;
  const size_t BD = (size_t)L.bmax * L.D;
  const size_t box = L.site_box;
  const size_t box2 = (size_t)L.bmax * L.bmax * L.D * L.D;
  const bool dm = c->compress == PEPS_COMPRESS_DENSMAT;
  size_t r = dm ? 0 : 2 * (size_t)L.Ly * BD * BD;
  size_t s1 = (size_t)L.Lx * (L.Ly + 1) * box;
  size_t s2 = (size_t)(L.Lx - 1) * (L.Ly + 1) * box2;
  size_t g = 0;
  if (c->env_gm && !dm) g += 2 * env_slab_elems(L, c->g.dtype);
  if (c->s1_gm) g += (size_t)L.Lx * strip1_slab_elems(L);
  if (c->s2_gm) g += (size_t)(L.Lx - 1) * strip2_slab_elems(L, c->g.dtype);
  size_t e = env_internal ? env_tensor_elems_per_sample(L) : 0;
  return (r + s1 + s2 + g + e) * c->tsize + (env_internal ? L.n_slots * sizeof(double) : 0);
}

static int chunk_size(const peps_ctx* c, int n, bool env_internal) {
  const size_t per = per_sample_scratch(c, env_internal);
  size_t ch = c->chunk_budget / (per ? per : 1);
  if (ch < 16) ch = 16;
  if (ch >= (size_t)n) return n;
  // equal chunks: no small tail launch
  const size_t nch = ((size_t)n + ch - 1) / ch;
  return (int)(((size_t)n + nch - 1) / nch);
}

// environments of one chunk of m samples
template <int M>
static peps_status run_envs(peps_ctx* c, const uint8_t* samples, int m, char* env_t,
                            double* env_l, int* flags, hipStream_t st) {
  const Lattice& L = c->L;
  const size_t BD = (size_t)L.bmax * L.D;
  peps_status s;
  if (c->compress == PEPS_COMPRESS_DENSMAT) {
    const int grid = env_dm_grid(L, c->g.dtype, m * (c->bottom_only ? 1 : 2));
    if ((s = c->gws_dm.ensure((size_t)grid * env_dm_slab_elems(L, c->g.dtype) * c->tsize)) !=
        PEPS_OK)
      return s;
    ProfScope ps(c, st, PEPS_PROF_ENV);
    HIPCHK(launch_env_dm<M>(L, c->d_tab, c->theta_c.p, samples, env_t, env_l, flags, m,
                            c->gws_dm.p, grid, st, c->bottom_only));
    return PEPS_OK;
  }
  s = c->rscr.ensure((size_t)m * 2 * L.Ly * BD * BD * c->tsize);
  if (s != PEPS_OK) return s;
  void* gws = nullptr;
  if (c->env_gm) {
    if ((s = c->gws_env.ensure((size_t)m * 2 * env_slab_elems(L, c->g.dtype) * c->tsize)) != PEPS_OK) return s;
    gws = c->gws_env.p;
  }
  ProfScope ps(c, st, PEPS_PROF_ENV);
  HIPCHK(launch_env_sweep<M>(L, c->d_tab, c->theta_c.p, samples, env_t, env_l, c->rscr.p, flags,
                             m, c->jac_sweeps, gws, st, c->bottom_only));
  return PEPS_OK;
}

// strips of one chunk of m samples
template <int M>
static peps_status run_strips(peps_ctx* c, const uint8_t* sm, int m, const char* et,
                              double* eloc, void* O, int* flags, hipStream_t st) {
  const Lattice& L = c->L;
  const size_t box = L.site_box;
  const size_t box2 = (size_t)L.bmax * L.bmax * L.D * L.D;
  const int nparts = 1 + L.Lx + (L.Lx - 1);
  const bool want_e = eloc != nullptr;
  const bool want_o = O != nullptr;
  peps_status s = c->rt1.ensure((size_t)m * L.Lx * (L.Ly + 1) * box * c->tsize);
  if (s != PEPS_OK) return s;
  void* g1 = nullptr;
  void* g2 = nullptr;
  if (c->s1_gm) {
    if ((s = c->gws_s1.ensure((size_t)m * L.Lx * strip1_slab_elems(L) * c->tsize)) != PEPS_OK)
      return s;
    g1 = c->gws_s1.p;
  }
  HamDev H = c->H;
  if (!c->has_ham) H = HamDev{};
  if (want_e) {
    s = c->rt2.ensure((size_t)m * (L.Lx - 1) * (L.Ly + 1) * box2 * c->tsize);
    if (s != PEPS_OK) return s;
    s = c->epart.ensure((size_t)m * nparts * 2 * sizeof(double));
    if (s != PEPS_OK) return s;
    if (c->s2_gm && H.n_strips) {
      if ((s = c->gws_s2.ensure((size_t)m * (L.Lx - 1) * strip2_slab_elems(L, c->g.dtype) * c->tsize)) !=
          PEPS_OK)
        return s;
      g2 = c->gws_s2.p;
    }
  }
  if (want_e) HIPCHK(hipMemsetAsync(c->epart.p, 0, (size_t)m * nparts * 2 * sizeof(double), st));
  {
    ProfScope ps(c, st, PEPS_PROF_STRIP1);
    HIPCHK(launch_strip1<M>(L, c->d_tab, c->theta_c.p, sm, et, H, c->rt1.p, (double*)c->epart.p,
                            O, flags, m, want_e, want_o, g1, st));
  }
  if (want_e) {
    if (H.n_strips) {
      ProfScope ps(c, st, PEPS_PROF_STRIP2);
      HIPCHK(launch_strip2<M>(L, c->d_tab, c->theta_c.p, sm, et, H, c->rt2.p,
                              (double*)c->epart.p, flags, m, g2, st));
    }
    ProfScope ps(c, st, PEPS_PROF_ESUM);
    HIPCHK(launch_energy_diag_sum(L, H, sm, (const double*)c->epart.p, nparts, eloc, m, st));
  }
  return PEPS_OK;
}

static peps_status check_common(peps_ctx* c, const double* theta, const uint8_t* samples, int n) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (!theta) return fail(PEPS_ERR_ARG, "null theta");
  if (n < 0) return fail(PEPS_ERR_ARG, "negative sample count");
  if (n > 0 && !samples) return fail(PEPS_ERR_ARG, "null samples");
  return PEPS_OK;
}

// Every requested output of n samples, chunk by chunk: environments (unless
// the caller's cache already holds them), the amplitude, then the strips.
// Without a caller cache the environments of one chunk live in the
// context's workspace only, so the batch size is not bounded by memory.
template <int M>
static peps_status evaluate_impl(peps_ctx* c, const double* theta, const uint8_t* samples, int n,
                                 void* env_cache, bool env_given, double* logpsi, double* eloc,
                                 void* O, int* flags, hipStream_t st) {
  (void)theta;
  const Lattice& L = c->L;
  const size_t per_t = env_tensor_elems_per_sample(L) * c->tsize;
  const bool internal = env_cache == nullptr;
  const int ch = chunk_size(c, n, internal);
  char* cache_t = nullptr;
  double* cache_l = nullptr;
  if (internal) {
    peps_status s = c->env_int.ensure((size_t)ch * (per_t + L.n_slots * sizeof(double)));
    if (s != PEPS_OK) return s;
  } else {
    cache_t = (char*)env_cache;
    cache_l = (double*)((char*)env_cache + (size_t)n * per_t);
  }
  if (flags) HIPCHK(hipMemsetAsync(flags, 0, (size_t)n * sizeof(int32_t), st));
  const size_t ob = c->tsize;  // bytes of one O entry
  for (int c0 = 0; c0 < n; c0 += ch) {
    const int m = std::min(ch, n - c0);
    const uint8_t* sm = samples + (size_t)c0 * L.N;
    char* et;
    double* el;
    if (internal) {
      et = (char*)c->env_int.p;
      el = (double*)((char*)c->env_int.p + (size_t)m * per_t);
    } else {
      et = cache_t + (size_t)c0 * per_t;
      el = cache_l + (size_t)c0 * L.n_slots;
    }
    int* fl = flags ? flags + c0 : nullptr;
    if (!env_given) {
      peps_status s = run_envs<M>(c, sm, m, et, el, fl, st);
      if (s != PEPS_OK) return s;
    }
    if (logpsi) {
      ProfScope ps(c, st, PEPS_PROF_OVERLAP);
      HIPCHK(launch_overlap<M>(L, c->d_tab, et, el, c->icut, logpsi + (size_t)c0 * 2, fl, m, st));
    }
    if (eloc || O) {
      peps_status s = run_strips<M>(c, sm, m, et, eloc ? eloc + (size_t)c0 * 2 : nullptr,
                                    O ? (char*)O + (size_t)c0 * L.n_compact * ob : nullptr, fl,
                                    st);
      if (s != PEPS_OK) return s;
    }
  }
  return PEPS_OK;
}

static peps_status dispatch(peps_ctx* c, const double* theta, const uint8_t* samples, int n,
                            void* env_cache, bool env_given, double* logpsi, double* eloc, void* O,
                            int* flags, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) return PEPS_OK;
  if (eloc && !c->has_ham) return fail(PEPS_ERR_ARG, "no Hamiltonian set");
  // no host round trip: a non-finite theta is reported in the flags
  peps_status s = prepare_theta(c, theta, st, false);
  if (s != PEPS_OK) return s;
  switch (c->g.dtype) {
    case PEPS_F64:
      s = evaluate_impl<MODE_F64>(c, theta, samples, n, env_cache, env_given, logpsi, eloc, O,
                                  flags, st);
      break;
    case PEPS_F32:
      s = evaluate_impl<MODE_F32>(c, theta, samples, n, env_cache, env_given, logpsi, eloc, O,
                                  flags, st);
      break;
    case PEPS_BF16:
      s = evaluate_impl<MODE_BF16>(c, theta, samples, n, env_cache, env_given, logpsi, eloc, O,
                                   flags, st);
      break;
    case PEPS_C128:
      s = evaluate_impl<MODE_C128>(c, theta, samples, n, env_cache, env_given, logpsi, eloc, O,
                                   flags, st);
      break;
    default:
      s = evaluate_impl<MODE_C64>(c, theta, samples, n, env_cache, env_given, logpsi, eloc, O,
                                  flags, st);
      break;
  }
  if (s != PEPS_OK) return s;
  if (flags) HIPCHK(launch_flag_bad(flags, n, (const int*)c->bad.p, st));
  return PEPS_OK;
}

extern "C" {

peps_status peps_amplitude(peps_ctx* c, const double* theta, const uint8_t* samples, int n,
                           void* env_cache, double* logpsi, int32_t* flags, void* stream) {
  peps_status s = check_common(c, theta, samples, n);
  if (s != PEPS_OK) return s;
  if (n > 0 && !logpsi && !env_cache) return fail(PEPS_ERR_ARG, "no output requested");
  return dispatch(c, theta, samples, n, env_cache, false, logpsi, nullptr, nullptr, flags, stream);
}

peps_status peps_local_energy(peps_ctx* c, const double* theta, const uint8_t* samples, int n,
                              const void* env_cache, double* eloc, int32_t* flags, void* stream) {
  peps_status s = check_common(c, theta, samples, n);
  if (s != PEPS_OK) return s;
  if (n > 0 && !eloc) return fail(PEPS_ERR_ARG, "null eloc");
  if (!c->has_ham) return fail(PEPS_ERR_ARG, "no Hamiltonian set");
  return dispatch(c, theta, samples, n, (void*)env_cache, env_cache != nullptr, nullptr, eloc,
                  nullptr, flags, stream);
}

}  // extern "C"

template <int M>
static peps_status direct_rows(peps_ctx* c, int n, uint64_t seed, uint64_t offset,
                               uint8_t* samples, double* logp, int32_t* flags, hipStream_t st) {
  const Lattice& L = c->L;
  peps_ctx* d = c->dbl;
  const size_t BD = (size_t)L.bmax * L.D;
  const size_t per_t = env_tensor_elems_per_sample(L) * c->tsize;
  const size_t slab = direct_slab_elems(L, d->L);
  size_t per = per_t + L.n_slots * sizeof(double) + (size_t)L.Ly * BD * BD * c->tsize +
               slab * c->tsize;
  if (c->env_gm) per += env_slab_elems(L, c->g.dtype) * c->tsize;
  size_t ch = c->chunk_budget / per;
  if (ch < 1) ch = 1;
  if (ch > (size_t)n) ch = n;
  peps_status s;
  if ((s = c->env_int.ensure(ch * (per_t + L.n_slots * sizeof(double)))) != PEPS_OK) return s;
  if ((s = c->rscr.ensure(ch * L.Ly * BD * BD * c->tsize)) != PEPS_OK) return s;
  if ((s = c->dir_slab.ensure(ch * slab * c->tsize)) != PEPS_OK) return s;
  void* gws = nullptr;
  if (c->env_gm) {
    if ((s = c->gws_env.ensure(ch * env_slab_elems(L, c->g.dtype) * c->tsize)) != PEPS_OK)
      return s;
    gws = c->gws_env.p;
  }
  HIPCHK(hipMemsetAsync(logp, 0, (size_t)n * sizeof(double), st));
  if (flags) HIPCHK(hipMemsetAsync(flags, 0, (size_t)n * sizeof(int32_t), st));
  for (size_t c0 = 0; c0 < (size_t)n; c0 += ch) {
    const int m = (int)std::min(ch, (size_t)n - c0);
    uint8_t* sm = samples + c0 * L.N;
    char* et = (char*)c->env_int.p;
    double* el = (double*)(et + (size_t)m * per_t);
    int* fl = flags ? flags + c0 : nullptr;
    for (int i = 0; i < L.Lx; ++i) {
      {
        ProfScope ps(c, st, PEPS_PROF_SAMPLE);
        HIPCHK(launch_direct_row<M>(L, c->d_tab, c->theta_c.p, et, d->L, d->d_tab, c->dir_env2.p,
                                    sm, logp + c0, fl, m, i, seed, offset + c0, c->dir_slab.p,
                                    st));
      }
      if (i <= L.Lx - 2) {
        ProfScope ps(c, st, PEPS_PROF_ENV);
        HIPCHK(launch_env_top_step<M>(L, c->d_tab, c->theta_c.p, sm, et, el, c->rscr.p, fl, m, i,
                                      c->jac_sweeps, gws, st));
      }
    }
  }
  return PEPS_OK;
}

extern "C" {

peps_status peps_direct_sample(peps_ctx* c, const double* theta, int n, int chi_double,
                               int refresh, uint64_t seed, uint64_t offset, uint8_t* samples,
                               double* logp, double* logw, int32_t* flags, void* stream) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (!theta) return fail(PEPS_ERR_ARG, "null theta");
  if (n < 0) return fail(PEPS_ERR_ARG, "negative sample count");
  if (n > 0 && (!samples || !logp)) return fail(PEPS_ERR_ARG, "null samples or logp");
  if (chi_double < 1) return fail(PEPS_ERR_ARG, "chi_double = %d must be >= 1", chi_double);
  if (!refresh && (!c->dbl || !c->dbl_built || c->dbl_chi != chi_double))
    return fail(PEPS_ERR_ARG, "no double-layer environments with chi_double = %d to reuse",
                chi_double);
  if (n == 0 && !refresh) return PEPS_OK;
  hipStream_t st = (hipStream_t)stream;
  const Lattice& L = c->L;
  peps_status s;
  {
    // the row kernel stages E, two site tensors and D^l of a column in LDS:
    // reject shapes that do not fit before anything is queued
    const size_t D2 = (size_t)L.D * L.D, bm2 = std::max<size_t>((size_t)chi_double, D2);
    const size_t lds = ((size_t)L.bmax * L.D * L.bmax + 2 * D2 * D2 + bm2 * D2 * bm2) * c->tsize;
    if (lds > kLdsDyn)
      return fail(PEPS_ERR_UNSUPPORTED,
                  "direct sampler: %zu bytes of LDS per row workgroup (chi = %d, D = %d, "
                  "chi_double = %d) above %zu", lds, L.chi, L.D, chi_double, kLdsDyn);
  }
  if (!c->dbl || c->dbl_chi != chi_double) {
    if (c->dbl) peps_destroy(c->dbl);
    c->dbl = nullptr;
    c->dbl_chi = 0;
    c->dbl_built = false;
    peps_geom g2 = c->g;
    g2.D = c->g.D * c->g.D;
    g2.chi = chi_double;
    if ((s = peps_create(&g2, &c->dbl)) != PEPS_OK) return s;
    c->dbl->bottom_only = true;
    c->dbl_chi = chi_double;
  }
  peps_ctx* d = c->dbl;
  if (refresh) {
    c->dbl_built = false;
    const bool cx = is_complex(c->g.dtype);
    const size_t nth2 = (size_t)d->L.n_params * (cx ? 2 : 1);
    if ((s = c->dir_th2.ensure(nth2 * sizeof(double))) != PEPS_OK) return s;
    if ((s = c->dir_zero.ensure((size_t)L.N)) != PEPS_OK) return s;
    if ((s = c->dir_env2.ensure(peps_env_cache_bytes(d, 1))) != PEPS_OK) return s;
    if ((s = c->dir_lp2.ensure(2 * sizeof(double) + sizeof(int32_t))) != PEPS_OK) return s;
    HIPCHK(hipMemsetAsync(c->dir_zero.p, 0, (size_t)L.N, st));
    HIPCHK(launch_double_theta(L, c->d_tab, d->L, d->d_tab, theta, (double*)c->dir_th2.p, cx,
                               st));
    // D^l of the double layer: the bottom environments of one all-zero
    // configuration (no top sweep, no amplitude)
    s = peps_amplitude(d, (const double*)c->dir_th2.p, (const uint8_t*)c->dir_zero.p, 1,
                       c->dir_env2.p, nullptr, (int32_t*)((double*)c->dir_lp2.p + 2), stream);
    if (s != PEPS_OK) return s;
    c->dbl_built = true;
  }
  if (n == 0) return PEPS_OK;
  if ((s = prepare_theta(c, theta, st)) != PEPS_OK) return s;
  switch (c->g.dtype) {
    case PEPS_F64: s = direct_rows<MODE_F64>(c, n, seed, offset, samples, logp, flags, st); break;
    case PEPS_F32: s = direct_rows<MODE_F32>(c, n, seed, offset, samples, logp, flags, st); break;
    case PEPS_BF16: s = direct_rows<MODE_BF16>(c, n, seed, offset, samples, logp, flags, st); break;
    case PEPS_C128: s = direct_rows<MODE_C128>(c, n, seed, offset, samples, logp, flags, st); break;
    default: s = direct_rows<MODE_C64>(c, n, seed, offset, samples, logp, flags, st);
  }
  if (s != PEPS_OK) return s;
  if (logw) {
    if ((s = c->dir_lp.ensure((size_t)n * 2 * sizeof(double))) != PEPS_OK) return s;
    if ((s = c->dir_fl.ensure((size_t)n * sizeof(int32_t))) != PEPS_OK) return s;
    s = dispatch(c, theta, samples, n, nullptr, false, (double*)c->dir_lp.p, nullptr, nullptr,
                 (int*)c->dir_fl.p, stream);
    if (s != PEPS_OK) return s;
    HIPCHK(launch_direct_logw(n, (const double*)c->dir_lp.p, logp, (const int*)c->dir_fl.p, logw,
                              flags, st));
  }
  return PEPS_OK;
}

peps_status peps_set_truncation(peps_ctx* c, double max_weight) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (!std::isfinite(max_weight) || max_weight < 0.0 || max_weight >= 1.0)
    return fail(PEPS_ERR_ARG, "maximal truncated weight %g outside [0, 1)", max_weight);
  c->L.trunc_w = max_weight;
  return PEPS_OK;
}

peps_status peps_set_compression(peps_ctx* c, int method) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (method != PEPS_COMPRESS_CANONICAL && method != PEPS_COMPRESS_DENSMAT)
    return fail(PEPS_ERR_ARG, "unknown compression method %d", method);
  if (method == PEPS_COMPRESS_DENSMAT && !c->dm_ok)
    return fail(PEPS_ERR_UNSUPPORTED,
                "density-matrix truncation: chi = %d, chi*D = %d and dtype %d exceed the "
                "kernel's limits (chi*D padded to <= 256, packed rho in LDS)",
                c->g.chi, c->L.bmax * c->g.D, (int)c->g.dtype);
  c->compress = method;
  return PEPS_OK;
}

peps_status peps_set_minsr_solver(peps_ctx* c, int solver) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (solver != PEPS_MINSR_CHOLESKY && solver != PEPS_MINSR_EIGH && solver != PEPS_MINSR_AUTO)
    return fail(PEPS_ERR_ARG, "unknown minSR solver %d", solver);
  c->minsr_solver = solver;
  return PEPS_OK;
}

peps_status peps_local_energy_strict(peps_ctx* c, const double* theta, const uint8_t* samples,
                                     int n, double* eloc, int32_t* flags, void* stream) {
  peps_status s = check_common(c, theta, samples, n);
  if (s != PEPS_OK) return s;
  if (n > 0 && !eloc) return fail(PEPS_ERR_ARG, "null eloc");
  if (!c->has_ham) return fail(PEPS_ERR_ARG, "no Hamiltonian set");
  if (n == 0) return PEPS_OK;
  if ((long long)n * (1 + c->n_moves) > (long long)INT_MAX)
    return fail(PEPS_ERR_UNSUPPORTED, "%d samples x %d moves exceed the int32 batch index", n,
                c->n_moves);
  hipStream_t st = (hipStream_t)stream;
  const Lattice& L = c->L;
  if ((s = c->str_idx.ensure((size_t)(2 * n + 1) * sizeof(int))) != PEPS_OK) return s;
  int* cnt = (int*)c->str_idx.p;
  int* off = cnt + n;
  HIPCHK(launch_strict_count(L, c->H, c->n_moves, samples, n, cnt, off, st));
  int nb = 0;
  HIPCHK(hipMemcpyAsync(&nb, off + n, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (nb < n || (long long)nb > (long long)n * (1 + c->n_moves))
    return fail(PEPS_ERR_ARG, "inconsistent neighbour count %d", nb);
  if ((s = c->str_batch.ensure((size_t)nb * L.N)) != PEPS_OK) return s;
  if ((s = c->str_coef.ensure(((size_t)(nb - n) + 1) * 2 * sizeof(double))) != PEPS_OK) return s;
  if ((s = c->str_lp.ensure((size_t)nb * 2 * sizeof(double))) != PEPS_OK) return s;
  if ((s = c->str_fl.ensure((size_t)nb * sizeof(int))) != PEPS_OK) return s;
  uint8_t* batch = (uint8_t*)c->str_batch.p;
  double* coef = (double*)c->str_coef.p;
  double* lp = (double*)c->str_lp.p;
  int* fl = (int*)c->str_fl.p;
  HIPCHK(launch_strict_expand(L, c->H, c->n_moves, samples, n, off, batch, coef, st));
  s = dispatch(c, theta, batch, nb, nullptr, false, lp, nullptr, nullptr, fl, stream);
  if (s != PEPS_OK) return s;
  {
    ProfScope ps(c, st, PEPS_PROF_ESUM);
    HIPCHK(launch_energy_diag_sum(L, c->H, samples, nullptr, 1, eloc, n, st));
    HIPCHK(launch_strict_combine(n, off, coef, lp, fl, eloc, flags, st));
  }
  return PEPS_OK;
}

peps_status peps_logderiv(peps_ctx* c, const double* theta, const uint8_t* samples, int n,
                          const void* env_cache, void* O, void* stream) {
  peps_status s = check_common(c, theta, samples, n);
  if (s != PEPS_OK) return s;
  if (n > 0 && !O) return fail(PEPS_ERR_ARG, "null O");
  return dispatch(c, theta, samples, n, (void*)env_cache, env_cache != nullptr, nullptr, nullptr,
                  O, nullptr, stream);
}

peps_status peps_evaluate(peps_ctx* c, const double* theta, const uint8_t* samples, int n,
                          double* logpsi, double* eloc, void* O, int32_t* flags, void* stream) {
  peps_status s = check_common(c, theta, samples, n);
  if (s != PEPS_OK) return s;
  if (eloc && !c->has_ham) return fail(PEPS_ERR_ARG, "no Hamiltonian set");
  return dispatch(c, theta, samples, n, nullptr, false, logpsi, eloc, O, flags, stream);
}

peps_status minsr_step(peps_ctx* c, const void* O, const uint8_t* samples, int n,
                       const double* eloc, double eps, double rcond, double* dtheta, double* diag,
                       void* stream) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (n < 2) return fail(PEPS_ERR_ARG, "minSR needs at least 2 samples (got %d)", n);
  if (!O || !samples || !eloc || !dtheta || !diag) return fail(PEPS_ERR_ARG, "null pointer");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(PEPS_ERR_ARG, "eps must be finite and >= 0");
  if (!(rcond >= 0.0 && rcond < 1.0)) return fail(PEPS_ERR_ARG, "rcond must be in [0, 1)");
  if ((size_t)n * n > ((size_t)1 << 33)) return fail(PEPS_ERR_UNSUPPORTED, "n = %d too large", n);
  hipStream_t st = (hipStream_t)stream;
  const Lattice& L = c->L;
  const int mode = c->g.dtype == PEPS_BF16 ? MODE_F32 : c->g.dtype;
  size_t b_mean, b_T, b_vec;
  minsr_ws_bytes(L, mode, n, &b_mean, &b_T, &b_vec);
  peps_status s = c->mean.ensure(b_mean);
  if (s != PEPS_OK) return s;
  s = c->Tm.ensure(b_T);
  if (s != PEPS_OK) return s;
  s = c->vec.ensure(b_vec);
  if (s != PEPS_OK) return s;
  const int solver = c->minsr_solver;
  if (solver == PEPS_MINSR_EIGH && n > MINSR_EIG_MAX)
    return fail(PEPS_ERR_UNSUPPORTED, "the eigendecomposition solve takes n <= %d (got %d)",
                MINSR_EIG_MAX, n);
  void* eig = nullptr;
  if (solver != PEPS_MINSR_CHOLESKY && n <= MINSR_EIG_MAX) {
    s = c->eig_ws.ensure(eigh_ws_bytes(n, is_complex(c->g.dtype)));
    if (s != PEPS_OK) return s;
    eig = c->eig_ws.p;
  }
  ProfScope ps(c, st, PEPS_PROF_MINSR);
  HIPCHK(launch_minsr(L, c->d_tab, mode, O, samples, n, eloc, eps, rcond, dtheta, diag,
                      c->mean.p, c->Tm.p, c->vec.p, solver, eig, st));
  return PEPS_OK;
}

peps_status minsr_step_noalloc(peps_ctx* c, const void* O, const uint8_t* samples, int n,
                               const double* eloc, double eps, double rcond, double* dtheta,
                               double* diag, void* stream) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (n < 2) return fail(PEPS_ERR_ARG, "minSR needs at least 2 samples (got %d)", n);
  if (!O || !samples || !eloc || !dtheta || !diag) return fail(PEPS_ERR_ARG, "null pointer");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(PEPS_ERR_ARG, "eps must be finite and >= 0");
  if (!(rcond >= 0.0 && rcond < 1.0)) return fail(PEPS_ERR_ARG, "rcond must be in [0, 1)");
  if (c->minsr_solver != PEPS_MINSR_CHOLESKY)
    return fail(PEPS_ERR_UNSUPPORTED,
                "minsr_step_noalloc runs the certified Cholesky solve only (solver %d set)",
                c->minsr_solver);
  const Lattice& L = c->L;
  const int mode = c->g.dtype == PEPS_BF16 ? MODE_F32 : c->g.dtype;
  size_t b_mean, b_T, b_vec;
  minsr_ws_bytes(L, mode, n, &b_mean, &b_T, &b_vec);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t need = up(b_mean) + up(b_T) + up(b_vec);
  if (need > PEPS_NOALLOC_SCRATCH_BYTES)
    return fail(PEPS_ERR_UNSUPPORTED,
                "minsr_step_noalloc: n = %d with %d parameters needs %zu bytes of workspace, "
                "above its fixed %zu-byte scratch (use minsr_step)",
                n, L.n_params, need, PEPS_NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  peps_status s = scratch_ptr(&base);
  if (s != PEPS_OK) return s;
  char* b = (char*)base;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_minsr(L, c->d_tab, mode, O, samples, n, eloc, eps, rcond, dtheta, diag, b,
                      b + up(b_mean), b + up(b_mean) + up(b_T), PEPS_MINSR_CHOLESKY, nullptr, st));
  return PEPS_OK;
}

peps_status peps_logderiv_vjp(peps_ctx* c, const void* O, const uint8_t* samples, int n,
                              const double* g, double* grad_theta, void* stream) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (n < 0) return fail(PEPS_ERR_ARG, "negative sample count");
  if (!grad_theta || (n > 0 && (!O || !samples || !g))) return fail(PEPS_ERR_ARG, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  const bool cx = is_complex(c->g.dtype);
  if (n == 0) {
    HIPCHK(hipMemsetAsync(grad_theta, 0, (size_t)c->L.n_params * (cx ? 2 : 1) * sizeof(double),
                          st));
    return PEPS_OK;
  }
  const int mode = c->g.dtype == PEPS_BF16 ? MODE_F32 : c->g.dtype;
  HIPCHK(launch_vjp(c->L, c->d_tab, mode, O, samples, n, g, grad_theta, st));
  return PEPS_OK;
}

peps_status peps_rotate_basis(peps_ctx* c, const double* theta, int basis, double* theta_out,
                              void* stream) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (!theta || !theta_out) return fail(PEPS_ERR_ARG, "null pointer");
  if (basis < PEPS_BASIS_Z || basis > PEPS_BASIS_Y)
    return fail(PEPS_ERR_ARG, "basis %d (0 = Z, 1 = X, 2 = Y)", basis);
  const bool cx = is_complex(c->g.dtype);
  if (basis == PEPS_BASIS_Y && !cx)
    return fail(PEPS_ERR_UNSUPPORTED, "the Y rotation gives complex tensors: use a complex context");
  hipStream_t st = (hipStream_t)stream;
  if (basis == PEPS_BASIS_Z) {
    if (theta_out != theta)
      HIPCHK(hipMemcpyAsync(theta_out, theta, (size_t)c->L.n_params * (cx ? 2 : 1) * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    return PEPS_OK;
  }
  HIPCHK(launch_rotate_basis(c->L, c->d_tab, basis == PEPS_BASIS_X ? ROT_X : ROT_Y, cx, theta,
                             theta_out, st));
  return PEPS_OK;
}

peps_status peps_energy_diag(peps_ctx* c, const uint8_t* samples, int n, double* eloc,
                             void* stream) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (n < 0) return fail(PEPS_ERR_ARG, "negative sample count");
  if (n > 0 && (!samples || !eloc)) return fail(PEPS_ERR_ARG, "null pointer");
  if (!c->has_ham) return fail(PEPS_ERR_ARG, "no Hamiltonian set");
  if (n == 0) return PEPS_OK;
  HIPCHK(launch_energy_diag_sum(c->L, c->H, samples, nullptr, 0, eloc, n, (hipStream_t)stream));
  return PEPS_OK;
}

peps_status peps_profile(peps_ctx* c, int enable) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  c->prof = enable != 0;
  return PEPS_OK;
}

peps_status peps_profile_read(peps_ctx* c, double* ms, long* counts, int reset) {
  if (!c || !ms || !counts) return fail(PEPS_ERR_ARG, "null pointer");
  for (auto& e : c->pending) {
    HIPCHK(hipEventSynchronize(e.b));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
    c->prof_ms[e.kind] += t;
    c->prof_n[e.kind] += 1;
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  c->pending.clear();
  for (int k = 0; k < PEPS_PROF_KINDS; ++k) {
    ms[k] = c->prof_ms[k];
    counts[k] = c->prof_n[k];
    if (reset) {
      c->prof_ms[k] = 0.0;
      c->prof_n[k] = 0;
    }
  }
  return PEPS_OK;
}

static peps_status sample_imh(peps_ctx* c, const double* theta, int n_chains, int per_chain,
                              int burn_in, int thin, uint64_t seed, uint64_t offset,
                              const peps_proposal* pr, uint8_t* samples, double* logpsi,
                              int32_t* accepted, hipStream_t st) {
  const Lattice& L = c->L;
  if (!pr || !pr->made || !pr->params) return fail(PEPS_ERR_ARG, "IMH needs a proposal");
  if (pr->made->N != L.N)
    return fail(PEPS_ERR_ARG, "proposal over %d sites, lattice has %d", pr->made->N, L.N);
  const size_t nc = (size_t)n_chains;
  peps_status s;
  if ((s = c->imh_st.ensure(nc * L.N)) != PEPS_OK) return s;
  if ((s = c->imh_pr.ensure(nc * L.N)) != PEPS_OK) return s;
  if ((s = c->imh_stlp.ensure(nc * 2 * sizeof(double))) != PEPS_OK) return s;
  if ((s = c->imh_prlp.ensure(nc * 2 * sizeof(double))) != PEPS_OK) return s;
  if ((s = c->imh_stlq.ensure(nc * sizeof(double))) != PEPS_OK) return s;
  if ((s = c->imh_prlq.ensure(nc * sizeof(double))) != PEPS_OK) return s;
  uint8_t* state = (uint8_t*)c->imh_st.p;
  uint8_t* prop = (uint8_t*)c->imh_pr.p;
  double* st_lp = (double*)c->imh_stlp.p;
  double* st_lq = (double*)c->imh_stlq.p;
  double* pr_lp = (double*)c->imh_prlp.p;
  double* pr_lq = (double*)c->imh_prlq.p;
  if (pr->init) {
    HIPCHK(hipMemcpyAsync(state, pr->init, nc * L.N, hipMemcpyDeviceToDevice, st));
    if ((s = made_logq(pr->made, pr->params, state, n_chains, st_lq, st)) != PEPS_OK) return s;
  } else {
    if ((s = made_sample(pr->made, pr->params, n_chains, seed, offset, state, st_lq, st)) !=
        PEPS_OK)
      return s;
  }
  if ((s = peps_amplitude(c, theta, state, n_chains, nullptr, st_lp, nullptr, st)) != PEPS_OK)
    return s;
  const long long total = (long long)burn_in + (long long)per_chain * thin;
  int j = 0;
  for (long long t = 1; t <= total; ++t) {
    if ((s = made_sample(pr->made, pr->params, n_chains, seed, offset + (uint64_t)t, prop, pr_lq,
                         st)) != PEPS_OK)
      return s;
    if ((s = peps_amplitude(c, theta, prop, n_chains, nullptr, pr_lp, nullptr, st)) != PEPS_OK)
      return s;
    if ((s = imh_step(n_chains, L.N, state, st_lp, st_lq, prop, pr_lp, pr_lq, seed,
                      offset + (uint64_t)t, accepted, st)) != PEPS_OK)
      return s;
    if (t > burn_in && (t - burn_in) % thin == 0 && j < per_chain) {
      HIPCHK(launch_imh_record(n_chains, L.N, state, st_lp, per_chain, j, samples, logpsi, st));
      ++j;
    }
  }
  return PEPS_OK;
}

peps_status peps_sample(peps_ctx* c, const double* theta, int kind, int n_chains, int per_chain,
                        int burn_in, int thin, uint64_t seed, uint64_t offset,
                        const peps_proposal* proposal, uint8_t* samples, double* logpsi,
                        int32_t* accepted, void* stream) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (!theta || !samples) return fail(PEPS_ERR_ARG, "null theta or samples");
  if (kind != PEPS_SAMPLE_EXCHANGE && kind != PEPS_SAMPLE_FLIP && kind != PEPS_SAMPLE_IMH)
    return fail(PEPS_ERR_ARG, "unknown sampler kind %d", kind);
  if (n_chains < 1 || per_chain < 1 || burn_in < 0 || thin < 1)
    return fail(PEPS_ERR_ARG, "need n_chains >= 1, per_chain >= 1, burn_in >= 0, thin >= 1");
  if ((long long)burn_in + (long long)per_chain * thin > (1LL << 30))
    return fail(PEPS_ERR_ARG, "too many sweeps");
  hipStream_t st = (hipStream_t)stream;
  if (kind == PEPS_SAMPLE_IMH) {
    if (accepted) HIPCHK(hipMemsetAsync(accepted, 0, (size_t)n_chains * sizeof(int32_t), st));
    return sample_imh(c, theta, n_chains, per_chain, burn_in, thin, seed, offset, proposal,
                      samples, logpsi, accepted, st);
  }
  const Lattice& L = c->L;
  if (L.N > 1024) return fail(PEPS_ERR_UNSUPPORTED, "sampler holds at most 1024 sites");
  peps_status s = prepare_theta(c, theta, st);
  if (s != PEPS_OK) return s;
  const size_t BD = (size_t)L.bmax * L.D;
  const size_t box = L.site_box;
  const size_t box2 = (size_t)L.bmax * L.bmax * L.D * L.D;
  const size_t nc = (size_t)n_chains;
  if ((s = c->env_int.ensure(nc * env_tensor_elems_per_sample(L) * c->tsize)) != PEPS_OK) return s;
  if ((s = c->eloc_tmp.ensure(nc * L.n_slots * sizeof(double))) != PEPS_OK) return s;
  if ((s = c->rscr.ensure(nc * L.Ly * BD * BD * c->tsize)) != PEPS_OK) return s;
  if ((s = c->rt1.ensure(nc * (L.Ly + 1) * box * c->tsize)) != PEPS_OK) return s;
  if ((s = c->rt2.ensure(nc * (L.Ly + 1) * box2 * c->tsize)) != PEPS_OK) return s;
  void* gws = nullptr;
  if (c->smp_gm) {
    if ((s = c->gws_smp.ensure(nc * sample_slab_elems(L, c->g.dtype) * c->tsize)) != PEPS_OK) return s;
    gws = c->gws_smp.p;
  }
  if ((s = c->smp_state.ensure(sample_state_bytes(L, n_chains))) != PEPS_OK) return s;
  // the density-matrix truncation for the chains' environments when chosen
  void* dm_slabs = nullptr;
  if (c->compress == PEPS_COMPRESS_DENSMAT) {
    const int mode = c->g.dtype;
    if ((s = c->gws_dm.ensure(nc * env_dm_slab_elems(L, mode) * c->tsize)) != PEPS_OK) return s;
    dm_slabs = c->gws_dm.p;
  }
  {
    ProfScope ps(c, st, PEPS_PROF_SAMPLE);
#define MET(MODE)                                                                               \
  HIPCHK(launch_metropolis<MODE>(L, c->d_tab, c->theta_c.p, kind, n_chains, per_chain, burn_in, \
                                 thin, seed, offset, samples, accepted, c->env_int.p,           \
                                 (double*)c->eloc_tmp.p, c->rscr.p, c->rt1.p, c->rt2.p,         \
                                 c->jac_sweeps, gws, c->smp_state.p, dm_slabs, st))
    switch (c->g.dtype) {
      case PEPS_F64: MET(MODE_F64); break;
      case PEPS_F32: MET(MODE_F32); break;
      case PEPS_BF16: MET(MODE_BF16); break;
      case PEPS_C128: MET(MODE_C128); break;
      default: MET(MODE_C64);
    }
#undef MET
  }
  if (logpsi)
    return peps_amplitude(c, theta, samples, n_chains * per_chain, nullptr, logpsi, nullptr, st);
  return PEPS_OK;
}

peps_status peps_vmc_step(peps_ctx* c, double* theta, int kind, int n_chains, int per_chain,
                          int burn_in, int thin, uint64_t seed, uint64_t offset, double tau,
                          double eps, double rcond, uint8_t* samples, double* eloc,
                          int32_t* flags, double* diag, void* stream) {
  if (!c) return fail(PEPS_ERR_ARG, "null context");
  if (!theta || !samples || !eloc || !diag) return fail(PEPS_ERR_ARG, "null pointer");
  if (!c->has_ham) return fail(PEPS_ERR_ARG, "no Hamiltonian set");
  if (!std::isfinite(tau)) return fail(PEPS_ERR_ARG, "tau must be finite");
  if (n_chains < 1 || per_chain < 1) return fail(PEPS_ERR_ARG, "need n_chains, per_chain >= 1");
  const long long nl = (long long)n_chains * per_chain;
  if (nl < 2 || nl > (1 << 24)) return fail(PEPS_ERR_ARG, "batch of %lld samples", nl);
  const int n = (int)nl;
  hipStream_t st = (hipStream_t)stream;
  const Lattice& L = c->L;
  const size_t nth = (size_t)L.n_params * (is_complex(c->g.dtype) ? 2 : 1);
  peps_status s = c->vmc_O.ensure((size_t)n * L.n_compact * c->tsize);
  if (s != PEPS_OK) return s;
  if ((s = c->vmc_dth.ensure(nth * sizeof(double))) != PEPS_OK) return s;
  if ((s = c->vmc_lp.ensure((size_t)n * 2 * sizeof(double))) != PEPS_OK) return s;
  s = peps_sample(c, theta, kind, n_chains, per_chain, burn_in, thin, seed, offset, nullptr,
                  samples, nullptr, nullptr, stream);
  if (s != PEPS_OK) return s;
  s = peps_evaluate(c, theta, samples, n, (double*)c->vmc_lp.p, eloc, c->vmc_O.p, flags, stream);
  if (s != PEPS_OK) return s;
  s = minsr_step(c, c->vmc_O.p, samples, n, eloc, eps, rcond, (double*)c->vmc_dth.p, diag,
                 stream);
  if (s != PEPS_OK) return s;
  HIPCHK(launch_theta_update(theta, (const double*)c->vmc_dth.p, diag, tau, nth, st));
  double cert = 0.0;
  HIPCHK(hipMemcpyAsync(&cert, diag + 3, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (cert != 0.0)
    return fail(PEPS_ERR_NONFINITE, "minSR certificate failed; theta left unchanged");
  return PEPS_OK;
}

// ---------------------------------------------------------------------------
// learned proposal
// ---------------------------------------------------------------------------

peps_status made_create(int N, int H, int n_up, int bf16, made_ctx** out) {
  if (!out) return fail(PEPS_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (N < 2 || N > 4096) return fail(PEPS_ERR_ARG, "N = %d outside 2..4096", N);
  if (H < 1 || H > 256) return fail(PEPS_ERR_UNSUPPORTED, "hidden width %d outside 1..256", H);
  if (n_up < -1 || n_up > N) return fail(PEPS_ERR_ARG, "n_up = %d outside -1..N", n_up);
  made_ctx* m = new made_ctx();
  m->N = N;
  m->H = H;
  m->n_up = n_up;
  m->bf16 = bf16 ? 1 : 0;
  *out = m;
  return PEPS_OK;
}

void made_destroy(made_ctx* m) {
  if (!m) return;
  m->a.release();
  m->lg.release();
  m->dlg.release();
  m->da.release();
  m->logq.release();
  m->xb.release();
  m->gr.release();
  m->ptab.release();
  delete m;
}

size_t made_num_params(const made_ctx* m) {
  return m ? (size_t)2 * m->N * m->H + m->N + m->H : 0;
}

static peps_status made_ws(made_ctx* m, int B, bool grad) {
  peps_status s;
  if ((s = m->a.ensure((size_t)B * m->H * sizeof(float))) != PEPS_OK) return s;
  if ((s = m->lg.ensure((size_t)B * m->N * sizeof(float))) != PEPS_OK) return s;
  if ((s = m->logq.ensure((size_t)B * sizeof(double))) != PEPS_OK) return s;
  if (grad) {
    if ((s = m->dlg.ensure((size_t)B * m->N * sizeof(float))) != PEPS_OK) return s;
    if ((s = m->da.ensure((size_t)B * m->H * sizeof(float))) != PEPS_OK) return s;
  }
  return PEPS_OK;
}

peps_status made_loss_grad(made_ctx* m, const float* params, const uint8_t* x, int B,
                           float* grads, double* loss, void* stream) {
  if (!m || !params || !x || !grads || !loss) return fail(PEPS_ERR_ARG, "null pointer");
  if (B < 1) return fail(PEPS_ERR_ARG, "batch %d < 1", B);
  peps_status s = made_ws(m, B, true);
  if (s != PEPS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_made_forward(m->N, m->H, m->n_up, m->bf16, params, x, B, (float*)m->a.p,
                             (float*)m->lg.p, st));
  HIPCHK(launch_made_head(m->N, m->H, m->n_up, x, B, (const float*)m->lg.p, (float*)m->dlg.p,
                          (double*)m->logq.p, st));
  HIPCHK(launch_made_backward(m->N, m->H, m->n_up, m->bf16, params, x, B, (const float*)m->a.p,
                              (const float*)m->dlg.p, (float*)m->da.p, grads,
                              (const double*)m->logq.p, loss, st));
  return PEPS_OK;
}

peps_status made_adam_step(made_ctx* m, float* params, const float* grads, float* mom,
                           float* var, int t, double lr, double beta1, double beta2, double eps,
                           void* stream) {
  if (!m || !params || !grads || !mom || !var) return fail(PEPS_ERR_ARG, "null pointer");
  if (t < 1) return fail(PEPS_ERR_ARG, "Adam step counter starts at 1");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(PEPS_ERR_ARG, "bad Adam hyper-parameters");
  HIPCHK(launch_made_adam((int)made_num_params(m), params, grads, mom, var, t, (float)lr,
                          (float)beta1, (float)beta2, (float)eps, (hipStream_t)stream));
  return PEPS_OK;
}

static unsigned long long splitmix64(unsigned long long& x) {
  unsigned long long z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

peps_status made_train(made_ctx* m, float* params, const uint8_t* data, int M, int steps,
                       int batch, int t0, double lr, double beta1, double beta2, double eps,
                       uint64_t seed, float* mom, float* var, double* losses, void* stream) {
  if (!m || !params || !data || !mom || !var || !losses) return fail(PEPS_ERR_ARG, "null pointer");
  if (M < 1 || steps < 0 || batch < 1 || t0 < 0)
    return fail(PEPS_ERR_ARG, "need M >= 1, steps >= 0, batch >= 1, t0 >= 0");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(PEPS_ERR_ARG, "bad Adam hyper-parameters");
  if (steps == 0) return PEPS_OK;
  hipStream_t st = (hipStream_t)stream;
  peps_status s = made_ws(m, batch, true);
  if (s != PEPS_OK) return s;
  if ((s = m->xb.ensure((size_t)batch * m->N)) != PEPS_OK) return s;
  // one permutation r -> (a r + c) mod M per epoch, a coprime with M
  const long long total = (long long)steps * batch;
  const long long epochs = total / M + 2;
  m->hptab.assign(2 * (size_t)epochs, 0ull);
  unsigned long long sm = seed;
  for (long long e = 0; e < epochs; ++e) {
    unsigned long long a = M > 1 ? splitmix64(sm) % (unsigned long long)M : 1ull;
    if (a == 0) a = 1;
    auto gcd = [](unsigned long long x, unsigned long long y) {
      while (y) {
        const unsigned long long t = x % y;
        x = y;
        y = t;
      }
      return x;
    };
    while (gcd(a, (unsigned long long)M) != 1ull) a = a + 1 < (unsigned long long)M ? a + 1 : 1;
    m->hptab[2 * e] = a;
    m->hptab[2 * e + 1] = splitmix64(sm) % (unsigned long long)M;
  }
  if ((s = m->ptab.ensure(m->hptab.size() * sizeof(unsigned long long))) != PEPS_OK) return s;
  HIPCHK(hipMemcpyAsync(m->ptab.p, m->hptab.data(), m->hptab.size() * sizeof(unsigned long long),
                        hipMemcpyHostToDevice, st));
  const int np = (int)made_num_params(m);
  if ((s = m->gr.ensure((size_t)np * sizeof(float))) != PEPS_OK) return s;
  float* grads = (float*)m->gr.p;
  uint8_t* xb = (uint8_t*)m->xb.p;
  for (int i = 0; i < steps; ++i) {
    HIPCHK(launch_made_gather(data, M, m->N, batch, (long long)i * batch,
                              (const unsigned long long*)m->ptab.p, xb, st));
    HIPCHK(launch_made_forward(m->N, m->H, m->n_up, m->bf16, params, xb, batch, (float*)m->a.p,
                               (float*)m->lg.p, st));
    HIPCHK(launch_made_head(m->N, m->H, m->n_up, xb, batch, (const float*)m->lg.p,
                            (float*)m->dlg.p, (double*)m->logq.p, st));
    HIPCHK(launch_made_backward(m->N, m->H, m->n_up, m->bf16, params, xb, batch,
                                (const float*)m->a.p, (const float*)m->dlg.p, (float*)m->da.p,
                                grads, (const double*)m->logq.p, losses + i, st));
    HIPCHK(launch_made_adam(np, params, grads, mom, var, t0 + i + 1, (float)lr, (float)beta1,
                            (float)beta2, (float)eps, st));
  }
  return PEPS_OK;
}

peps_status peps_tau_int(const double* series, int n_chains, int T, int ranked, double c,
                         double* work, double* out, void* stream) {
  if (!series || !work || !out) return fail(PEPS_ERR_ARG, "null pointer");
  if (n_chains < 1 || T < 1) return fail(PEPS_ERR_ARG, "need n_chains >= 1 and T >= 1");
  if (!(c > 0.0)) return fail(PEPS_ERR_ARG, "window constant must be positive");
  if ((long long)n_chains * T > (1LL << 24))
    return fail(PEPS_ERR_UNSUPPORTED, "at most 2^24 observations");
  HIPCHK(launch_tau_int(series, n_chains, T, ranked, c, work, out, (hipStream_t)stream));
  return PEPS_OK;
}

peps_status made_sample(made_ctx* m, const float* params, int n, uint64_t seed, uint64_t offset,
                        uint8_t* out, double* logq, void* stream) {
  if (!m || !params || !out || !logq) return fail(PEPS_ERR_ARG, "null pointer");
  if (n < 0) return fail(PEPS_ERR_ARG, "negative count");
  if (n == 0) return PEPS_OK;
  HIPCHK(launch_made_sample(m->N, m->H, m->n_up, m->bf16, params, n, seed, offset, out, logq,
                            (hipStream_t)stream));
  return PEPS_OK;
}

peps_status made_logq(made_ctx* m, const float* params, const uint8_t* x, int n, double* logq,
                      void* stream) {
  if (!m || !params || !x || !logq) return fail(PEPS_ERR_ARG, "null pointer");
  if (n < 0) return fail(PEPS_ERR_ARG, "negative count");
  if (n == 0) return PEPS_OK;
  peps_status s = made_ws(m, n, false);
  if (s != PEPS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_made_forward(m->N, m->H, m->n_up, m->bf16, params, x, n, (float*)m->a.p,
                             (float*)m->lg.p, st));
  HIPCHK(launch_made_head(m->N, m->H, m->n_up, x, n, (const float*)m->lg.p, nullptr, logq, st));
  return PEPS_OK;
}

peps_status imh_step(int n_chains, int N, uint8_t* state, double* state_logpsi,
                     double* state_logq, const uint8_t* prop, const double* prop_logpsi,
                     const double* prop_logq, uint64_t seed, uint64_t step, int32_t* accepted,
                     void* stream) {
  if (n_chains < 1 || N < 1) return fail(PEPS_ERR_ARG, "bad sizes");
  if (!state || !state_logpsi || !state_logq || !prop || !prop_logpsi || !prop_logq)
    return fail(PEPS_ERR_ARG, "null pointer");
  HIPCHK(launch_imh(n_chains, N, state, state_logpsi, state_logq, prop, prop_logpsi, prop_logq,
                    seed, step, accepted, (hipStream_t)stream));
  return PEPS_OK;
}

}  // extern "C"
