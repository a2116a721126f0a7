"""ctypes binding of libpepsmin.so (declared in include/pepsmin.h).

Argument marshalling only: torch tensors provide device memory and the
stream, every step of the computation runs in the library's HIP kernels.
There is no fallback: if the library is missing or a call fails, an
exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpepsmin.so")

PEPS_OK = 0
STATUS_NAMES = {0: "PEPS_OK", 1: "PEPS_ERR_ARG", 2: "PEPS_ERR_UNSUPPORTED", 3: "PEPS_ERR_HIP",
                4: "PEPS_ERR_OOM", 5: "PEPS_ERR_NONFINITE"}
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "c128": 3, "c64": 4}
COMPLEX = ("c128", "c64")
FLAG_ZERO, FLAG_NONFINITE, FLAG_NOCONV, FLAG_DEGENERATE = 1, 2, 4, 8
SAMPLE_EXCHANGE, SAMPLE_FLIP, SAMPLE_IMH = 0, 1, 2
COMPRESS = {"canonical": 0, "densmat": 1}
MINSR_SOLVER = {"cholesky": 0, "eigh": 1, "auto": 2}
BASIS = {"z": 0, "x": 1, "y": 2}

# every symbol the header declares
EXPORTS = ["peps_create", "peps_destroy", "peps_last_error", "peps_num_params",
           "peps_env_cache_bytes", "peps_set_hamiltonian", "peps_amplitude",
           "peps_local_energy", "peps_logderiv", "peps_evaluate", "minsr_step", "peps_sample",
           "peps_profile", "peps_profile_read", "made_create", "made_destroy",
           "made_num_params", "made_loss_grad", "made_adam_step", "made_sample", "made_logq",
           "imh_step", "peps_logderiv_vjp", "peps_vmc_step", "peps_local_energy_strict",
           "peps_set_truncation", "peps_direct_sample", "peps_set_compression",
           "peps_set_minsr_solver",
           "minsr_step_noalloc", "made_train", "peps_tau_int", "peps_rotate_basis",
           "peps_energy_diag"]
PROF_KINDS = ["env", "overlap", "strip1", "strip2", "esum", "minsr", "sample", "unused"]


class PepsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Proposal(ctypes.Structure):
    _fields_ = [("made", ctypes.c_void_p), ("params", ctypes.c_void_p), ("init", ctypes.c_void_p)]


class Geom(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("d", ctypes.c_int),
                ("D", ctypes.c_int), ("chi", ctypes.c_int), ("dtype", ctypes.c_int)]


_lib = None


def load():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run paper_2503_12557_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, Z, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_uint64
    lib.peps_create.argtypes = [ctypes.POINTER(Geom), ctypes.POINTER(P)]
    lib.peps_create.restype = I
    lib.peps_destroy.argtypes = [P]
    lib.peps_destroy.restype = None
    lib.peps_last_error.argtypes = []
    lib.peps_last_error.restype = ctypes.c_char_p
    lib.peps_num_params.argtypes = [P]
    lib.peps_num_params.restype = Z
    lib.peps_env_cache_bytes.argtypes = [P, I]
    lib.peps_env_cache_bytes.restype = Z
    lib.peps_set_hamiltonian.argtypes = [P, I, P, P, P, I, P, P, P]
    lib.peps_set_hamiltonian.restype = I
    lib.peps_amplitude.argtypes = [P, P, P, I, P, P, P, P]
    lib.peps_amplitude.restype = I
    lib.peps_local_energy.argtypes = [P, P, P, I, P, P, P, P]
    lib.peps_local_energy.restype = I
    lib.peps_local_energy_strict.argtypes = [P, P, P, I, P, P, P]
    lib.peps_local_energy_strict.restype = I
    lib.peps_set_truncation.argtypes = [P, ctypes.c_double]
    lib.peps_set_truncation.restype = I
    lib.peps_set_compression.argtypes = [P, I]
    lib.peps_set_compression.restype = I
    lib.peps_set_minsr_solver.argtypes = [P, I]
    lib.peps_set_minsr_solver.restype = I
    lib.peps_direct_sample.argtypes = [P, P, I, I, I, ctypes.c_uint64, ctypes.c_uint64, P, P, P,
                                       P, P]
    lib.peps_direct_sample.restype = I
    lib.peps_logderiv.argtypes = [P, P, P, I, P, P, P]
    lib.peps_logderiv.restype = I
    lib.peps_evaluate.argtypes = [P, P, P, I, P, P, P, P, P]
    lib.peps_evaluate.restype = I
    lib.minsr_step.argtypes = [P, P, P, I, P, D, D, P, P, P]
    lib.minsr_step.restype = I
    lib.minsr_step_noalloc.argtypes = [P, P, P, I, P, D, D, P, P, P]
    lib.minsr_step_noalloc.restype = I
    lib.peps_sample.argtypes = [P, P, I, I, I, I, I, U64, U64, P, P, P, P, P]
    lib.peps_sample.restype = I
    lib.peps_vmc_step.argtypes = [P, P, I, I, I, I, I, U64, U64, D, D, D, P, P, P, P, P]
    lib.peps_vmc_step.restype = I
    lib.peps_profile.argtypes = [P, I]
    lib.peps_profile.restype = I
    lib.peps_profile_read.argtypes = [P, P, P, I]
    lib.peps_profile_read.restype = I
    lib.made_create.argtypes = [I, I, I, I, ctypes.POINTER(P)]
    lib.made_create.restype = I
    lib.made_destroy.argtypes = [P]
    lib.made_destroy.restype = None
    lib.made_num_params.argtypes = [P]
    lib.made_num_params.restype = Z
    lib.made_loss_grad.argtypes = [P, P, P, I, P, P, P]
    lib.made_loss_grad.restype = I
    lib.made_adam_step.argtypes = [P, P, P, P, P, I, D, D, D, D, P]
    lib.made_adam_step.restype = I
    lib.made_train.argtypes = [P, P, P, I, I, I, I, D, D, D, D, U64, P, P, P, P]
    lib.made_train.restype = I
    lib.peps_tau_int.argtypes = [P, I, I, I, D, P, P, P]
    lib.peps_tau_int.restype = I
    lib.made_sample.argtypes = [P, P, I, U64, U64, P, P, P]
    lib.made_sample.restype = I
    lib.made_logq.argtypes = [P, P, P, I, P, P]
    lib.made_logq.restype = I
    lib.imh_step.argtypes = [I, I, P, P, P, P, P, P, U64, U64, P, P]
    lib.imh_step.restype = I
    lib.peps_logderiv_vjp.argtypes = [P, P, P, I, P, P, P]
    lib.peps_logderiv_vjp.restype = I
    lib.peps_rotate_basis.argtypes = [P, P, I, P, P]
    lib.peps_rotate_basis.restype = I
    lib.peps_energy_diag.argtypes = [P, P, I, P, P]
    lib.peps_energy_diag.restype = I
    _lib = lib
    return lib


def torch_uint8():
    import torch
    return torch.uint8


def _check(st):
    if st != PEPS_OK:
        raise PepsError(st, load().peps_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One geometry (Lx x Ly, D, chi) and one compute precision."""

    def __init__(self, Lx, Ly, D, chi, dtype="f64", d=2):
        lib = load()
        self.Lx, self.Ly, self.D, self.chi, self.d = Lx, Ly, D, chi, d
        self.dtype = dtype
        g = Geom(Lx, Ly, d, D, chi, DTYPES[dtype])
        h = ctypes.c_void_p()
        _check(lib.peps_create(ctypes.byref(g), ctypes.byref(h)))
        self._h = h
        self.n_params = lib.peps_num_params(h)
        self.n_compact = self.n_params // d

    def close(self):
        if getattr(self, "_h", None):
            load().peps_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def is_complex(self):
        return self.dtype in COMPLEX

    @property
    def theta_dtype(self):
        import torch
        return torch.complex128 if self.is_complex else torch.float64

    @property
    def o_dtype(self):
        import torch
        return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32,
                "c128": torch.complex128, "c64": torch.complex64}[self.dtype]

    def env_cache_bytes(self, n):
        return load().peps_env_cache_bytes(self._h, n)

    def set_hamiltonian(self, ham):
        """ham: dict from hamiltonians.* (host numpy arrays)."""
        nt = len(ham["nsites"])
        ns = np.ascontiguousarray(ham["nsites"], dtype=np.int32)
        st = np.ascontiguousarray(ham["sites"], dtype=np.int32).reshape(-1)
        mats = np.ascontiguousarray(ham["mats"], dtype=np.float64).reshape(-1)
        pij = np.ascontiguousarray(ham["pair_ij"], dtype=np.int32).reshape(-1)
        pv = np.ascontiguousarray(ham["pair_v"], dtype=np.float64)
        on = ham.get("onsite")
        on = None if on is None else np.ascontiguousarray(on, dtype=np.float64).reshape(-1)
        self._ham_keep = (ns, st, mats, pij, pv, on)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None
        _check(load().peps_set_hamiltonian(self._h, nt, c(ns), c(st), c(mats), len(pv), c(pij),
                                          c(pv), c(on)))

    def _theta(self, theta):
        """theta as the library reads it: FP64, or interleaved (re, im) FP64
        pairs for complex parameters."""
        assert theta.dtype == self.theta_dtype and theta.is_cuda and theta.numel() == self.n_params
        theta = theta.contiguous()
        return theta

    def _args(self, theta, samples):
        assert samples.dtype == torch_uint8() and samples.is_cuda
        assert samples.dim() == 2 and samples.shape[1] == self.Lx * self.Ly
        return self._theta(theta), samples.contiguous()

    def amplitude(self, theta, samples, env_cache=None, flags=None):
        import torch
        theta, samples = self._args(theta, samples)
        n = samples.shape[0]
        logpsi = torch.empty(n, 2, dtype=torch.float64, device=theta.device)
        if flags is None:
            flags = torch.zeros(n, dtype=torch.int32, device=theta.device)
        _check(load().peps_amplitude(self._h, _ptr(theta), _ptr(samples), n, _ptr(env_cache),
                                     _ptr(logpsi), _ptr(flags), _stream()))
        return logpsi, flags

    def new_env_cache(self, n, device="cuda"):
        import torch
        return torch.empty(self.env_cache_bytes(n), dtype=torch.uint8, device=device)

    def local_energy(self, theta, samples, env_cache=None, flags=None):
        import torch
        theta, samples = self._args(theta, samples)
        n = samples.shape[0]
        eloc = torch.empty(n, 2, dtype=torch.float64, device=theta.device)
        _check(load().peps_local_energy(self._h, _ptr(theta), _ptr(samples), n, _ptr(env_cache),
                                        _ptr(eloc), _ptr(flags), _stream()))
        return eloc

    def direct_sample(self, theta, n, chi_double, seed, offset=0, want_logw=True, refresh=True):
        """n independent configurations from the direct sampler; returns
        (samples [n, N] uint8, ln p [n], ln w [n] or None, flags [n]).
        refresh=False reuses the double-layer environments of the last
        refresh (possibly of older tensors)."""
        import torch
        theta = self._theta(theta)
        dev = theta.device
        samples = torch.empty(n, self.Lx * self.Ly, dtype=torch.uint8, device=dev)
        logp = torch.empty(n, dtype=torch.float64, device=dev)
        logw = torch.empty(n, dtype=torch.float64, device=dev) if want_logw else None
        flags = torch.zeros(n, dtype=torch.int32, device=dev)
        _check(load().peps_direct_sample(self._h, _ptr(theta), n, int(chi_double),
                                         1 if refresh else 0, int(seed), int(offset),
                                         _ptr(samples), _ptr(logp), _ptr(logw), _ptr(flags),
                                         _stream()))
        return samples, logp, logw, flags

    def set_truncation(self, max_weight):
        """Maximal truncated weight of every boundary-MPS truncation (0: keep
        chi singular values per bond)."""
        _check(load().peps_set_truncation(self._h, float(max_weight)))

    def set_compression(self, method):
        """Truncation algorithm of the environment kernels (evaluation and
        the Metropolis sampler): "canonical" (QR then SVD; the faster one at
        chi*D <= 64) or "densmat" (the density-matrix algorithm on the matrix
        cores; the faster one above, about 16x at 10x10 D=5 chi=25)."""
        _check(load().peps_set_compression(self._h, COMPRESS[method]))
        self.compression = method

    def set_minsr_solver(self, solver):
        """Solver of minsr_step: "cholesky" (certified, NaN when the
        certificate fails), "eigh" (eigendecomposition, n <= 3072) or
        "auto" (Cholesky, eigendecomposition after a failed certificate)."""
        _check(load().peps_set_minsr_solver(self._h, MINSR_SOLVER[solver]))
        self.minsr_solver = solver

    def local_energy_strict(self, theta, samples, flags=None):
        """E_loc with every amplitude from the full contraction at the one
        cut (the variational-bound estimator); returns eloc [n, 2]."""
        import torch
        theta, samples = self._args(theta, samples)
        n = samples.shape[0]
        eloc = torch.empty(n, 2, dtype=torch.float64, device=theta.device)
        _check(load().peps_local_energy_strict(self._h, _ptr(theta), _ptr(samples), n,
                                               _ptr(eloc), _ptr(flags), _stream()))
        return eloc

    def rotate_basis(self, theta, basis):
        """Parameters of U_b^(x N) Psi (basis "x": Hadamard, "y": H S^dagger,
        complex contexts only; "z" copies), same layout as theta."""
        import torch
        theta = self._theta(theta)
        out = torch.empty_like(theta)
        _check(load().peps_rotate_basis(self._h, _ptr(theta), BASIS[basis], _ptr(out), _stream()))
        return out

    def energy_diag(self, samples):
        """Diagonal part of the context's Hamiltonian per configuration,
        [n, 2] (re, im); no amplitude is computed."""
        import torch
        assert samples.dtype == torch_uint8() and samples.is_cuda
        assert samples.dim() == 2 and samples.shape[1] == self.Lx * self.Ly
        samples = samples.contiguous()
        n = samples.shape[0]
        eloc = torch.empty(n, 2, dtype=torch.float64, device=samples.device)
        _check(load().peps_energy_diag(self._h, _ptr(samples), n, _ptr(eloc), _stream()))
        return eloc

    def rotated_energy(self, theta, sets, n_chains=256, per_chain=8, burn_in=32, seed=0):
        """Rotated-basis estimate of <H> (Sec. "On reusing environments and
        the convenient treatment of long-range interactions"): for every
        (basis, diagonal term set) of ``sets`` the rotated PEPS is sampled
        with single-spin flips and the set's diagonal energy averaged.
        Replaces the context's Hamiltonian. Returns {basis: (mean, standard
        error over chains)} and their sum under "total"."""
        import torch
        out, tot, var = {}, 0.0, 0.0
        for b, ham in sets.items():
            th = self.rotate_basis(theta, b)
            self.set_hamiltonian(ham)
            smp, _ = self.sample(th, "flip", n_chains=n_chains, per_chain=per_chain,
                                 burn_in=burn_in, seed=seed)
            e = self.energy_diag(smp)[:, 0].reshape(n_chains, per_chain).mean(dim=1)
            mean = float(e.mean())
            err = float(e.std() / n_chains ** 0.5) if n_chains > 1 else float("nan")
            out[b] = (mean, err)
            tot += mean
            var += err * err
        out["total"] = (tot, var ** 0.5)
        return out

    def logderiv(self, theta, samples, env_cache=None):
        import torch
        theta, samples = self._args(theta, samples)
        n = samples.shape[0]
        O = torch.empty(n, self.n_compact, dtype=self.o_dtype, device=theta.device)
        _check(load().peps_logderiv(self._h, _ptr(theta), _ptr(samples), n, _ptr(env_cache),
                                    _ptr(O), _stream()))
        return O

    def evaluate(self, theta, samples, want_e=True, want_o=True, out=None):
        """Fused ln Psi + E_loc + O; returns (logpsi, eloc, O, flags)."""
        import torch
        theta, samples = self._args(theta, samples)
        n = samples.shape[0]
        dev = theta.device
        if out is None:
            out = (torch.empty(n, 2, dtype=torch.float64, device=dev),
                   torch.empty(n, 2, dtype=torch.float64, device=dev) if want_e else None,
                   torch.empty(n, self.n_compact, dtype=self.o_dtype, device=dev) if want_o else None,
                   torch.zeros(n, dtype=torch.int32, device=dev))
        logpsi, eloc, O, flags = out
        _check(load().peps_evaluate(self._h, _ptr(theta), _ptr(samples), n, _ptr(logpsi),
                                    _ptr(eloc), _ptr(O), _ptr(flags), _stream()))
        return logpsi, eloc, O, flags

    def minsr_step(self, O, samples, eloc, eps=1e-4, rcond=1e-12):
        import torch
        n = samples.shape[0]
        assert O.dtype == self.o_dtype and O.shape == (n, self.n_compact)
        dtheta = torch.empty(self.n_params, dtype=self.theta_dtype, device=O.device)
        diag = torch.zeros(8, dtype=torch.float64, device=O.device)
        _check(load().minsr_step(self._h, _ptr(O.contiguous()), _ptr(samples.contiguous()), n,
                                 _ptr(eloc.contiguous()), float(eps), float(rcond), _ptr(dtheta),
                                 _ptr(diag), _stream()))
        return dtheta, diag

    def minsr_step_noalloc(self, O, samples, eloc, eps=1e-4, rcond=1e-12, dtheta=None,
                           diag=None):
        """minsr_step with the library's fixed device workspace (no device
        allocation inside the call); dtheta and diag may be given."""
        import torch
        n = samples.shape[0]
        assert O.dtype == self.o_dtype and O.shape == (n, self.n_compact)
        if dtheta is None:
            dtheta = torch.empty(self.n_params, dtype=self.theta_dtype, device=O.device)
        if diag is None:
            diag = torch.zeros(8, dtype=torch.float64, device=O.device)
        _check(load().minsr_step_noalloc(self._h, _ptr(O), _ptr(samples), n, _ptr(eloc), float(eps),
                                         float(rcond), _ptr(dtheta), _ptr(diag), _stream()))
        return dtheta, diag

    def logderiv_vjp(self, O, samples, g):
        """sum_s g_s dln|Psi(S_s)|/dtheta (complex parameters: d/dRe + i d/dIm)."""
        import torch
        out = torch.empty(self.n_params, dtype=self.theta_dtype, device=O.device)
        _check(load().peps_logderiv_vjp(self._h, _ptr(O.contiguous()), _ptr(samples.contiguous()),
                                        samples.shape[0], _ptr(g.contiguous()), _ptr(out),
                                        _stream()))
        return out

    def log_abs_psi(self, theta, samples):
        """ln|Psi(S)| as a differentiable function of theta (see LogAbsPsi)."""
        return LogAbsPsi.apply(theta, samples, self)

    def profile(self, enable=True):
        _check(load().peps_profile(self._h, 1 if enable else 0))

    def profile_read(self, reset=True):
        """{kind: (total ms, launches)} from the library's HIP events."""
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_long * 8)()
        _check(load().peps_profile_read(self._h, ctypes.cast(ms, ctypes.c_void_p),
                                        ctypes.cast(cnt, ctypes.c_void_p), 1 if reset else 0))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(PROF_KINDS)}

    def sample(self, theta, kind="exchange", n_chains=256, per_chain=4, burn_in=32, thin=1,
               seed=0, offset=0, proposal=None, want_logpsi=False):
        """Markov chains of |Psi|^2: kind "exchange" / "flip" (local moves) or
        "imh" (independence MH with proposal = (Made, params, init or None)).
        Returns (samples, accepted) or (samples, accepted, logpsi)."""
        import torch
        theta = self._theta(theta)
        n = n_chains * per_chain
        dev = theta.device
        samples = torch.empty(n, self.Lx * self.Ly, dtype=torch.uint8, device=dev)
        acc = torch.zeros(n_chains, dtype=torch.int32, device=dev)
        lp = torch.empty(n, 2, dtype=torch.float64, device=dev) if want_logpsi else None
        k = {"exchange": SAMPLE_EXCHANGE, "flip": SAMPLE_FLIP, "imh": SAMPLE_IMH}[kind]
        pr = None
        if kind == "imh":
            made, params, init = proposal
            pr = Proposal(made._h.value, params.data_ptr(),
                          init.contiguous().data_ptr() if init is not None else None)
            self._keep = (params, init)
        _check(load().peps_sample(self._h, _ptr(theta.contiguous()), k, n_chains, per_chain,
                                  burn_in, thin, seed, offset,
                                  ctypes.byref(pr) if pr is not None else None, _ptr(samples),
                                  _ptr(lp), _ptr(acc), _stream()))
        return (samples, acc, lp) if want_logpsi else (samples, acc)

    def vmc_step(self, theta, tau, kind="exchange", n_chains=256, per_chain=4, burn_in=32,
                 thin=1, seed=0, offset=0, eps=1e-4, rcond=1e-12):
        """One optimisation step (sample, evaluate, minSR, theta -= tau * dtheta);
        theta (device, contiguous) is updated in place. Returns (samples,
        eloc, flags, diag)."""
        import torch
        assert theta.is_contiguous()
        th = self._theta(theta)
        n = n_chains * per_chain
        dev = theta.device
        samples = torch.empty(n, self.Lx * self.Ly, dtype=torch.uint8, device=dev)
        eloc = torch.empty(n, 2, dtype=torch.float64, device=dev)
        flags = torch.zeros(n, dtype=torch.int32, device=dev)
        diag = torch.zeros(8, dtype=torch.float64, device=dev)
        k = SAMPLE_EXCHANGE if kind == "exchange" else SAMPLE_FLIP
        _check(load().peps_vmc_step(self._h, _ptr(th), k, n_chains, per_chain, burn_in, thin,
                                    seed, offset, tau, eps, rcond, _ptr(samples), _ptr(eloc),
                                    _ptr(flags), _ptr(diag), _stream()))
        return samples, eloc, flags, diag

    def optimize(self, theta, steps, tau, kind="exchange", n_chains=256, per_chain=4,
                 burn_in=32, thin=1, seed=0, offset0=0, eps=1e-4, rcond=1e-12):
        """`steps` optimisation steps; step k uses sweep offset
        offset0 + k * (burn_in + per_chain * thin). Returns the batch-mean
        energy of every step (before its update); theta is updated in place."""
        stride = burn_in + per_chain * thin
        energies = []
        for k in range(steps):
            _, _, _, diag = self.vmc_step(theta, tau, kind, n_chains, per_chain, burn_in, thin,
                                          seed, offset0 + k * stride, eps, rcond)
            energies.append(float(diag[4].item()))
        return energies


class Made:
    """Masked autoregressive proposal q over N sites (hidden width H)."""

    def __init__(self, N, H=256, n_up=None, bf16=False):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.made_create(N, H, -1 if n_up is None else n_up, 1 if bf16 else 0,
                               ctypes.byref(h)))
        self._h = h
        self.N, self.H, self.n_up = N, H, n_up
        self.n_params = lib.made_num_params(h)

    def close(self):
        if getattr(self, "_h", None):
            load().made_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def loss_grad(self, params, x, grads=None, loss=None):
        import torch
        B = x.shape[0]
        if grads is None:
            grads = torch.empty_like(params)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=params.device)
        _check(load().made_loss_grad(self._h, _ptr(params), _ptr(x), B, _ptr(grads), _ptr(loss),
                                     _stream()))
        return loss, grads

    def adam(self, params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(load().made_adam_step(self._h, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), t,
                                     lr, beta1, beta2, eps, _stream()))

    def sample(self, params, n, seed=0, offset=0):
        import torch
        out = torch.empty(n, self.N, dtype=torch.uint8, device=params.device)
        lq = torch.empty(n, dtype=torch.float64, device=params.device)
        _check(load().made_sample(self._h, _ptr(params), n, seed, offset, _ptr(out), _ptr(lq),
                                  _stream()))
        return out, lq

    def logq(self, params, x):
        import torch
        lq = torch.empty(x.shape[0], dtype=torch.float64, device=params.device)
        _check(load().made_logq(self._h, _ptr(params), _ptr(x.contiguous()), x.shape[0], _ptr(lq),
                                _stream()))
        return lq

    def train(self, params, data, steps, batch=1024, lr=1e-3, seed=0):
        """Adam on mean -ln q over permuted mini-batches of `data` (uint8
        [M][N] on the device), all steps in one library call (made_train);
        returns the per-step losses (device tensor)."""
        import torch
        m = torch.zeros_like(params)
        v = torch.zeros_like(params)
        losses = torch.empty(steps, dtype=torch.float64, device=params.device)
        data = data.contiguous()
        _check(load().made_train(self._h, _ptr(params), _ptr(data), data.shape[0], steps, batch, 0,
                                 lr, 0.9, 0.999, 1e-8, int(seed), _ptr(m), _ptr(v), _ptr(losses),
                                 _stream()))
        return losses


def imh_step(state, state_lp, state_lq, prop, prop_lp, prop_lq, seed, step, accepted):
    """One independence Metropolis-Hastings step on device tensors."""
    n, N = state.shape
    _check(load().imh_step(n, N, _ptr(state), _ptr(state_lp), _ptr(state_lq), _ptr(prop),
                           _ptr(prop_lp), _ptr(prop_lq), seed, step, _ptr(accepted), _stream()))


def run_imh(ctx, theta, made, params, n_chains, n_steps, seed=0, record=None, init=None):
    """Independence MH chains driven by the learned proposal, in one library
    call (peps_sample with kind "imh"): every step draws one proposal per
    chain from q, evaluates its ln|Psi| and accepts with the PEPS as the
    arbiter. Chains start from `init` (uint8 [n_chains][N] on the device,
    e.g. local-Metropolis samples) or from a draw of q. Returns the final
    states, the visited states per step ([n_steps][n_chains][N] if record)
    and the acceptance counts."""
    s, acc = ctx.sample(theta, "imh", n_chains=n_chains, per_chain=n_steps, burn_in=0, thin=1,
                        seed=seed, offset=0, proposal=(made, params, init))
    hist = s.view(n_chains, n_steps, -1).permute(1, 0, 2)
    return hist[-1].contiguous(), (hist.contiguous() if record else None), acc


def _autograd_function():
    import torch

    class _LogAbsPsi(torch.autograd.Function):
        """ln|Psi(S)| of a batch with the hand-written adjoint as backward.

        Forward: peps_amplitude (ln|Psi| at the middle cut). Backward: the
        environments are rebuilt (not stored) and the one-row hole networks
        give O_k = d ln Psi_row(x)(S)/d theta_k (peps_logderiv); the gradient
        is sum_s g_s O_s for real parameters and sum_s g_s conj(O_s) (PyTorch's
        d/dRe + i d/dIm) for complex ones (peps_logderiv_vjp). In the exact-contraction
        regime this is the exact derivative of the forward value; below the
        exact Schmidt rank it is the strip derivative (the cut of the
        forward value and the strip of row x are different approximations).
        """

        @staticmethod
        def forward(fctx, theta, samples, ctx):
            lp, _ = ctx.amplitude(theta, samples)
            fctx.save_for_backward(theta, samples)
            fctx.pctx = ctx
            return lp[:, 0].clone()

        @staticmethod
        def backward(fctx, g):
            theta, samples = fctx.saved_tensors
            ctx = fctx.pctx
            O = ctx.logderiv(theta, samples)
            grad = ctx.logderiv_vjp(O, samples, g.to(torch.float64).contiguous())
            return grad, None, None

    return _LogAbsPsi


class _LazyFn:
    _fn = None

    def apply(self, *args):
        if _LazyFn._fn is None:
            _LazyFn._fn = _autograd_function()
        return _LazyFn._fn.apply(*args)


LogAbsPsi = _LazyFn()
