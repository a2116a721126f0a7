"""Helpers shared by the GPU tests: running the oracle on the same seeded
inputs the library gets, and comparing log-amplitudes."""
import numpy as np

import synth
from oracle import hamiltonian as OH
from oracle import peps


def oracle_eval(theta, Lx, Ly, D, chi, configs, model=None, want_O=False, method="canonical",
                cutoff=0.0):
    g = peps.Geometry(Lx, Ly, 2, D)
    ham = oracle_ham(model, Lx, Ly) if model else None
    return peps.evaluate(theta, g, configs, chi, ham, want_O=want_O, method=method,
                         cutoff=cutoff)


def oracle_ham(model, Lx, Ly):
    name, kw = model
    if name == "j1j2":
        return OH.j1j2(Lx, Ly, **kw)
    if name == "chiral":
        return OH.csl(Lx, Ly, **kw)
    if name == "rydberg":
        return OH.rydberg(Lx, Ly, **kw)
    raise ValueError(name)


def product_ham(model, Lx, Ly):
    from paper_2503_12557_amd import hamiltonians as HB
    name, kw = model
    if name == "j1j2":
        return HB.j1j2(Lx, Ly, **kw)
    if name == "chiral":
        return HB.chiral(Lx, Ly, J1=kw["J1"], J2=kw["J2"], Jchi=kw["Jchi"])
    if name == "rydberg":
        return HB.rydberg(Lx, Ly, **kw)
    raise ValueError(name)


def logpsi_to_complex(lp):
    """(ln|psi|, arg) pairs -> complex log."""
    lp = np.asarray(lp)
    return lp[:, 0] + 1j * lp[:, 1]


def rel_amp_err(gpu_lp, ora_lp):
    """|psi_gpu / psi_oracle - 1| per sample from complex logs."""
    d = logpsi_to_complex(gpu_lp) - np.asarray(ora_lp)
    return np.abs(np.exp(d) - 1.0)


def configs_for(model, N, n, seed):
    if model is not None and model[0] == "rydberg":
        return synth.bit_configs(N, n, seed)
    return synth.sz0_configs(N, n, seed)
