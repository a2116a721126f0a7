"""The strict (single-cut) local energy of the oracle: every amplitude of
E_loc is Psi(S)_i* from the full boundary-MPS contraction at the cut i*
(Sec. "On Variational Upper Bound"). Pinned by exact identities:
  * at an exact chi it equals (H Psi)(S) / Psi(S) from the sparse Hamiltonian;
  * at a truncating chi its average over p(S) ~ |Psi(S)_i*|^2, taken over
    every configuration, equals psi^H H psi / psi^H psi for the vector
    psi(S) = Psi(S)_i*, and so lies above the exact ground-state energy."""
import numpy as np
import scipy.sparse.linalg as spla

import synth
from oracle import hamiltonian as ham
from oracle import peps


def _basis_states(N):
    basis = ham.sz0_basis(N)
    return basis, np.array([ham.int_to_config(v, N) for v in basis])


def test_strict_energy_is_exact_at_exact_chi():
    Lx, Ly, D, chi = 4, 4, 2, 4
    g = peps.Geometry(Lx, Ly, 2, D)
    H = ham.j1j2(Lx, Ly, 1.0, 0.5)
    basis, confs = _basis_states(16)
    th = synth.theta(Lx, Ly, 2, D, seed=4)
    psi = peps.exact_amplitudes(th, g, confs)
    Hpsi = ham.sparse_matrix(H, basis) @ psi
    pick = np.random.default_rng(2).choice(len(basis), 3, replace=False)
    e = peps.local_energy_strict(th, g, confs[pick], chi, H)
    ref = Hpsi[pick] / psi[pick]
    assert np.abs(e - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_strict_energy_is_the_energy_of_the_fixed_cut_vector():
    # 3 x 2, D = 3, chi = 2: the bottom environment of rows 1-2 is truncated
    Lx, Ly, D, chi = 3, 2, 3, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    H = ham.j1j2(Lx, Ly, 1.0, 0.0)
    basis, confs = _basis_states(6)
    th = synth.theta(Lx, Ly, 2, D, seed=9)
    lp, _, _ = peps.evaluate(th, g, confs, chi)
    psi = np.exp(lp)                       # the fixed-cut amplitude vector
    exact = peps.exact_amplitudes(th, g, confs)
    assert np.abs(psi / exact - 1).max() > 1e-3   # chi = 2 truncates
    Hm = ham.sparse_matrix(H, basis)
    e_vec = float(np.real(np.vdot(psi, Hm @ psi) / np.vdot(psi, psi)))
    e = peps.local_energy_strict(th, g, confs, chi, H)
    p = np.abs(psi) ** 2
    e_avg = float(np.real((p * e).sum() / p.sum()))
    assert abs(e_avg - e_vec) <= 1e-10 * abs(e_vec)
    e0 = float(np.linalg.eigvalsh(Hm.toarray().real)[0])
    assert e_avg >= e0 - 1e-12
