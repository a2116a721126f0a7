"""Pins of the oracle's minSR step (CPU only): push-through identity with the
parameter-space SR form, eigh vs Cholesky, minimum-norm least squares and
energy descent at 4x4."""
import numpy as np
import pytest

import synth
from oracle import hamiltonian as ham
from oracle import minsr, peps


def _random_problem(ns, npar, cplx, seed):
    rng = np.random.default_rng(seed)
    O = rng.standard_normal((ns, npar))
    E = rng.standard_normal(ns)
    if cplx:
        O = O + 1j * rng.standard_normal((ns, npar))
        E = E + 1j * rng.standard_normal(ns)
    # inactive (zero) entries as in a real O matrix
    O[rng.random((ns, npar)) < 0.5] = 0
    return O, E


@pytest.mark.parametrize("cplx", [False, True])
def test_push_through_identity(cplx):
    # O^dag (O O^dag + eps)^-1 E = (O^dag O + eps)^-1 O^dag E
    O, E = _random_problem(64, 288, cplx, 1)
    a, _ = minsr.minsr_eigh(O, E, 1e-4, 1e-12)
    b = minsr.sr_parameter_space(O, E, 1e-4)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


@pytest.mark.parametrize("cplx", [False, True])
def test_eigh_equals_cholesky_when_cut_inactive(cplx):
    O, E = _random_problem(200, 500, cplx, 2)
    a, info = minsr.minsr_eigh(O, E, 1e-4, 1e-12)
    assert info['n_cut'] == 0
    b = minsr.minsr_cholesky(O, E, 1e-4)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


def test_zero_eps_is_minimum_norm_least_squares():
    O, E = _random_problem(50, 400, False, 3)
    a, _ = minsr.minsr_eigh(O, E, 0.0, 1e-12)
    Ob, Eb = minsr.centre(O, E)
    ref = np.linalg.lstsq(Ob, Eb, rcond=None)[0]
    assert np.abs(a - ref).max() <= 1e-9 * np.abs(ref).max()


def test_minsr_step_lowers_the_exact_energy_at_4x4():
    # one minSR step from exactly drawn samples lowers <H> for a small step
    Lx = Ly = 4
    g = peps.Geometry(Lx, Ly, 2, 2)
    H = ham.j1j2(Lx, Ly, 1.0, 0.0)
    basis = ham.sz0_basis(16)
    Hm = ham.sparse_matrix(H, basis)
    confs = np.array([ham.int_to_config(v, 16) for v in basis])
    th = synth.theta(Lx, Ly, 2, 2, seed=1)

    def energy(t):
        psi = peps.exact_amplitudes(t, g, confs)
        return float(np.real(np.vdot(psi, Hm @ psi) / np.vdot(psi, psi))), psi

    e0, psi = energy(th)
    p = np.abs(psi) ** 2
    p /= p.sum()
    rng = np.random.default_rng(5)
    pick = rng.choice(len(basis), 512, p=p)
    logpsi, eloc, Oc = peps.evaluate(th, g, confs[pick], 4, H, want_O=True)
    O = np.array([peps.expand_compact(Oc[i], g, confs[pick[i]]) for i in range(len(pick))])
    dth, _ = minsr.minsr_eigh(O, eloc.real, 1e-4, 1e-12)
    e1, _ = energy(th - 0.02 * dth.real)
    assert e1 < e0
