"""The oracle optimisation loop (repeated minSR steps) against exact
diagonalisation: at 2x2 every state is enumerated, so the variational
energy of each iterate is exact. It must stay above the ground-state energy
(variational principle) and fall well below the starting energy."""
import numpy as np
import pytest

import synth
from oracle import hamiltonian as ham
from oracle import peps, vmc


def _exact_energy(theta, g, Hm, confs):
    psi = peps.exact_amplitudes(theta, g, confs)
    return float(np.real(np.vdot(psi, Hm @ psi) / np.vdot(psi, psi)))


def test_minsr_loop_descends_towards_the_ground_state_at_2x2():
    Lx = Ly = 2
    g = peps.Geometry(Lx, Ly, 2, 2)
    H = ham.j1j2(Lx, Ly, 1.0, 0.0)
    basis = ham.sz0_basis(4)
    Hm = ham.sparse_matrix(H, basis).toarray()
    confs = np.array([ham.int_to_config(v, 4) for v in basis])
    e0 = float(np.linalg.eigvalsh(Hm.real)[0])
    # four-site Heisenberg ring: E0 = -2 J (S = 1/2, H = sum S_i . S_j)
    assert abs(e0 + 2.0) < 1e-12
    th0 = synth.theta(Lx, Ly, 2, 2, seed=1)
    e_start = _exact_energy(th0, g, Hm, confs)
    th, batch = vmc.optimize(th0, g, 4, H, 'exchange', 16, 4, 4, 1, seed=7, tau=0.1, eps=1e-4,
                             rcond=1e-12, steps=12)
    e_end = _exact_energy(th, g, Hm, confs)
    assert e_end >= e0 - 1e-12
    assert e_start - e_end > 0.5 * (e_start - e0)
    # the batch means follow the exact energies downwards
    assert batch[-3:].mean() < batch[:3].mean()


def test_step_offsets_use_disjoint_random_streams():
    # consecutive steps read disjoint Philox counters: a zero step (tau = 0)
    # keeps theta, yet the second step's samples differ from the first's
    Lx, Ly = 2, 2
    g = peps.Geometry(Lx, Ly, 2, 2)
    H = ham.j1j2(Lx, Ly, 1.0, 0.0)
    th0 = synth.theta(Lx, Ly, 2, 2, seed=3)
    a = vmc.step(th0, g, 4, H, 'exchange', 8, 2, 2, 1, 5, 0, 0.0, 1e-4, 1e-12)
    b = vmc.step(th0, g, 4, H, 'exchange', 8, 2, 2, 1, 5, 4, 0.0, 1e-4, 1e-12)
    assert np.array_equal(a[0], th0)
    assert not np.array_equal(a[2], b[2])
