"""Pins of the oracle's rotated-basis estimator (Sec. "On reusing
environments and the convenient treatment of long-range interactions"; the
unbiased estimator of App. "Sampling-based PEPS schemes can yield a
variational upper bound on the energy").

- each U_b takes its Pauli matrix to Z (the defining property), with the
  Paulis of the oracle's Hamiltonian module;
- the rotated parameters give the state vector U_b^(x N) psi, psi and the
  Kronecker product built densely and independently of the rotation code;
- the sum over the X, Y and Z sets of the exact rotated-basis expectations
  equals <psi|H|psi> / <psi|psi> of a long-range Heisenberg Hamiltonian in
  a uniform field, built from dense Kronecker products (real and complex
  tensors), which a transposed or conjugated U, or a wrong sign of the Y
  rotation, fails (the field terms are odd in the Paulis; a real state has
  no Y field energy, so the complex case holds the sign of U_y);
- the diagonal energy equals the diagonal of the dense Hamiltonian;
- rotating twice by X is the identity (H^2 = 1).
"""
import numpy as np
import pytest

import synth
from oracle import hamiltonian as ham
from oracle import peps, rotated

PAULI = {'x': 2 * ham.SX, 'y': 2 * ham.SY, 'z': 2 * ham.SZ}


def _state(theta, g):
    configs = [np.array([(v >> (g.N - 1 - n)) & 1 for n in range(g.N)], dtype=np.uint8)
               for v in range(2 ** g.N)]
    return peps.exact_amplitudes(theta, g, configs).astype(np.complex128)


def _long_range_pairs(g, alpha=1.5):
    out = []
    for i in range(g.N):
        for j in range(i + 1, g.N):
            xi, yi = divmod(i, g.Ly)
            xj, yj = divmod(j, g.Ly)
            r = np.hypot(xi - xj, yi - yj)
            out.append((i, j, 1.0 / r ** alpha))
    return out


@pytest.mark.parametrize('b', ['x', 'y', 'z'])
def test_rotation_takes_its_pauli_to_z(b):
    U = rotated.rotation(b)
    np.testing.assert_allclose(U @ U.conj().T, np.eye(2), atol=1e-15)
    np.testing.assert_allclose(U @ PAULI[b] @ U.conj().T, PAULI['z'], atol=1e-15)


@pytest.mark.parametrize('b', ['x', 'y'])
@pytest.mark.parametrize('cplx', [False, True])
def test_rotated_parameters_give_the_rotated_state(b, cplx):
    g = peps.Geometry(2, 3, 2, 2)
    theta = synth.theta(2, 3, 2, 2, seed=11, cplx=cplx)
    psi = _state(theta, g)
    Ufull = ham.kron(*([rotated.rotation(b)] * g.N))
    psi_b = _state(rotated.rotate_theta(theta, g, b), g)
    np.testing.assert_allclose(psi_b, Ufull @ psi, rtol=0, atol=1e-12 * np.abs(psi).max())


@pytest.mark.parametrize('cplx', [False, True])
def test_sum_of_rotated_sets_is_the_long_range_heisenberg_energy(cplx):
    g = peps.Geometry(2, 3, 2, 2)
    theta = synth.theta(2, 3, 2, 2, seed=12, cplx=cplx)
    psi = _state(theta, g)
    pairs = _long_range_pairs(g)
    # dense H = sum J_ij (X X + Y Y + Z Z) / 4 (spin operators)
    # plus a uniform field h . S on every site: its single-spin terms are odd
    # in each Pauli, so a rotation that maps sigma^b to -Z changes their sign
    field = {'x': 0.3, 'y': -0.7, 'z': 0.5}
    H = np.zeros((2 ** g.N, 2 ** g.N), dtype=np.complex128)
    for (i, j, J) in pairs:
        for P in (ham.SX, ham.SY, ham.SZ):
            H += J * ham.embed(ham.kron(P, P), (i, j), g.N)
    for n in range(g.N):
        for b, P in (('x', ham.SX), ('y', ham.SY), ('z', ham.SZ)):
            H += field[b] * ham.embed(P, (n,), g.N)
    e_dense = (psi.conj() @ H @ psi) / (psi.conj() @ psi)
    # each set in its rotated form: J S^z S^z on the pairs, h_b S^z per site
    zz = ham.kron(ham.SZ, ham.SZ)
    sets = {b: [((i, j), J * zz) for (i, j, J) in pairs]
            + [((n,), field[b] * ham.SZ) for n in range(g.N)] for b in 'xyz'}
    parts = [rotated.exact_set_expectation(theta, g, b, sets[b]) for b in 'xyz']
    e_rot = sum(parts)
    assert abs(e_rot - e_dense) < 1e-12 * max(1.0, abs(e_dense))
    # the sets separately are not equal (the pin is not trivially symmetric)
    assert max(p.real for p in parts) - min(p.real for p in parts) > 1e-3


def test_diagonal_energy_is_the_dense_diagonal():
    g = peps.Geometry(2, 3, 2, 2)
    rng = np.random.default_rng(5)
    H = ham.Hamiltonian(g.N)
    terms = []
    for (i, j) in [(0, 1), (0, 5), (2, 4)]:
        h = np.diag(rng.normal(size=4) + 1j * rng.normal(size=4))
        H.add((i, j), h)
        terms.append(((i, j), h))
    h3 = np.diag(rng.normal(size=8))
    H.add((1, 3, 5), h3)
    terms.append(((1, 3, 5), h3))
    H.pairs = [(0, 4, 0.7), (2, 3, -1.1)]
    H.onsite[:, 1] = rng.normal(size=g.N)
    dense = ham.sparse_matrix(H).toarray()
    for v in range(2 ** g.N):
        s = ham.int_to_config(v, g.N)
        e = rotated.diagonal_energy(terms, H.pairs, H.onsite, s)
        assert abs(e - dense[v, v]) < 1e-13


def test_rotating_twice_by_x_is_the_identity():
    g = peps.Geometry(3, 3, 2, 3)
    theta = synth.theta(3, 3, 2, 3, seed=13, cplx=False)
    back = rotated.rotate_theta(rotated.rotate_theta(theta, g, 'x'), g, 'x')
    np.testing.assert_allclose(back, theta, rtol=0, atol=1e-15 * np.abs(theta).max() * 4)
