"""Oracle rotated-basis energy estimator (Sec. "On reusing environments and
the convenient treatment of long-range interactions", last paragraphs, and
the unbiased estimator of App. "Sampling-based PEPS schemes can yield a
variational upper bound on the energy").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A Hamiltonian whose terms fall into sets that are each diagonal in one
product basis (for a long-range Heisenberg model: the X X, Y Y and Z Z
terms) is estimated set by set: the PEPS is rotated by one global
single-site unitary U_b that maps the basis of set b to the computational
one, configurations are drawn from |Psi_b(S)|^2 with Psi_b = U_b^(x N) Psi,
and the local energy of the set is its diagonal value in the rotated basis,
<Psi|H_b|Psi> / <Psi|Psi> = sum_S |Psi_b(S)|^2 h_b(S) / sum_S |Psi_b(S)|^2,
with h_b(S) = <S| U_b H_b U_b^dagger |S>. No amplitude ratio enters, so the
estimate does not depend on how the amplitudes were approximated.

Readings taken here:
  * the unitaries: U_z = 1, U_x = H (Hadamard, H X H = Z), U_y = H S^dagger
    with S = diag(1, i) (S^dagger Y S = X), so U_b sigma^b U_b^dagger = Z
    for every b; the rotated site tensor is T_b[s] = sum_p U_b[s, p] T[p]
    on the physical index (basis 0 = up, the +1 eigenvector of Z);
  * the sets carry their terms already in the rotated (diagonal) form, as
    (sites, h) with h diagonal, the way the library takes a Hamiltonian.
"""
from __future__ import annotations

import numpy as np

from . import peps

SQ2 = 1.0 / np.sqrt(2.0)


def rotation(basis: str) -> np.ndarray:
    """U_b with U_b sigma^b U_b^dagger = Z (b in 'z', 'x', 'y')."""
    if basis == 'z':
        return np.eye(2, dtype=np.complex128)
    h = SQ2 * np.array([[1, 1], [1, -1]], dtype=np.complex128)
    if basis == 'x':
        return h
    if basis == 'y':
        return h @ np.diag([1.0, -1.0j])
    raise ValueError(basis)


def rotate_theta(theta, g: peps.Geometry, basis: str):
    """Parameters of U_b^(x N) Psi: every site tensor's physical index
    multiplied by U_b. Returns complex128 for 'y' (and for complex theta),
    else float64."""
    U = rotation(basis)
    T = peps.site_tensors(theta, g)
    out = []
    for x in range(g.Lx):
        for y in range(g.Ly):
            t = T[(x, y)]
            out.append(np.einsum('sp,p...->s...', U, t).reshape(-1))
    th = np.concatenate(out)
    if basis != 'y' and not np.iscomplexobj(theta):
        assert np.abs(th.imag).max() == 0.0
        return th.real.copy()
    return th


def diagonal_energy(terms, pairs, onsite, s) -> complex:
    """h(S) of a diagonal Hamiltonian: sum_t h_t[c_t, c_t] (c_t the local
    index of the term's sites, first site most significant) + sum V_ij n_i
    n_j + sum onsite[n, s_n]."""
    e = 0.0 + 0.0j
    for sites, h in terms:
        c = 0
        for n in sites:
            c = 2 * c + int(s[n])
        e += h[c, c]
    for (i, j, v) in pairs:
        if s[i] == 1 and s[j] == 1:
            e += v
    if onsite is not None:
        for n in range(len(s)):
            e += onsite[n, int(s[n])]
    return e


def exact_set_expectation(theta, g: peps.Geometry, basis: str, terms):
    """sum_S |Psi_b(S)|^2 h_b(S) / sum_S |Psi_b(S)|^2 over all 2^N
    configurations, the amplitudes by brute-force contraction."""
    th = rotate_theta(theta, g, basis)
    configs = [np.array([(v >> (g.N - 1 - n)) & 1 for n in range(g.N)], dtype=np.uint8)
               for v in range(2 ** g.N)]
    amp = peps.exact_amplitudes(th, g, configs)
    w = np.abs(amp) ** 2
    h = np.array([diagonal_energy(terms, [], None, s) for s in configs])
    return complex(np.sum(w * h) / np.sum(w))
