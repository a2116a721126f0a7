"""Hamiltonian term tables for peps_set_hamiltonian (host side).

Basis per site: 0 = spin up (S^z = +1/2) or atom in |g>, 1 = spin down or
|r>. A k-site term is the matrix <c|h|c'> with the first site as the most
significant bit of c, stored in an 8 x 8 complex block.

Models (arXiv 2503.12557):
  * J1-J2 Heisenberg, Sec. "Entanglement scaling and comparison to Tree
    Tensor Networks";
  * chiral spin liquid: J1-J2 plus a three-spin chirality on the four
    triangles of every plaquette; the paper's plaquette ring term
    i*lam*(P - P^-1) equals 2*lam times that four-triangle sum (Sec.
    "Chiral spin liquid");
  * Rydberg array Omega/2 sum sigma^x - Delta sum n + sum_{i<j} V/r^6 n n
    (Sec. "Rydberg atom arrays and long-range interactions");
  * long-range Heisenberg sum_{i<j} J / r^alpha S_i . S_j (plus a uniform
    field h . S) as the three sets of the rotated-basis estimator, each in
    its diagonal form (Sec. "On reusing environments and the convenient
    treatment of long-range interactions").
"""
from __future__ import annotations

import numpy as np


def _pauli():
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]], dtype=complex)
    sz = np.array([[1, 0], [0, -1]], dtype=complex)
    return sx, sy, sz


def _spin_dot():
    sx, sy, sz = _pauli()
    return 0.25 * (np.kron(sx, sx) + np.kron(sy, sy) + np.kron(sz, sz))


def _triple():
    # S_i . (S_j x S_k) = sum over the Levi-Civita symbol eps_abc S_i^a S_j^b S_k^c
    s = [m / 2 for m in _pauli()]
    out = np.zeros((8, 8), dtype=complex)
    for a, b, c, sign in [(0, 1, 2, 1), (1, 2, 0, 1), (2, 0, 1, 1),
                          (0, 2, 1, -1), (2, 1, 0, -1), (1, 0, 2, -1)]:
        out += sign * np.kron(np.kron(s[a], s[b]), s[c])
    return out


class _Builder:
    def __init__(self, N):
        self.N = N
        self.nsites, self.sites, self.mats = [], [], []
        self.pair_ij, self.pair_v = [], []
        self.onsite = np.zeros((N, 2))

    def term(self, sites, h):
        k = len(sites)
        block = np.zeros((8, 8, 2))
        block[:2 ** k, :2 ** k, 0] = h.real
        block[:2 ** k, :2 ** k, 1] = h.imag
        self.nsites.append(k)
        self.sites.append(list(sites) + [-1] * (3 - k))
        self.mats.append(block)

    def done(self):
        return dict(nsites=np.array(self.nsites, dtype=np.int32),
                    sites=np.array(self.sites, dtype=np.int32).reshape(-1, 3),
                    mats=np.array(self.mats).reshape(-1, 8, 8, 2) if self.mats else np.zeros((0, 8, 8, 2)),
                    pair_ij=np.array(self.pair_ij, dtype=np.int32).reshape(-1, 2),
                    pair_v=np.array(self.pair_v, dtype=np.float64),
                    onsite=self.onsite)


def _bonds(Lx, Ly):
    nn, nnn = [], []
    for x in range(Lx):
        for y in range(Ly):
            n = x * Ly + y
            if y + 1 < Ly:
                nn.append((n, n + 1))
            if x + 1 < Lx:
                nn.append((n, n + Ly))
            if x + 1 < Lx and y + 1 < Ly:
                nnn.append((n, n + Ly + 1))
                nnn.append((n + 1, n + Ly))
    return nn, nnn


def j1j2(Lx, Ly, J1=1.0, J2=0.0):
    b = _Builder(Lx * Ly)
    h = _spin_dot()
    nn, nnn = _bonds(Lx, Ly)
    for (i, j) in nn:
        b.term((i, j), J1 * h)
    if J2:
        for (i, j) in nnn:
            b.term((i, j), J2 * h)
    return b.done()


def chiral(Lx, Ly, J1=1.0, J2=0.5, Jchi=0.2):
    b = _Builder(Lx * Ly)
    h = _spin_dot()
    nn, nnn = _bonds(Lx, Ly)
    for (i, j) in nn:
        b.term((i, j), J1 * h)
    for (i, j) in nnn:
        b.term((i, j), J2 * h)
    c = _triple()
    for x in range(Lx - 1):
        for y in range(Ly - 1):
            a = x * Ly + y
            bb, cc, e = a + 1, a + Ly + 1, a + Ly
            for tri in ((a, bb, cc), (bb, cc, e), (cc, e, a), (e, a, bb)):
                b.term(tri, Jchi * c)
    return b.done()


def rydberg(Lx, Ly, Omega=1.0, Delta=1.0, V=1.7 ** 6):
    N = Lx * Ly
    b = _Builder(N)
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    for n in range(N):
        b.term((n,), 0.5 * Omega * sx)
        b.onsite[n, 1] = -Delta
    for i in range(N):
        xi, yi = divmod(i, Ly)
        for j in range(i + 1, N):
            xj, yj = divmod(j, Ly)
            r2 = (xi - xj) ** 2 + (yi - yj) ** 2
            b.pair_ij.append((i, j))
            b.pair_v.append(V / float(r2) ** 3)
    return b.done()


def long_range_heisenberg_sets(Lx, Ly, J=1.0, alpha=3.0, field=(0.0, 0.0, 0.0)):
    """The X X, Y Y and Z Z parts of sum_{i<j} J / r_ij^alpha S_i . S_j +
    sum_n (h_x S^x_n + h_y S^y_n + h_z S^z_n), each rotated to the Z basis
    (J / r^alpha S^z S^z per pair, h_b S^z per site): keys "x", "y", "z" for
    the rotations of peps_rotate_basis."""
    N = Lx * Ly
    sz = 0.5 * np.diag([1.0, -1.0]).astype(complex)
    zz = np.kron(sz, sz)
    out = {}
    for b, h in zip("xyz", field):
        bld = _Builder(N)
        for i in range(N):
            xi, yi = divmod(i, Ly)
            for j in range(i + 1, N):
                xj, yj = divmod(j, Ly)
                r = float(np.hypot(xi - xj, yi - yj))
                bld.term((i, j), (J / r ** alpha) * zz)
            if h:
                bld.term((i,), h * sz)
        out[b] = bld.done()
    return out
