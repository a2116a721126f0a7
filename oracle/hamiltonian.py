"""Oracle Hamiltonians, built from explicit Pauli Kronecker products.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Basis: for spins s = 0 is up (S^z = +1/2) and s = 1 is down; for Rydberg
atoms s = 0 is |g> and s = 1 is |r> (n = s). A k-site term is a 2^k x 2^k
matrix h[c, c'] = <c|h|c'> with the first listed site as the most
significant bit of the local index c.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128) / 2
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128) / 2
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128) / 2
I2 = np.eye(2, dtype=np.complex128)
PAULI_X = 2 * SX
NUM = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def kron(*ms):
    out = np.ones((1, 1), dtype=np.complex128)
    for m in ms:
        out = np.kron(out, m)
    return out


def heisenberg_pair():
    """S_i . S_j on two sites."""
    return kron(SX, SX) + kron(SY, SY) + kron(SZ, SZ)


def chirality_triple():
    """S_i . (S_j x S_k) on three sites (Levi-Civita sum written out)."""
    return (kron(SX, SY, SZ) - kron(SX, SZ, SY)
            + kron(SY, SZ, SX) - kron(SY, SX, SZ)
            + kron(SZ, SX, SY) - kron(SZ, SY, SX))


def cyclic_permutation(k):
    """P moving the state of site j to site j+1 (mod k) on k spin-1/2 sites."""
    dim = 2 ** k
    P = np.zeros((dim, dim), dtype=np.complex128)
    for c in range(dim):
        bits = [(c >> (k - 1 - j)) & 1 for j in range(k)]
        nb = [bits[(j - 1) % k] for j in range(k)]
        c2 = 0
        for b in nb:
            c2 = 2 * c2 + b
        P[c2, c] = 1.0
    return P


class Hamiltonian:
    """A list of few-site terms (sites, h) plus diagonal long-range pairs
    sum V_ij n_i n_j and an on-site diagonal table onsite[n, s]."""

    def __init__(self, N):
        self.N = N
        self.terms = []
        self.pairs = []
        self.onsite = np.zeros((N, 2), dtype=np.complex128)

    def add(self, sites, h):
        self.terms.append((tuple(int(n) for n in sites), np.asarray(h, dtype=np.complex128)))

    def diagonal(self, s):
        e = 0.0 + 0.0j
        for (i, j, v) in self.pairs:
            if s[i] == 1 and s[j] == 1:
                e += v
        for n in range(self.N):
            e += self.onsite[n, int(s[n])]
        return e


def nn_bonds(Lx, Ly):
    out = []
    for x in range(Lx):
        for y in range(Ly):
            n = x * Ly + y
            if y + 1 < Ly:
                out.append((n, n + 1))
            if x + 1 < Lx:
                out.append((n, n + Ly))
    return out


def nnn_bonds(Lx, Ly):
    out = []
    for x in range(Lx - 1):
        for y in range(Ly - 1):
            n = x * Ly + y
            out.append((n, n + Ly + 1))
            out.append((n + 1, n + Ly))
    return out


def plaquette_triangles(Lx, Ly):
    """The four triangles of each plaquette a=(x,y), b=(x,y+1), c=(x+1,y+1),
    e=(x+1,y), taken in the cyclic order a->b->c->e."""
    out = []
    for x in range(Lx - 1):
        for y in range(Ly - 1):
            a = x * Ly + y
            b = a + 1
            c = a + Ly + 1
            e = a + Ly
            out += [(a, b, c), (b, c, e), (c, e, a), (e, a, b)]
    return out


def j1j2(Lx, Ly, J1=1.0, J2=0.0):
    """J1 sum_<ij> S_i.S_j + J2 sum_<<ij>> S_i.S_j (Sec. "J1-J2 model")."""
    H = Hamiltonian(Lx * Ly)
    h = heisenberg_pair()
    for (i, j) in nn_bonds(Lx, Ly):
        H.add((i, j), J1 * h)
    if J2 != 0.0:
        for (i, j) in nnn_bonds(Lx, Ly):
            H.add((i, j), J2 * h)
    return H


def csl(Lx, Ly, J1=1.0, J2=0.5, Jchi=0.2):
    """J1-J2 Heisenberg plus J_chi on the four triangles of every plaquette
    of S_i.(S_j x S_k). The paper's ring term i*lam*(P - P^-1) on a plaquette
    equals 2*lam times that four-triangle sum (Sec. "Chiral spin liquid")."""
    H = j1j2(Lx, Ly, J1, J2)
    c = chirality_triple()
    for tri in plaquette_triangles(Lx, Ly):
        H.add(tri, Jchi * c)
    return H


def rydberg(Lx, Ly, Omega=1.0, Delta=1.0, V=1.7 ** 6):
    """Omega/2 sum sigma^x - Delta sum n + sum_{i<j} V/r_ij^6 n_i n_j
    (Sec. "Rydberg atom arrays"), r in lattice units, V = (R_b/a)^6."""
    N = Lx * Ly
    H = Hamiltonian(N)
    for n in range(N):
        H.add((n,), 0.5 * Omega * PAULI_X)
        H.onsite[n, 1] += -Delta
    for i in range(N):
        for j in range(i + 1, N):
            xi, yi = divmod(i, Ly)
            xj, yj = divmod(j, Ly)
            r2 = (xi - xj) ** 2 + (yi - yj) ** 2
            H.pairs.append((i, j, V / r2 ** 3))
    return H


def sparse_matrix(H: Hamiltonian, basis=None):
    """<S|H|S'> on the full 2^N basis (or a list of basis states closed
    under H), indices with site 0 as the most significant bit."""
    N = H.N
    if basis is None:
        states = np.arange(2 ** N, dtype=np.int64)
    else:
        states = np.asarray(basis, dtype=np.int64)
    index = {int(v): i for i, v in enumerate(states)}
    rows, cols, vals = [], [], []
    bits = ((states[:, None] >> (N - 1 - np.arange(N))[None, :]) & 1).astype(np.int64)
    diag = np.zeros(len(states), dtype=np.complex128)
    for (i, j, v) in H.pairs:
        diag += v * (bits[:, i] & bits[:, j])
    for n in range(N):
        diag += H.onsite[n, bits[:, n]]
    for sites, h in H.terms:
        k = len(sites)
        c = np.zeros(len(states), dtype=np.int64)
        for n in sites:
            c = 2 * c + bits[:, n]
        for c2 in range(2 ** k):
            col = h[c, c2]
            nz = np.nonzero(col)[0]
            if len(nz) == 0:
                continue
            tgt = states.copy()
            for j, n in enumerate(sites):
                b = (c2 >> (k - 1 - j)) & 1
                tgt = (tgt & ~(1 << (N - 1 - n))) | (b << (N - 1 - n))
            for r in nz:
                t = int(tgt[r])
                if t not in index:
                    raise ValueError('basis not closed under H')
                rows.append(r)
                cols.append(index[t])
                vals.append(col[r])
    m = sp.coo_matrix((vals, (rows, cols)), shape=(len(states), len(states))).tocsr()
    return m + sp.diags(diag)


def sz0_basis(N):
    """All N-spin configurations with floor(N/2) up spins (s = 0), as integers."""
    out = [v for v in range(2 ** N) if bin(v).count('1') == N - N // 2]
    return np.array(out, dtype=np.int64)


def int_to_config(v, N):
    return np.array([(int(v) >> (N - 1 - n)) & 1 for n in range(N)], dtype=np.uint8)


def chirality_identity_residual():
    """|| i(P_4 - P_4^-1) - 2 sum_tri chi || on one plaquette (a, b, c, e)
    ordered cyclically; zero when the two forms of the CSL term agree."""
    P = cyclic_permutation(4)
    lhs = 1j * (P - P.conj().T)
    # sites 0..3 = a, b, c, e in cyclic order
    chi = chirality_triple()
    rhs = np.zeros((16, 16), dtype=np.complex128)
    for tri in [(0, 1, 2), (1, 2, 3), (2, 3, 0), (3, 0, 1)]:
        rhs += embed(chi, tri, 4)
    return lhs, rhs


def embed(h, sites, N):
    """Embed a k-site operator acting on ``sites`` into N sites."""
    k = len(sites)
    dim = 2 ** N
    out = np.zeros((dim, dim), dtype=np.complex128)
    for s in range(dim):
        bits = [(s >> (N - 1 - n)) & 1 for n in range(N)]
        c = 0
        for n in sites:
            c = 2 * c + bits[n]
        for c2 in range(2 ** k):
            v = h[c, c2]
            if v == 0:
                continue
            b2 = list(bits)
            for j, n in enumerate(sites):
                b2[n] = (c2 >> (k - 1 - j)) & 1
            t = 0
            for b in b2:
                t = 2 * t + b
            out[s, t] += v
    return out


def csl_paper_constants():
    """J1, J2, lambda of the paper's chiral spin liquid point."""
    return (2 * math.cos(0.06 * math.pi) * math.cos(0.14 * math.pi),
            2 * math.cos(0.06 * math.pi) * math.sin(0.14 * math.pi),
            2 * math.sin(0.06 * math.pi))
