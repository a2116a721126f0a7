"""Oracle local Metropolis sampler with a counter-based random generator.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper needs samples from p(S) = |Psi(S)|^2 / <Psi|Psi> (Eq.
local_estimator) and names Markov-chain samplers as the alternative to its
direct sampler (Sec. "On Direct Sampling"). This is the plain local-update
chain: exchanges of neighbouring anti-aligned spins (conserving S^z) or single
flips, each accepted with probability min(1, |Psi(S')/Psi(S)|^2), where the
ratio is taken inside the strip that holds the move, reusing its
environments (Sec. "On reusing environments").

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), written from its published definition.
Key = (seed mod 2^32, seed >> 32); counters:
  * move decision: (move id, sweep + offset, chain, 0x4d4f5645);
  * initial state:  (site, 0, chain, 0x494e4954).
A uniform double is ((x1 << 32 | x0) >> 11) * 2^-53, and a move is accepted
iff u < |R|^2.

Sweep (exchange): rebuild the bottom environments from the current state;
for each row x from the top: the horizontal bonds (x,y)-(x,y+1) left to right
inside the one-row strip, then (if x < Lx-1) the vertical bonds
(x,y)-(x+1,y) left to right inside the two-row strip of rows x, x+1, then the
row is absorbed into the top environment. Move ids count every bond in that
order, (2*Ly - 1) per row; an aligned pair is not proposed. Sweep (flip):
every site in row-major order inside its one-row strip, move id = site.
Initial state: the floor(N/2) sites with the smallest (key, site) pairs of
the initial-state counters are up (exchange), or each site is up iff the low
bit of x0 is 0 (flip).
"""
from __future__ import annotations

import numpy as np

from . import peps

_M0 = 0xD2511F53
_M1 = 0xCD9E8D57
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF
TAG_MOVE = 0x4D4F5645
TAG_INIT = 0x494E4954


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on one 128-bit counter and a 64-bit key."""
    c0, c1, c2, c3 = [int(v) & _MASK for v in ctr]
    k0, k1 = [int(v) & _MASK for v in key]
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
    return c0, c1, c2, c3


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & _MASK, seed >> 32


def uniform(x0, x1):
    return (((x1 << 32) | x0) >> 11) * (1.0 / 9007199254740992.0)


def initial_state(N, chain, seed, kind):
    key = seed_key(seed)
    if kind == 'exchange':
        keys = [(philox4x32_10((n, 0, chain, TAG_INIT), key)[0], n) for n in range(N)]
        order = sorted(keys)
        s = np.ones(N, dtype=np.uint8)
        for _, n in order[:N // 2]:
            s[n] = 0
        return s
    s = np.zeros(N, dtype=np.uint8)
    for n in range(N):
        s[n] = philox4x32_10((n, 0, chain, TAG_INIT), key)[0] & 1
    return s


def _trivial(Ly, dt):
    return [np.ones((1, 1, 1), dtype=dt) for _ in range(Ly)]


def _sweep(T, g, s, chi, kind, key, chain, sweep_ctr, cutoff=0.0, method='canonical'):
    """One sweep in place on s; returns the number of accepted moves.
    method: the boundary-MPS truncation ('canonical' QR -> SVD or the
    'densmat' density-matrix algorithm), used for every environment."""
    Lx, Ly = g.Lx, g.Ly
    A = peps.project(T, g, s)
    dt = A[(0, 0)].dtype
    B, _ = peps.bottom_environments(A, g, chi, method, cutoff)
    compress = (peps.compress_canonical if method == 'canonical'
                else peps.compress_density_matrix)
    acc = 0
    U = None

    def tens(x, y):
        return T[(x, y)][int(s[x * Ly + y])]

    def decide(move, R):
        x0, x1, _, _ = philox4x32_10((move, sweep_ctr, chain, TAG_MOVE), key)
        return uniform(x0, x1) < abs(R) ** 2

    for x in range(Lx):
        up = U if x > 0 else _trivial(Ly, dt)
        down = B[x + 1] if x < Lx - 1 else _trivial(Ly, dt)
        st = peps.Strip1(up, [tens(x, y) for y in range(Ly)], down)
        L = st.Lf[0]
        if kind == 'exchange':
            for y in range(Ly - 1):
                n1, n2 = x * Ly + y, x * Ly + y + 1
                if s[n1] != s[n2]:
                    cur = [tens(x, y), tens(x, y + 1)]
                    new = [T[(x, y)][int(s[n2])], T[(x, y + 1)][int(s[n1])]]
                    den = _close1(st, L, y, cur)
                    num = _close1(st, L, y, new)
                    if decide(x * (2 * Ly - 1) + y, num / den):
                        s[n1], s[n2] = s[n2], s[n1]
                        acc += 1
                L = st.step_left(L, y, tens(x, y))
            if x < Lx - 1:
                down2 = B[x + 2] if x + 2 < Lx else _trivial(Ly, dt)
                st2 = peps.Strip2(up, [tens(x, y) for y in range(Ly)],
                                  [tens(x + 1, y) for y in range(Ly)], down2)
                L2 = st2.Lf[0]
                for y in range(Ly):
                    n1, n2 = x * Ly + y, (x + 1) * Ly + y
                    if s[n1] != s[n2]:
                        cur = [(tens(x, y), tens(x + 1, y))]
                        new = [(T[(x, y)][int(s[n2])], T[(x + 1, y)][int(s[n1])])]
                        den = _close2(st2, L2, y, cur)
                        num = _close2(st2, L2, y, new)
                        if decide(x * (2 * Ly - 1) + Ly - 1 + y, num / den):
                            s[n1], s[n2] = s[n2], s[n1]
                            acc += 1
                    L2 = st2.step_left(L2, y, tens(x, y), tens(x + 1, y))
        else:
            for y in range(Ly):
                n = x * Ly + y
                cur = [tens(x, y)]
                new = [T[(x, y)][1 - int(s[n])]]
                den = _close1(st, L, y, cur)
                num = _close1(st, L, y, new)
                if decide(n, num / den):
                    s[n] = 1 - s[n]
                    acc += 1
                L = st.step_left(L, y, tens(x, y))
        if x < Lx - 1:
            Acur = peps.project(T, g, s)
            if x == 0:
                U, _ = peps.normalize(peps.top_row_mps(Acur, g, 0))
            else:
                U, _ = peps.normalize(compress(peps.absorb(U, Acur, g, x, True), chi, cutoff))
    return acc


def _close1(st, L, y0, tensors):
    for j, a in enumerate(tensors):
        L = st.step_left(L, y0 + j, a)
    return np.einsum('amc,amc->', L, st.Rt[y0 + len(tensors)])


def _close2(st, L, y0, cols):
    for j, (a1, a2) in enumerate(cols):
        L = st.step_left(L, y0 + j, a1, a2)
    return np.einsum('amnc,amnc->', L, st.Rt[y0 + len(cols)])


def metropolis(theta, g, chi, kind, n_chains, per_chain, burn_in, thin, seed,
               offset=0, cutoff=0.0, method='canonical'):
    """Samples [n_chains * per_chain, N] (chain-major) and accepted counts.
    cutoff: maximal truncated weight of every boundary-MPS truncation
    (``peps.kept_count``), 0 for a fixed chi; method: the truncation
    algorithm ('canonical' or 'densmat').

    Sample j of a chain is the state after sweep burn_in + (j+1)*thin - 1.
    """
    T = peps.site_tensors(theta, g)
    key = seed_key(seed)
    out = np.empty((n_chains * per_chain, g.N), dtype=np.uint8)
    acc = np.zeros(n_chains, dtype=np.int64)
    total = burn_in + per_chain * thin
    for c in range(n_chains):
        s = initial_state(g.N, c, seed, kind)
        j = 0
        for sw in range(total):
            acc[c] += _sweep(T, g, s, chi, kind, key, c, sw + offset, cutoff, method)
            if sw >= burn_in and (sw - burn_in) % thin == thin - 1:
                out[c * per_chain + j] = s
                j += 1
    return out, acc
