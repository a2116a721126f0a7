"""Oracle direct sampler of PEPS configurations (Sec. "On Direct Sampling";
App. "Direct sampling of PEPS", Eq. prob_from_cond_prob and the row-by-row
sampling algorithm there).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

p(S) = prod_i p(S_i | S_<i) over rows i from the top. The conditional
density matrix of row i is T^u_{S<i}[i] . D^l[i+1] . (T^u_{S<i}[i])^*:
  * T^u_{S<i}[i]: the top boundary MPS E^u[i-1] of the already sampled rows
    (single layer, bond chi, the same E^u as the amplitude contraction)
    times the tensors of row i with their physical legs open;
  * D^l[i+1]: the boundary MPS of the double-layer network of rows
    i+1..Lx-1 (every site tensor sum_p T[p] x conj(T[p]), bond D^2), from
    the bottom with bond chi_d, computed once per tensor set.
Row i is then sampled like an MPS, site by site from the left: with the left
environment Lc of the sites already fixed and the right environment R of the
remaining sites (their physical legs traced), q_p = Lc . col(p) . R and
p(s_y = p | ...) = q_p / (q_0 + q_1). After the row is fixed, E^u[i] absorbs
it and is truncated to chi.

Readings taken here:
  * D_s (the bond of T^u_{S<i}[i]) is not truncated: T^u keeps bond chi*D,
    so the conditionals are exact given E^u and D^l;
  * a negative q_p (possible once chi_d truncates) counts as 0; if both are
    0 the site is drawn with probability 1/2 each;
  * random numbers: Philox4x32-10 (``sampler.philox4x32_10``) with key from
    the seed and counter (site, j mod 2^32, j >> 32, 0x44495243) for sample
    j = offset + index; s = 0 iff u < q_0 / (q_0 + q_1).
"""
from __future__ import annotations

import math

import numpy as np

from . import peps
from .sampler import philox4x32_10, seed_key, uniform

TAG_DIRECT = 0x44495243


def double_layer(T, g: peps.Geometry):
    """Site tensors of the double-layer network: legs (l l', r r', u u', d d')
    fused ket-major, sum_p T[p] x conj(T[p])."""
    out = {}
    for x in range(g.Lx):
        for y in range(g.Ly):
            t = T[(x, y)]
            _, Dl, Dr, Du, Dd = t.shape
            m = np.einsum('plrud,pLRUD->lLrRuUdD', t, t.conj())
            out[(x, y)] = m.reshape(Dl * Dl, Dr * Dr, Du * Du, Dd * Dd)
    return out


def double_bottom_environments(T, g: peps.Geometry, chi_d: int):
    """D^l[x] for x = Lx-1..1: boundary MPS of the double layer from the
    bottom, truncated to chi_d (canonical truncation, as for E^l)."""
    B, _ = peps.bottom_environments(double_layer(T, g), g, chi_d)
    return B


def _unit(t):
    m = np.abs(t).max()
    return t / m if m > 0 else t


def _right_step(E, Tp, G, R1):
    """One column, physical value p, absorbed into the right environment:
    R[e,l,b,m,h] = E[e,u,f] Tp[l,r,u,d] G[b,d,w,g] conj(Tp)[m,s,v,w]
    conj(E)[h,v,k] R1[f,r,g,s,k], contracted one tensor at a time."""
    t = np.einsum('euf,frgsk->eurgsk', E, R1, optimize=True)
    t = np.einsum('lrud,eurgsk->eldgsk', Tp, t, optimize=True)
    t = np.einsum('bdwg,eldgsk->elbwsk', G, t, optimize=True)
    t = np.einsum('msvw,elbwsk->elbmvk', Tp.conj(), t, optimize=True)
    return np.einsum('hvk,elbmvk->elbmh', E.conj(), t, optimize=True)


def _left_step(Lc, E, Tp, G):
    """The same column absorbed into the left environment:
    C[f,r,g,s,k] = Lc[e,l,b,m,h] E[e,u,f] Tp[l,r,u,d] G[b,d,w,g]
    conj(Tp)[m,s,v,w] conj(E)[h,v,k]."""
    t = np.einsum('elbmh,euf->lbmhuf', Lc, E, optimize=True)
    t = np.einsum('lbmhuf,lrud->bmhfrd', t, Tp, optimize=True)
    t = np.einsum('bmhfrd,bdwg->mhfrgw', t, G, optimize=True)
    t = np.einsum('mhfrgw,msvw->hfrgsv', t, Tp.conj(), optimize=True)
    return np.einsum('hfrgsv,hvk->frgsk', t, E.conj(), optimize=True)


def _walk(T, g, chi, Dl_env, uniforms=None, fixed=None):
    """One configuration row by row. With ``uniforms`` the sites are drawn;
    with ``fixed`` they are forced. Returns (s, ln p(s))."""
    Lx, Ly = g.Lx, g.Ly
    s = np.zeros(Lx * Ly, dtype=np.uint8)
    logp = 0.0
    U = None
    dt = np.result_type(T[(0, 0)], np.float64)
    one3 = np.ones((1, 1, 1), dtype=dt)
    for i in range(Lx):
        Es = [one3] * Ly if i == 0 else U
        if i + 1 <= Lx - 1:
            Ds = [d.reshape(d.shape[0], int(round(math.sqrt(d.shape[1]))),
                            int(round(math.sqrt(d.shape[1]))), d.shape[2])
                  for d in Dl_env[i + 1]]
        else:
            Ds = [np.ones((1, 1, 1, 1), dtype=dt)] * Ly
        Ts = [T[(i, y)] for y in range(Ly)]
        # right environments: physical legs of sites y.. traced
        R = [None] * (Ly + 1)
        R[Ly] = np.ones((1, 1, 1, 1, 1), dtype=dt)
        for y in range(Ly - 1, -1, -1):
            acc = 0
            for p in range(2):
                acc = acc + _right_step(Es[y], Ts[y][p], Ds[y], R[y + 1])
            R[y] = _unit(acc)
        Lc = np.ones((1, 1, 1, 1, 1), dtype=dt)
        for y in range(Ly):
            n = i * Ly + y
            cand, q = [], []
            for p in range(2):
                c = _left_step(Lc, Es[y], Ts[y][p], Ds[y])
                cand.append(c)
                q.append(max(0.0, float(np.real(np.sum(c * R[y + 1])))))
            tot = q[0] + q[1]
            p0 = q[0] / tot if tot > 0 else 0.5
            if fixed is not None:
                b = int(fixed[n])
            else:
                b = 0 if uniforms[n] < p0 else 1
            pb = p0 if b == 0 else 1.0 - p0
            logp += math.log(pb) if pb > 0 else -math.inf
            s[n] = b
            Lc = _unit(cand[b])
        if i <= Lx - 2:
            A = peps.project(T, g, s)
            if i == 0:
                U, _ = peps.normalize(peps.top_row_mps(A, g, 0))
            else:
                U, _ = peps.normalize(peps.compress_canonical(peps.absorb(U, A, g, i, True), chi))
    return s, logp


def sample(theta, g: peps.Geometry, chi: int, chi_d: int, n: int, seed: int, offset: int = 0,
           theta_double=None):
    """n independent configurations and ln p(S) of each. theta_double: the
    tensors D^l is built from, when they are older than theta (the stale
    double-layer environments of the paper's asynchronous scheme; p stays
    the sampler's own, so the importance weights remain exact)."""
    T = peps.site_tensors(theta, g)
    T2 = T if theta_double is None else peps.site_tensors(theta_double, g)
    Dl_env = double_bottom_environments(T2, g, chi_d)
    key = seed_key(seed)
    out = np.zeros((n, g.N), dtype=np.uint8)
    logp = np.zeros(n)
    for j in range(n):
        jj = offset + j
        u = np.empty(g.N)
        for site in range(g.N):
            r = philox4x32_10((site, jj & 0xFFFFFFFF, jj >> 32, TAG_DIRECT), key)
            u[site] = uniform(r[0], r[1])
        out[j], logp[j] = _walk(T, g, chi, Dl_env, uniforms=u)
    return out, logp


def log_prob(theta, g: peps.Geometry, chi: int, chi_d: int, configs, theta_double=None):
    """ln p(S) of given configurations under the direct sampler."""
    T = peps.site_tensors(theta, g)
    T2 = T if theta_double is None else peps.site_tensors(theta_double, g)
    Dl_env = double_bottom_environments(T2, g, chi_d)
    return np.array([_walk(T, g, chi, Dl_env, fixed=np.asarray(s))[1] for s in configs])
