"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself: it only draws random
PEPS parameters and random spin configurations from numpy's PCG64 generator,
so that the CPU oracle and the GPU library can be fed identical inputs.

Parameter layout (used by both sides, defined here only as the order in
which random numbers are drawn): sites in row-major order n = x*Ly + y, and
inside a site the C-order tensor (p, l, r, u, d) with physical index p first,
then the left, right, up and down virtual legs. Virtual legs on an open edge
have dimension 1.
"""
from __future__ import annotations

import numpy as np


def site_leg_dims(Lx: int, Ly: int, D: int, x: int, y: int):
    """(Dl, Dr, Du, Dd) of site (x, y) on an open Lx x Ly lattice."""
    return (1 if y == 0 else D, 1 if y == Ly - 1 else D,
            1 if x == 0 else D, 1 if x == Lx - 1 else D)


def num_params(Lx: int, Ly: int, d: int, D: int) -> int:
    n = 0
    for x in range(Lx):
        for y in range(Ly):
            a, b, c, e = site_leg_dims(Lx, Ly, D, x, y)
            n += d * a * b * c * e
    return n


def theta(Lx: int, Ly: int, d: int, D: int, seed: int, mu: float = 0.0,
          cplx: bool = False) -> np.ndarray:
    """Random PEPS parameters: i.i.d. N(mu, 1) (real) or N(0,1)+i N(0,1).

    For complex tensors all real parts are drawn first, then all imaginary
    parts.
    """
    rng = np.random.default_rng(seed)
    n = num_params(Lx, Ly, d, D)
    if cplx:
        re = rng.standard_normal(n)
        im = rng.standard_normal(n)
        return re + 1j * im
    return mu + rng.standard_normal(n)


def sz0_configs(N: int, n: int, seed: int) -> np.ndarray:
    """n uniformly random configurations of N spins with floor(N/2) up spins.

    Value 0 is spin up, 1 is spin down. Returns uint8 [n, N].
    """
    rng = np.random.default_rng(seed)
    base = np.zeros(N, dtype=np.uint8)
    base[N // 2:] = 1
    if N % 2:
        base[N // 2] = 1
    out = np.empty((n, N), dtype=np.uint8)
    for i in range(n):
        out[i] = rng.permutation(base)
    return out


def bit_configs(N: int, n: int, seed: int, p1: float = 0.5) -> np.ndarray:
    """n configurations of N independent bits, P(bit = 1) = p1. uint8 [n, N]."""
    rng = np.random.default_rng(seed)
    return (rng.random((n, N)) < p1).astype(np.uint8)


def uniform_tensor_theta(Lx: int, Ly: int, d: int, D: int, seed: int) -> np.ndarray:
    """Parameters whose physical slices are identical on every site.

    T[x,y][p] = A[x,y] for all p: the amplitude is the same for every
    configuration (detached physical legs), at any contraction bond.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for x in range(Lx):
        for y in range(Ly):
            dims = site_leg_dims(Lx, Ly, D, x, y)
            a = rng.standard_normal(int(np.prod(dims)))
            parts.append(np.tile(a, d))
    return np.concatenate(parts)


def product_theta(Lx: int, Ly: int, d: int, D: int, seed: int):
    """Rank-one site tensors T = phi (x) a (x) b (x) c (x) e with positive legs.

    Returns (theta, factors) where factors[(x, y)] = (phi, l, r, u, dn) are
    the vectors the tensor is the outer product of.
    """
    rng = np.random.default_rng(seed)
    parts = []
    factors = {}
    for x in range(Lx):
        for y in range(Ly):
            Dl, Dr, Du, Dd = site_leg_dims(Lx, Ly, D, x, y)
            phi = rng.standard_normal(d)
            vl = 0.5 + rng.random(Dl)
            vr = 0.5 + rng.random(Dr)
            vu = 0.5 + rng.random(Du)
            vd = 0.5 + rng.random(Dd)
            t = np.einsum('p,l,r,u,d->plrud', phi, vl, vr, vu, vd)
            parts.append(t.ravel())
            factors[(x, y)] = (phi, vl, vr, vu, vd)
    return np.concatenate(parts), factors
