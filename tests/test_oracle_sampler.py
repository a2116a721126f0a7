"""Pins of the oracle sampler (CPU only): Philox known-answer vectors,
conservation of S^z, and chi-square tests of long-chain histograms against
|Psi|^2 on lattices small enough to enumerate."""
import itertools

import numpy as np
import pytest
from scipy import stats

import synth
from oracle import peps, sampler


def test_philox4x32_10_known_answers():
    # known-answer vectors published with the Random123 library
    assert sampler.philox4x32_10((0, 0, 0, 0), (0, 0)) == (
        0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert sampler.philox4x32_10((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2) == (
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert sampler.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344),
                                 (0xA4093822, 0x299F31D0)) == (
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_uniform_range_and_mean():
    key = sampler.seed_key(123)
    u = [sampler.uniform(*sampler.philox4x32_10((i, 0, 0, 0), key)[:2]) for i in range(4000)]
    assert min(u) >= 0.0 and max(u) < 1.0
    assert abs(np.mean(u) - 0.5) < 0.02


def _chi2_pvalue(samples, probs, index):
    counts = np.zeros(len(probs))
    for s in samples:
        counts[index[tuple(int(v) for v in s)]] += 1
    exp = probs * len(samples)
    keep = exp > 5
    # merge the small bins into one
    c = np.append(counts[keep], counts[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        c, e = c[:-1], e[:-1]
    return stats.chisquare(c, e).pvalue


@pytest.mark.slow
def test_exchange_chain_histogram_matches_psi_squared():
    Lx, Ly, D, chi = 2, 3, 2, 4
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=3)
    confs = [np.array(c, dtype=np.uint8) for c in itertools.product([0, 1], repeat=6)
             if sum(c) == 3]
    psi = peps.exact_amplitudes(th, g, np.array(confs))
    p = np.abs(psi) ** 2
    p /= p.sum()
    index = {tuple(int(v) for v in c): i for i, c in enumerate(confs)}
    samples, acc = sampler.metropolis(th, g, chi, 'exchange', 4, 400, 10, 2, seed=7)
    for s in samples:
        assert int(s.sum()) == 3
    assert acc.sum() > 0
    assert _chi2_pvalue(samples, p, index) > 1e-3


@pytest.mark.slow
def test_flip_chain_histogram_matches_psi_squared():
    Lx, Ly, D, chi = 2, 2, 2, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=4)
    confs = [np.array(c, dtype=np.uint8) for c in itertools.product([0, 1], repeat=4)]
    psi = peps.exact_amplitudes(th, g, np.array(confs))
    p = np.abs(psi) ** 2
    p /= p.sum()
    index = {tuple(int(v) for v in c): i for i, c in enumerate(confs)}
    samples, _ = sampler.metropolis(th, g, chi, 'flip', 4, 500, 10, 1, seed=9)
    assert _chi2_pvalue(samples, p, index) > 1e-3


def test_initial_states():
    for c in range(5):
        s = sampler.initial_state(16, c, 42, 'exchange')
        assert int((s == 0).sum()) == 8
    a = sampler.initial_state(16, 0, 42, 'exchange')
    b = sampler.initial_state(16, 1, 42, 'exchange')
    assert not np.array_equal(a, b)
