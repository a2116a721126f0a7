"""The oracle direct sampler (App. "Direct sampling of PEPS"). Pins: in the
exact regime (chi and chi_d large enough that no truncation happens) p(S) is
|Psi(S)|^2 / <Psi|Psi> from enumeration of the exact state; at truncating
chi_d the conditionals still give a normalised p (sum over all 2^N
configurations is 1) that differs from |Psi|^2; drawn samples carry the
ln p of their own walk; their histogram passes a chi-square test against p."""
import itertools

import numpy as np
from scipy import stats

import synth
from oracle import direct, peps


def _all_configs(N):
    return np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.uint8)


def test_exact_regime_gives_psi_squared():
    Lx, Ly, D = 3, 3, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=7)
    cf = _all_configs(9)
    psi = peps.exact_amplitudes(th, g, cf)
    p_exact = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    lp = direct.log_prob(th, g, 4, 16, cf)
    assert np.abs(np.exp(lp) - p_exact).max() < 1e-12 * p_exact.max() * 10


def test_exact_regime_complex():
    Lx, Ly, D = 2, 3, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=8, cplx=True)
    cf = _all_configs(6)
    psi = peps.exact_amplitudes(th, g, cf)
    p_exact = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    lp = direct.log_prob(th, g, 4, 4, cf)
    assert np.abs(np.exp(lp) / p_exact - 1).max() < 1e-10


def test_truncated_double_layer_is_normalised_but_not_exact():
    Lx, Ly, D = 3, 3, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=3)
    cf = _all_configs(9)
    p = np.exp(direct.log_prob(th, g, 4, 2, cf))
    assert abs(p.sum() - 1) < 1e-12
    psi = peps.exact_amplitudes(th, g, cf)
    p_exact = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    assert np.abs(p - p_exact).max() > 1e-4


def test_drawn_samples_carry_their_walk_probability():
    Lx, Ly, D = 3, 4, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=5)
    s, lp = direct.sample(th, g, 3, 3, 6, seed=11, offset=2)
    assert np.allclose(lp, direct.log_prob(th, g, 3, 3, s), rtol=0, atol=1e-12)
    # other offsets give other draws
    s2, _ = direct.sample(th, g, 3, 3, 6, seed=11, offset=8)
    assert not np.array_equal(s, s2)


def test_histogram_matches_the_sampler_distribution():
    Lx, Ly, D = 2, 3, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=2)
    n = 1500
    s, _ = direct.sample(th, g, 4, 4, n, seed=21)
    cf = _all_configs(6)
    p = np.exp(direct.log_prob(th, g, 4, 4, cf))
    idx = {tuple(int(v) for v in c): k for k, c in enumerate(cf)}
    counts = np.zeros(len(cf))
    for row in s:
        counts[idx[tuple(int(v) for v in row)]] += 1
    exp = p * n
    keep = exp > 5
    c = np.append(counts[keep], counts[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        c, e = c[:-1], e[:-1]
    assert stats.chisquare(c, e).pvalue > 1e-3


def test_stale_double_layer_keeps_p_normalised():
    # D^l from older tensors (the asynchronous scheme): p is still a
    # normalised distribution, now away from |Psi|^2 even at exact chi_d
    Lx, Ly, D = 3, 3, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=7)
    old = synth.theta(Lx, Ly, 2, D, seed=70)
    cf = _all_configs(9)
    p = np.exp(direct.log_prob(th, g, 4, 16, cf, theta_double=old))
    assert abs(p.sum() - 1) < 1e-12
    psi = peps.exact_amplitudes(th, g, cf)
    assert np.abs(p - np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)).max() > 1e-4
