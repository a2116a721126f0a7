"""Boundary-MPS truncation by a maximal truncated weight (Sec. "On the
boundary MPS method": D_c chosen dynamically; App. on the variational upper
bound for the cutoff study). Pins: the kept-count rule on spectra whose
answer is known by hand; one bond of a two-site MPS, where the canonical
truncation must equal the best rank-r approximation of the dense matrix
(Eckart-Young) with r fixed by the discarded weight of numpy's SVD; a zero
cutoff is the fixed-chi contraction bit for bit; a cutoff of 1 keeps one
state per bond; and the contraction error falls as the cutoff is tightened."""
import numpy as np

import synth
from oracle import peps


def test_kept_count_on_hand_spectra():
    sv = np.sqrt(np.array([0.5, 0.3, 0.15, 0.04, 0.01]))   # weights sum to 1
    assert peps.kept_count(sv, 5, 0.0) == 5
    assert peps.kept_count(sv, 3, 0.0) == 3
    assert peps.kept_count(sv, 5, 0.011) == 4     # drop 0.01
    assert peps.kept_count(sv, 5, 0.051) == 3     # drop 0.04 + 0.01
    assert peps.kept_count(sv, 5, 0.049) == 4
    assert peps.kept_count(sv, 5, 0.2) == 3       # 0.2 < 0.15 + 0.05
    assert peps.kept_count(sv, 5, 0.21) == 2
    assert peps.kept_count(sv, 5, 0.99) == 1
    assert peps.kept_count(sv, 2, 0.011) == 2     # chi caps the count
    assert peps.kept_count(sv, 5, 1e-9) == 5


def test_one_bond_is_the_best_rank_r_approximation():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((1, 6, 5))
    b = rng.standard_normal((5, 7, 1))
    M = np.einsum('akb,bjc->kj', a, b)       # dense 6 x 7 state
    s = np.linalg.svd(M, compute_uv=False)
    w = s ** 2 / (s ** 2).sum()
    for cutoff in (1e-3, 3e-2, 0.2):
        tail = np.array([w[r:].sum() for r in range(len(w) + 1)])
        r = int(min(k for k in range(1, len(w) + 1) if tail[k] <= cutoff))
        out = peps.compress_canonical([a, b], 5, cutoff)
        assert out[1].shape[0] == r
        Mt = np.einsum('akb,bjc->kj', out[0], out[1])
        U, S, Vh = np.linalg.svd(M)
        best = (U[:, :r] * S[:r]) @ Vh[:r]
        assert np.abs(Mt - best).max() < 1e-12 * np.abs(M).max()


def test_zero_cutoff_is_fixed_chi_and_full_cutoff_keeps_one_state():
    Lx, Ly, D, chi = 5, 4, 3, 4
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=12)
    cf = synth.sz0_configs(Lx * Ly, 3, seed=2)
    a, _, _ = peps.evaluate(th, g, cf, chi)
    b, _, _ = peps.evaluate(th, g, cf, chi, cutoff=0.0)
    assert np.array_equal(a, b)
    A = peps.project(peps.site_tensors(th, g), g, cf[0])
    U, _ = peps.top_environments(A, g, chi, 'canonical', 1.0)
    for x in range(1, Lx - 1):
        assert all(t.shape[0] == 1 and t.shape[2] == 1 for t in U[x])


def test_error_falls_with_the_cutoff():
    # 6 x 6, D = 3: the reference keeps chi = 27 with no cutoff (chi = 40
    # gives the same amplitudes); tighter cutoffs approach it
    Lx, Ly, D = 6, 6, 3
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=5, mu=0.5)
    cf = synth.sz0_configs(Lx * Ly, 4, seed=3)
    ref, _, _ = peps.evaluate(th, g, cf, 27)
    errs = []
    for cut in (1e-2, 1e-4, 1e-6, 1e-9, 1e-12):
        lp, _, _ = peps.evaluate(th, g, cf, 27, cutoff=cut)
        errs.append(np.abs(np.exp(lp - ref) - 1).max())
    assert errs[0] > 0.1 and errs[-1] < 1e-5
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs


def test_density_matrix_cutoff_equals_canonical():
    # the density-matrix truncation applies the same kept-count rule to the
    # square roots of its eigenvalues: with a cutoff it must keep the same
    # states as the canonical sweep (same bond dimensions, same amplitudes)
    cases = [(4, 4, 2, 4, 5, 0.0, 1e-3), (5, 4, 3, 6, 7, 0.5, 1e-2), (4, 5, 3, 5, 9, 0.0, 1e-2)]
    for Lx, Ly, D, chi, seed, mu, cut in cases:
        g = peps.Geometry(Lx, Ly, 2, D)
        th = synth.theta(Lx, Ly, 2, D, seed=seed, mu=mu)
        cf = synth.sz0_configs(Lx * Ly, 3, seed=seed + 1)
        a, _, _ = peps.evaluate(th, g, cf, chi, cutoff=cut)
        b, _, _ = peps.evaluate(th, g, cf, chi, method='densmat', cutoff=cut)
        c, _, _ = peps.evaluate(th, g, cf, chi)
        assert np.abs(np.exp(a - b) - 1).max() < 1e-10
        assert np.abs(np.exp(a - c) - 1).max() > 1e-6   # the cutoff changes the result
        A = peps.project(peps.site_tensors(th, g), g, cf[0])
        U1, _ = peps.top_environments(A, g, chi, 'canonical', cut)
        U2, _ = peps.top_environments(A, g, chi, 'densmat', cut)
        for x in range(1, Lx - 1):
            assert [t.shape for t in U1[x]] == [t.shape for t in U2[x]]
