"""Pins of the oracle's amplitude and boundary-MPS code against brute force,
closed forms and invariants (CPU only)."""
import math

import numpy as np
import pytest

import synth
from oracle import peps


def _cases():
    # (Lx, Ly, D, chi) with chi at or above the exact Schmidt rank of every
    # boundary MPS: a row-x cut of an Ly-wide strip has rank <= D^min(y, Ly-y)
    return [(2, 2, 2, 1), (2, 3, 3, 1), (3, 3, 2, 4), (3, 2, 3, 3),
            (4, 4, 2, 4), (3, 4, 2, 4), (4, 3, 3, 9)]


@pytest.mark.parametrize("Lx,Ly,D,chi", _cases())
def test_boundary_mps_exact_regime_matches_brute_force(Lx, Ly, D, chi):
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=11 + Lx * 7 + Ly + D)
    T = peps.site_tensors(th, g)
    for s in synth.sz0_configs(g.N, 4, seed=3):
        A = peps.project(T, g, s)
        ref = peps.brute_amplitude(A, g)
        sc = peps.SampleContraction(T, g, s, chi)
        assert abs(np.exp(sc.logpsi) - ref) <= 1e-12 * max(1.0, abs(ref))
        # E^u[i] . E^l[i+1] is the same number for every cut i
        for i in range(Lx - 1):
            v = np.exp(peps.log_amplitude_at(sc.U, sc.fU, sc.B, sc.fB, i))
            assert abs(v - ref) <= 1e-12 * max(1.0, abs(ref))


def test_complex_tensors_exact_regime():
    g = peps.Geometry(3, 3, 2, 2)
    th = synth.theta(3, 3, 2, 2, seed=5, cplx=True)
    T = peps.site_tensors(th, g)
    for s in synth.sz0_configs(9, 4, seed=4):
        ref = peps.brute_amplitude(peps.project(T, g, s), g)
        sc = peps.SampleContraction(T, g, s, 4)
        assert abs(np.exp(sc.logpsi) - ref) <= 1e-12 * abs(ref)


def test_strip_amplitudes_equal_psi_in_exact_regime():
    g = peps.Geometry(4, 4, 2, 2)
    th = synth.theta(4, 4, 2, 2, seed=1)
    T = peps.site_tensors(th, g)
    for s in synth.sz0_configs(16, 3, seed=9):
        sc = peps.SampleContraction(T, g, s, 4)
        ref = np.exp(sc.logpsi)
        for x in range(4):
            st = sc.strip1(x)
            scale = (sc.fU[x - 1] if x > 0 else 0.0) + (sc.fB[x + 1] if x < 3 else 0.0)
            assert abs(st.value * math.exp(scale) - ref) <= 1e-12 * abs(ref)
        for x in range(3):
            st = sc.strip2(x)
            scale = (sc.fU[x - 1] if x > 0 else 0.0) + (sc.fB[x + 2] if x + 2 < 4 else 0.0)
            assert abs(st.value * math.exp(scale) - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("chi", [2, 3, 5])
def test_canonical_and_density_matrix_truncation_agree(chi):
    # the two truncation algorithms give the same truncated state
    g = peps.Geometry(5, 5, 2, 3)
    th = synth.theta(5, 5, 2, 3, seed=21)
    T = peps.site_tensors(th, g)
    for s in synth.sz0_configs(25, 3, seed=2):
        a = peps.SampleContraction(T, g, s, chi, 'canonical').logpsi
        b = peps.SampleContraction(T, g, s, chi, 'densmat').logpsi
        assert abs(np.exp(a - b) - 1) < 1e-9


@pytest.mark.parametrize("chi", [1, 2, 3])
def test_product_state_closed_form_at_any_chi(chi):
    # rank-one positive-leg tensors: the network factorises into one phi per
    # site times one scalar product per bond, for any contraction bond
    Lx, Ly, D = 4, 5, 3
    g = peps.Geometry(Lx, Ly, 2, D)
    th, fac = synth.product_theta(Lx, Ly, 2, D, seed=8)
    T = peps.site_tensors(th, g)
    for s in synth.sz0_configs(g.N, 3, seed=1):
        ref = 1.0
        for x in range(Lx):
            for y in range(Ly):
                phi, vl, vr, vu, vd = fac[(x, y)]
                ref *= phi[s[x * Ly + y]]
                # open legs have dimension 1 and contribute their one entry
                for v in (vl, vr, vu, vd):
                    if v.size == 1:
                        ref *= float(v[0])
                if y + 1 < Ly:
                    ref *= float(vr @ fac[(x, y + 1)][1])
                if x + 1 < Lx:
                    ref *= float(vd @ fac[(x + 1, y)][3])
        sc = peps.SampleContraction(T, g, s, chi)
        assert abs(np.exp(sc.logpsi) - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("chi", [1, 2, 4])
def test_uniform_amplitude_construction(chi):
    # identical physical slices: every configuration has the same amplitude
    g = peps.Geometry(4, 4, 2, 3)
    th = synth.uniform_tensor_theta(4, 4, 2, 3, seed=3)
    T = peps.site_tensors(th, g)
    vals = [peps.SampleContraction(T, g, s, chi).logpsi
            for s in synth.bit_configs(16, 4, seed=5)]
    assert max(abs(v - vals[0]) for v in vals) < 1e-12


def test_horizontal_gauge_invariance_at_truncating_chi():
    # M M^-1 on a horizontal bond leaves every boundary-MPS state vector,
    # hence its truncation and the amplitude, unchanged
    Lx, Ly, D, chi = 5, 4, 3, 3
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=31)
    T = peps.site_tensors(th, g)
    rng = np.random.default_rng(0)
    T2 = {k: v.copy() for k, v in T.items()}
    for x in range(Lx):
        for y in range(Ly - 1):
            M = rng.standard_normal((D, D)) + 3 * np.eye(D)
            T2[(x, y)] = np.einsum('plrud,rs->plsud', T2[(x, y)], M)
            T2[(x, y + 1)] = np.einsum('sl,plrud->psrud', np.linalg.inv(M), T2[(x, y + 1)])
    for s in synth.sz0_configs(g.N, 3, seed=6):
        a = peps.SampleContraction(T, g, s, chi).logpsi
        b = peps.SampleContraction(T2, g, s, chi).logpsi
        assert abs(np.exp(a - b) - 1) < 1e-9


def test_vertical_gauge_invariance_in_exact_regime():
    Lx, Ly, D, chi = 4, 4, 2, 4
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=32)
    T = peps.site_tensors(th, g)
    rng = np.random.default_rng(1)
    T2 = {k: v.copy() for k, v in T.items()}
    for x in range(Lx - 1):
        for y in range(Ly):
            M = rng.standard_normal((D, D)) + 3 * np.eye(D)
            T2[(x, y)] = np.einsum('plrud,ds->plrus', T2[(x, y)], M)
            T2[(x + 1, y)] = np.einsum('su,plrud->plrsd', np.linalg.inv(M), T2[(x + 1, y)])
    for s in synth.sz0_configs(g.N, 3, seed=6):
        a = peps.SampleContraction(T, g, s, chi).logpsi
        b = peps.SampleContraction(T2, g, s, chi).logpsi
        assert abs(np.exp(a - b) - 1) < 1e-11


def test_truncation_error_vanishes_at_exact_chi():
    # relative contraction error |Psi(chi) - Psi(chi_max)| / |Psi(chi_max)|
    g = peps.Geometry(4, 5, 2, 2)
    th = synth.theta(4, 5, 2, 2, seed=12)
    T = peps.site_tensors(th, g)
    s = synth.sz0_configs(20, 1, seed=1)[0]
    ref = np.exp(peps.SampleContraction(T, g, s, 16).logpsi)
    brute = peps.brute_amplitude(peps.project(T, g, s), g)
    assert abs(ref - brute) < 1e-12 * abs(brute)
    errs = [abs(np.exp(peps.SampleContraction(T, g, s, c).logpsi) - ref) / abs(ref)
            for c in (1, 2, 4, 8)]
    assert errs[-1] < 1e-12
    assert errs[0] > 1e-6


def test_parameter_count():
    # 4x4, d=2, D=2 open lattice: 4 corners of d*D^2, 8 edges of d*D^3, 4 bulk d*D^4
    assert peps.Geometry(4, 4, 2, 2).n_params == 4 * 8 + 8 * 16 + 4 * 32 == 288
    assert synth.num_params(8, 8, 2, 4) == peps.Geometry(8, 8, 2, 4).n_params == 21632
    assert peps.Geometry(10, 10, 2, 5).n_params == 88200
