"""Pins of the oracle's local energies and log-derivatives (CPU only):
exact diagonalisation / full state vectors at 4x4, closed forms, identities
and finite differences."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import hamiltonian as ham
from oracle import peps


def _config_int(s):
    v = 0
    for b in s:
        v = 2 * v + int(b)
    return v


def _full_state(theta, g, basis):
    confs = np.array([ham.int_to_config(v, g.N) for v in basis])
    return peps.exact_amplitudes(theta, g, confs), confs


@pytest.mark.parametrize("model", ["j1j2", "csl", "rydberg"])
def test_local_energy_equals_H_psi_over_psi_at_4x4(model):
    # exact contraction (chi = 4 >= every Schmidt rank at 4x4, D = 2):
    # E_loc(S) must equal (H Psi)(S) / Psi(S) on the full vector
    Lx, Ly = (4, 4) if model != "rydberg" else (3, 4)
    g = peps.Geometry(Lx, Ly, 2, 2)
    if model == "j1j2":
        H = ham.j1j2(Lx, Ly, 1.0, 0.5)
        th = synth.theta(Lx, Ly, 2, 2, seed=1)
        basis = ham.sz0_basis(16)
    elif model == "csl":
        H = ham.csl(Lx, Ly, 1.0, 0.5, 0.2)
        th = synth.theta(Lx, Ly, 2, 2, seed=4, cplx=True)
        basis = ham.sz0_basis(16)
    else:
        H = ham.rydberg(Lx, Ly, 1.0, 3.0, 1.7 ** 6)
        th = synth.theta(Lx, Ly, 2, 2, seed=5)
        basis = np.arange(2 ** 12)
    psi, confs = _full_state(th, g, basis)
    Hm = ham.sparse_matrix(H, basis)
    Hpsi = Hm @ psi
    T = peps.site_tensors(th, g)
    rng = np.random.default_rng(0)
    for i in rng.choice(len(basis), 6, replace=False):
        sc = peps.SampleContraction(T, g, confs[i], 4)
        e = sc.local_energy(H)
        ref = Hpsi[i] / psi[i]
        assert abs(e - ref) <= 1e-11 * max(1.0, abs(ref))


def test_energy_expectation_is_above_ground_state_at_4x4():
    Lx = Ly = 4
    g = peps.Geometry(Lx, Ly, 2, 2)
    H = ham.j1j2(Lx, Ly, 1.0, 0.0)
    basis = ham.sz0_basis(16)
    th = synth.theta(Lx, Ly, 2, 2, seed=1)
    psi, _ = _full_state(th, g, basis)
    Hm = ham.sparse_matrix(H, basis)
    e_var = float(np.real(np.vdot(psi, Hm @ psi) / np.vdot(psi, psi)))
    e0 = float(spla.eigsh(Hm.real, k=1, which='SA')[0][0])
    # known ground-state energy of the 4x4 open Heisenberg model is about -9.19
    assert -9.3 < e0 < -9.1
    assert e_var >= e0 - 1e-12


@pytest.mark.parametrize("chi", [1, 3])
def test_uniform_amplitude_energy_closed_form(chi):
    # every ratio is exactly 1, so E_loc(S) = sum_t sum_S' <S|h_t|S'> + diag
    Lx, Ly, D = 4, 4, 3
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.uniform_tensor_theta(Lx, Ly, 2, D, seed=2)
    T = peps.site_tensors(th, g)
    for H in (ham.csl(Lx, Ly, 1.0, 0.5, 0.2), ham.rydberg(Lx, Ly, 1.0, 1.0, 24.137569)):
        for s in synth.bit_configs(g.N, 3, seed=4):
            ref = H.diagonal(s)
            for sites, h in H.terms:
                c = 0
                for n in sites:
                    c = 2 * c + int(s[n])
                ref += h[c].sum()
            e = peps.SampleContraction(T, g, s, chi).local_energy(H)
            assert abs(e - ref) < 1e-12 * max(1, abs(ref))


def test_heisenberg_uniform_amplitude_energy_value():
    # with all ratios 1 every Heisenberg bond contributes exactly J/4
    Lx, Ly = 4, 5
    g = peps.Geometry(Lx, Ly, 2, 2)
    th = synth.uniform_tensor_theta(Lx, Ly, 2, 2, seed=3)
    T = peps.site_tensors(th, g)
    H = ham.j1j2(Lx, Ly, 1.0, 0.5)
    n_nn = Lx * (Ly - 1) + (Lx - 1) * Ly
    n_nnn = 2 * (Lx - 1) * (Ly - 1)
    for s in synth.sz0_configs(g.N, 3, seed=1):
        e = peps.SampleContraction(T, g, s, 2).local_energy(H)
        assert abs(e - (n_nn + 0.5 * n_nnn) / 4) < 1e-12


def test_rydberg_long_range_sum_independent_loop():
    Lx, Ly = 5, 4
    H = ham.rydberg(Lx, Ly, 1.0, 3.0, 24.137569)
    for s in synth.bit_configs(Lx * Ly, 5, seed=8):
        ref = 0.0
        for i in range(Lx * Ly):
            ref += -3.0 * s[i]
            for j in range(Lx * Ly):
                if j <= i:
                    continue
                dx = i // Ly - j // Ly
                dy = i % Ly - j % Ly
                ref += 24.137569 / float(dx * dx + dy * dy) ** 3 * s[i] * s[j]
        assert abs(H.diagonal(s) - ref) < 1e-13 * max(1, abs(ref))


def test_chirality_identity_on_a_plaquette():
    # i (P - P^-1) over a plaquette = 2 * (sum of the chiralities of its four
    # triangles), with P the cyclic permutation of the plaquette's spins
    lhs, rhs = ham.chirality_identity_residual()
    # (P maps the state of each site to the next one in the cyclic order)
    assert np.abs(lhs - 2 * rhs).max() < 1e-14
    # the chirality term is Hermitian and purely imaginary
    c = ham.chirality_triple()
    assert np.abs(c - c.conj().T).max() < 1e-15
    assert np.abs(c.real).max() < 1e-15


def test_logderiv_matches_brute_force_hole_tensor():
    # at exact chi, O = (dPsi/dA[x,y]) / Psi with the hole network contracted
    # by one einsum
    for (Lx, Ly, D, chi, cplx) in [(3, 3, 2, 4, False), (4, 4, 2, 4, False), (3, 3, 2, 4, True)]:
        g = peps.Geometry(Lx, Ly, 2, D)
        th = synth.theta(Lx, Ly, 2, D, seed=40 + Lx, cplx=cplx)
        T = peps.site_tensors(th, g)
        s = synth.sz0_configs(g.N, 1, seed=2)[0]
        sc = peps.SampleContraction(T, g, s, chi)
        Oc = sc.logderiv_compact()
        A = peps.project(T, g, s)
        psi = peps.brute_amplitude(A, g)
        for x in range(Lx):
            for y in range(Ly):
                h = peps.brute_amplitude(A, g, skip=(x, y)) / psi
                o = g.compact_offset(x, y)
                got = Oc[o:o + h.size]
                assert np.abs(got - h.ravel()).max() <= 1e-11 * max(1, np.abs(h).max())


@pytest.mark.parametrize("chi", [2, 4])
def test_logderiv_homogeneity_at_truncating_chi(chi):
    # Psi_row(x) is linear in every tensor of row x:
    # sum over a site's active entries of theta_k O_k = 1
    g = peps.Geometry(5, 5, 2, 3)
    th = synth.theta(5, 5, 2, 3, seed=9)
    T = peps.site_tensors(th, g)
    for s in synth.sz0_configs(25, 2, seed=3):
        Oc = peps.SampleContraction(T, g, s, chi).logderiv_compact()
        for x in range(5):
            for y in range(5):
                o = g.compact_offset(x, y)
                b = g.block[(x, y)]
                a = T[(x, y)][int(s[x * 5 + y])].ravel()
                assert abs(np.dot(a, Oc[o:o + b]) - 1) < 1e-12


def test_logderiv_central_finite_differences():
    # O_k = d ln Psi_row(x(k)) / d theta_k; the row amplitude is linear in
    # theta_k, so the central difference is exact up to rounding
    Lx, Ly, D, chi = 5, 4, 3, 4
    g = peps.Geometry(Lx, Ly, 2, D)
    th = synth.theta(Lx, Ly, 2, D, seed=17)
    s = synth.sz0_configs(g.N, 1, seed=5)[0]
    Oc = peps.SampleContraction(peps.site_tensors(th, g), g, s, chi).logderiv_compact()
    O = peps.expand_compact(Oc, g, s)
    rng = np.random.default_rng(3)
    active = np.nonzero(O)[0]
    idx = list(rng.choice(active, 12, replace=False)) + [int(np.nonzero(O == 0)[0][0])]
    h = 1e-6
    for k in idx:
        x = None
        for (xx, yy), off in g.offset.items():
            if off <= k < off + g.d * g.block[(xx, yy)]:
                x = xx
        vals = []
        for sgn in (+1, -1):
            t2 = th.copy()
            t2[k] += sgn * h
            sc = peps.SampleContraction(peps.site_tensors(t2, g), g, s, chi)
            vals.append(sc.strip1(x).value)
        sc0 = peps.SampleContraction(peps.site_tensors(th, g), g, s, chi)
        fd = (vals[0] - vals[1]) / (2 * h) / sc0.strip1(x).value
        assert abs(fd - O[k]) <= 1e-7 * max(1.0, abs(O[k]))


def test_logderiv_product_state_closed_form():
    # rank-one tensors: O at site (x, y) is the outer product of the
    # neighbours' bond vectors divided by phi(s) and the four bond overlaps
    Lx, Ly, D = 3, 4, 2
    g = peps.Geometry(Lx, Ly, 2, D)
    th, fac = synth.product_theta(Lx, Ly, 2, D, seed=12)
    T = peps.site_tensors(th, g)
    s = synth.sz0_configs(g.N, 1, seed=7)[0]
    Oc = peps.SampleContraction(T, g, s, 2).logderiv_compact()
    for x in range(Lx):
        for y in range(Ly):
            phi, vl, vr, vu, vd = fac[(x, y)]
            nl = fac[(x, y - 1)][2] if y > 0 else np.ones(1)
            nr = fac[(x, y + 1)][1] if y < Ly - 1 else np.ones(1)
            nu = fac[(x - 1, y)][4] if x > 0 else np.ones(1)
            nd = fac[(x + 1, y)][3] if x < Lx - 1 else np.ones(1)
            ref = np.einsum('l,r,u,d->lrud', nl, nr, nu, nd)
            ref /= phi[s[x * Ly + y]] * (vl @ nl) * (vr @ nr) * (vu @ nu) * (vd @ nd)
            o = g.compact_offset(x, y)
            assert np.abs(Oc[o:o + ref.size] - ref.ravel()).max() < 1e-12 * np.abs(ref).max()
