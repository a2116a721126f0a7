"""Parity of the HIP library (through the C-ABI) with the FP64 CPU oracle on
identical seeded inputs. FP64 bar: 1e-10 relative on Psi, E_loc, O and the
minSR step."""
import numpy as np
import pytest

import synth
from oracle import minsr as OM
from oracle import peps
from tests.gpu_util import (configs_for, logpsi_to_complex, oracle_eval, product_ham,
                            rel_amp_err)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_12557_amd import load
    load()
    return torch.device("cuda:0")


def _ctx(Lx, Ly, D, chi, dtype="f64", model=None):
    from paper_2503_12557_amd import Context
    c = Context(Lx, Ly, D, chi, dtype)
    if model is not None:
        c.set_hamiltonian(product_ham(model, Lx, Ly))
    return c


def _to(dev, theta, cf):
    return (torch.from_numpy(np.ascontiguousarray(theta)).to(dev),
            torch.from_numpy(np.ascontiguousarray(cf)).to(dev))


J1J2 = ("j1j2", dict(J1=1.0, J2=0.5))
CHIRAL = ("chiral", dict(J1=1.0, J2=0.5, Jchi=0.2))
RYD = ("rydberg", dict(Omega=1.0, Delta=3.0, V=1.7 ** 6))

# (Lx, Ly, D, chi): exact regime, truncating, ragged (Lx != Ly, chi not a
# power of two), and the 8x8 D=4 chi=16 shape
AMP_CASES = [(4, 4, 2, 4), (2, 3, 2, 2), (3, 5, 3, 2), (6, 5, 3, 4), (5, 7, 2, 3), (8, 8, 4, 16)]


@pytest.mark.parametrize("Lx,Ly,D,chi", AMP_CASES)
def test_amplitude_matches_oracle(dev, Lx, Ly, D, chi):
    n = 6 if Lx * Ly > 40 else 12
    theta = synth.theta(Lx, Ly, 2, D, seed=100 + Lx + Ly + D)
    cf = synth.sz0_configs(Lx * Ly, n, seed=5)
    ctx = _ctx(Lx, Ly, D, chi)
    th, sm = _to(dev, theta, cf)
    lp, flags = ctx.amplitude(th, sm)
    torch.cuda.synchronize()
    ora, _, _ = oracle_eval(theta, Lx, Ly, D, chi, cf)
    fl = flags.cpu().numpy()
    ok = (fl & 8) == 0
    assert (fl & 7).max() == 0
    err = rel_amp_err(lp.cpu().numpy(), ora)
    assert err[ok].max() <= 1e-10, err


def test_amplitude_exact_regime_matches_brute_force(dev):
    Lx = Ly = 4
    theta = synth.theta(4, 4, 2, 2, seed=1)
    cf = synth.sz0_configs(16, 64, seed=2)
    ctx = _ctx(4, 4, 2, 4)
    th, sm = _to(dev, theta, cf)
    lp, _ = ctx.amplitude(th, sm)
    psi = peps.exact_amplitudes(theta, peps.Geometry(4, 4, 2, 2), cf)
    got = np.exp(logpsi_to_complex(lp.cpu().numpy()))
    assert np.abs(got / psi - 1).max() < 1e-10


@pytest.mark.parametrize("Lx,Ly,D,chi,model", [
    (4, 4, 2, 4, J1J2), (5, 4, 3, 4, J1J2), (4, 5, 2, 3, CHIRAL), (4, 4, 2, 4, RYD),
    (3, 6, 3, 5, RYD)])
def test_local_energy_matches_oracle(dev, Lx, Ly, D, chi, model):
    n = 8
    theta = synth.theta(Lx, Ly, 2, D, seed=7 + D)
    cf = configs_for(model, Lx * Ly, n, seed=11)
    ctx = _ctx(Lx, Ly, D, chi, model=model)
    th, sm = _to(dev, theta, cf)
    env = ctx.new_env_cache(n)
    lp, flags = ctx.amplitude(th, sm, env_cache=env)
    el = ctx.local_energy(th, sm, env_cache=env)
    el_fresh = ctx.local_energy(th, sm)
    torch.cuda.synchronize()
    ora_lp, ora_e, _ = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model)
    got = el.cpu().numpy()
    got = got[:, 0] + 1j * got[:, 1]
    ok = (flags.cpu().numpy() & 8) == 0
    err = np.abs(got - ora_e) / np.maximum(1.0, np.abs(ora_e))
    assert err[ok].max() <= 1e-10, err
    assert torch.equal(el, el_fresh)


@pytest.mark.parametrize("Lx,Ly,D,chi", [(4, 4, 2, 4), (5, 4, 3, 4), (6, 6, 2, 3)])
def test_logderiv_matches_oracle(dev, Lx, Ly, D, chi):
    n = 6
    theta = synth.theta(Lx, Ly, 2, D, seed=3 + Lx)
    cf = synth.sz0_configs(Lx * Ly, n, seed=12)
    ctx = _ctx(Lx, Ly, D, chi)
    th, sm = _to(dev, theta, cf)
    O = ctx.logderiv(th, sm).cpu().numpy()
    _, _, ora_O = oracle_eval(theta, Lx, Ly, D, chi, cf, want_O=True)
    scale = np.maximum(1.0, np.abs(ora_O).max(axis=1, keepdims=True))
    assert (np.abs(O - ora_O) / scale).max() <= 1e-10


def test_evaluate_fused_equals_separate_calls(dev):
    Lx, Ly, D, chi = 5, 5, 3, 4
    theta = synth.theta(Lx, Ly, 2, D, seed=9)
    cf = synth.sz0_configs(Lx * Ly, 10, seed=13)
    ctx = _ctx(Lx, Ly, D, chi, model=J1J2)
    th, sm = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    env = ctx.new_env_cache(10)
    lp2, _ = ctx.amplitude(th, sm, env_cache=env)
    el2 = ctx.local_energy(th, sm, env_cache=env)
    O2 = ctx.logderiv(th, sm, env_cache=env)
    assert torch.equal(lp, lp2)
    assert torch.equal(el, el2)
    assert torch.equal(O, O2)


def test_minsr_step_matches_oracle(dev):
    # 4x4 D=2 chi=4 (exact contraction), eps = 1e-4, rcond = 1e-12
    Lx, Ly, D, chi = 4, 4, 2, 4
    n = 192
    theta = synth.theta(Lx, Ly, 2, D, seed=1)
    cf = synth.sz0_configs(16, n, seed=3)
    ctx = _ctx(Lx, Ly, D, chi, model=("j1j2", dict(J1=1.0, J2=0.0)))
    th, sm = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    dth, diag = ctx.minsr_step(O, sm, el, eps=1e-4, rcond=1e-12)
    torch.cuda.synchronize()
    g = peps.Geometry(Lx, Ly, 2, D)
    _, ora_e, ora_Oc = oracle_eval(theta, Lx, Ly, D, chi, cf, model=("j1j2", dict(J1=1.0, J2=0.0)),
                                   want_O=True)
    Ofull = np.array([peps.expand_compact(ora_Oc[i], g, cf[i]) for i in range(n)])
    ref, info = OM.minsr_eigh(Ofull, ora_e.real, 1e-4, 1e-12)
    got = dth.cpu().numpy()
    assert diag.cpu().numpy()[3] == 0.0
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_minsr_step_ragged_batch(dev):
    # n not a multiple of the 64-row tiles, truncating contraction
    Lx, Ly, D, chi = 5, 4, 3, 4
    n = 150
    theta = synth.theta(Lx, Ly, 2, D, seed=4)
    cf = synth.sz0_configs(Lx * Ly, n, seed=8)
    ctx = _ctx(Lx, Ly, D, chi, model=J1J2)
    th, sm = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    dth, diag = ctx.minsr_step(O, sm, el, eps=1e-3, rcond=1e-12)
    # the oracle step on the library's own O would not be independent, so
    # compare against the oracle's O and E computed from the same inputs
    g = peps.Geometry(Lx, Ly, 2, D)
    _, ora_e, ora_Oc = oracle_eval(theta, Lx, Ly, D, chi, cf, model=J1J2, want_O=True)
    Ofull = np.array([peps.expand_compact(ora_Oc[i], g, cf[i]) for i in range(n)])
    ref = OM.minsr_cholesky(Ofull, ora_e.real, 1e-3)
    got = dth.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_uniform_amplitude_gives_closed_form_energy(dev):
    Lx, Ly, D, chi = 5, 6, 3, 4
    theta = synth.uniform_tensor_theta(Lx, Ly, 2, D, seed=2)
    cf = synth.sz0_configs(Lx * Ly, 8, seed=3)
    ctx = _ctx(Lx, Ly, D, chi, model=J1J2)
    th, sm = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    lpn = lp.cpu().numpy()
    assert np.abs(lpn - lpn[0]).max() < 1e-10
    n_nn = Lx * (Ly - 1) + (Lx - 1) * Ly
    n_nnn = 2 * (Lx - 1) * (Ly - 1)
    e = el.cpu().numpy()
    assert np.abs(e[:, 0] - (n_nn + 0.5 * n_nnn) / 4).max() < 1e-10
    assert np.abs(e[:, 1]).max() == 0.0


def test_nonfinite_theta_is_flagged_without_a_host_check(dev):
    # the evaluation calls do not synchronise: a non-finite parameter shows
    # up as the non-finite flag of every sample
    Lx, Ly, D, chi = 3, 4, 2, 4
    theta = synth.theta(Lx, Ly, 2, D, seed=9)
    theta[7] = np.nan
    cf = synth.sz0_configs(Lx * Ly, 5, seed=3)
    ctx = _ctx(Lx, Ly, D, chi, "f64", J1J2)
    th, sm = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    torch.cuda.synchronize()
    assert ((fl.cpu().numpy() & 2) != 0).all()
    theta[7] = 0.5
    th, _ = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    torch.cuda.synchronize()
    assert (fl.cpu().numpy() & 2).max() == 0
