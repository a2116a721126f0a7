"""Complex tensors (complex128 and complex64 modes) against the complex128
oracle on identical seeded inputs: amplitudes (including the exact regime
against brute-force enumeration), local energies of the J1-J2 and chiral
Hamiltonians, holomorphic log-derivatives, the Metropolis chains and the
complex minSR step (Hermitian Gram, dtheta = Obar^H (T + eps I)^-1 ebar).

complex128 bar: 1e-10 relative, as for FP64. complex64: 1e-3 relative on
Psi, E_loc and O (FP32 unit roundoff amplified by the cancellation of
random complex tensors, the same bound as the FP32 mode). The 8x8 D=4 chi=16
complex128 case does not fit in LDS and runs the global working-set
variant of every kernel."""
import numpy as np
import pytest

import synth
from oracle import minsr as OM
from oracle import peps, sampler
from tests.gpu_util import logpsi_to_complex, oracle_eval, product_ham, rel_amp_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

J1J2 = ("j1j2", dict(J1=1.0, J2=0.5))
CHIRAL = ("chiral", dict(J1=1.0, J2=0.5, Jchi=0.2))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ctx(Lx, Ly, D, chi, dtype, model=None):
    from paper_2503_12557_amd import Context
    c = Context(Lx, Ly, D, chi, dtype)
    if model is not None:
        c.set_hamiltonian(product_ham(model, Lx, Ly))
    return c


def _to(dev, theta, cf):
    return (torch.from_numpy(np.ascontiguousarray(theta)).to(dev),
            torch.from_numpy(np.ascontiguousarray(cf)).to(dev))


@pytest.mark.parametrize("Lx,Ly,D,chi", [(4, 4, 2, 4), (3, 5, 3, 2), (6, 5, 3, 4), (5, 7, 2, 3),
                                         (8, 8, 4, 16)])
def test_c128_amplitude_matches_oracle(dev, Lx, Ly, D, chi):
    n = 3 if Lx * Ly > 40 else 8
    theta = synth.theta(Lx, Ly, 2, D, seed=200 + Lx + D, cplx=True)
    cf = synth.sz0_configs(Lx * Ly, n, seed=6)
    ctx = _ctx(Lx, Ly, D, chi, "c128")
    th, sm = _to(dev, theta, cf)
    lp, flags = ctx.amplitude(th, sm)
    torch.cuda.synchronize()
    ora, _, _ = oracle_eval(theta, Lx, Ly, D, chi, cf)
    fl = flags.cpu().numpy()
    ok = (fl & 8) == 0
    assert (fl & 7).max() == 0
    err = rel_amp_err(lp.cpu().numpy(), ora)
    assert err[ok].max() <= 1e-10, err


def test_c128_exact_regime_matches_enumeration(dev):
    theta = synth.theta(4, 4, 2, 2, seed=8, cplx=True)
    cf = synth.sz0_configs(16, 32, seed=2)
    ctx = _ctx(4, 4, 2, 4, "c128")
    th, sm = _to(dev, theta, cf)
    lp, _ = ctx.amplitude(th, sm)
    psi = peps.exact_amplitudes(theta, peps.Geometry(4, 4, 2, 2), cf)
    got = np.exp(logpsi_to_complex(lp.cpu().numpy()))
    assert np.abs(got / psi - 1).max() < 1e-10


@pytest.mark.parametrize("Lx,Ly,D,chi,model", [(4, 4, 2, 4, J1J2), (4, 5, 2, 3, CHIRAL),
                                               (5, 4, 3, 4, CHIRAL)])
def test_c128_local_energy_and_logderiv_match_oracle(dev, Lx, Ly, D, chi, model):
    n = 6
    theta = synth.theta(Lx, Ly, 2, D, seed=17 + D, cplx=True)
    cf = synth.sz0_configs(Lx * Ly, n, seed=21)
    ctx = _ctx(Lx, Ly, D, chi, "c128", model)
    th, sm = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    torch.cuda.synchronize()
    ora_lp, ora_e, ora_O = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True)
    ok = (fl.cpu().numpy() & 8) == 0
    got = el.cpu().numpy()
    got = got[:, 0] + 1j * got[:, 1]
    err = np.abs(got - ora_e) / np.maximum(1.0, np.abs(ora_e))
    assert err[ok].max() <= 1e-10, err
    On = O.cpu().numpy()
    scale = np.maximum(1.0, np.abs(ora_O).max(axis=1, keepdims=True))
    assert (np.abs(On - ora_O) / scale)[ok].max() <= 1e-10
    assert rel_amp_err(lp.cpu().numpy(), ora_lp)[ok].max() <= 1e-10


def test_c64_against_oracle(dev):
    Lx, Ly, D, chi = 6, 6, 3, 6
    theta = synth.theta(Lx, Ly, 2, D, seed=22, cplx=True)
    cf = synth.sz0_configs(Lx * Ly, 8, seed=4)
    ctx = _ctx(Lx, Ly, D, chi, "c64", CHIRAL)
    th, sm = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    torch.cuda.synchronize()
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=CHIRAL, want_O=True)
    e = el.cpu().numpy()
    e = e[:, 0] + 1j * e[:, 1]
    e_psi = rel_amp_err(lp.cpu().numpy(), olp).max()
    e_el = (np.abs(e - oel) / np.maximum(1, np.abs(oel))).max()
    On = O.cpu().numpy()
    e_O = (np.abs(On - oO) / np.maximum(1, np.abs(oO).max(1, keepdims=True))).max()
    print("c64 psi %.2e eloc %.2e O %.2e" % (e_psi, e_el, e_O))
    assert max(e_psi, e_el, e_O) < 1e-3


@pytest.mark.parametrize("Lx,Ly,D,chi", [(4, 4, 2, 4), (5, 4, 3, 3)])
def test_c128_chains_identical_to_oracle(dev, Lx, Ly, D, chi):
    theta = synth.theta(Lx, Ly, 2, D, seed=40 + D, cplx=True)
    ctx = _ctx(Lx, Ly, D, chi, "c128")
    th = torch.from_numpy(theta).to(dev)
    sm, acc = ctx.sample(th, "exchange", n_chains=4, per_chain=3, burn_in=2, thin=2, seed=99,
                         offset=1)
    torch.cuda.synchronize()
    g = peps.Geometry(Lx, Ly, 2, D)
    ref, ref_acc = sampler.metropolis(theta, g, chi, "exchange", 4, 3, 2, 2, seed=99, offset=1)
    assert np.array_equal(sm.cpu().numpy(), ref)
    assert np.array_equal(acc.cpu().numpy(), ref_acc)


@pytest.mark.parametrize("dtype,n,eps", [("c128", 150, 1e-4), ("c64", 96, 1e-2)])
def test_complex_minsr_matches_oracle(dev, dtype, n, eps):
    # exact contraction (4x4, D=2, chi=4), chiral Hamiltonian: complex O and
    # complex E_loc; the oracle step uses its own O and E. complex64 O carries
    # FP32 rounding, which the solve amplifies by up to |T| / eps, so that
    # case uses a stronger shift
    Lx, Ly, D, chi = 4, 4, 2, 4
    theta = synth.theta(Lx, Ly, 2, D, seed=3, cplx=True)
    cf = synth.sz0_configs(16, n, seed=7)
    ctx = _ctx(Lx, Ly, D, chi, dtype, CHIRAL)
    th, sm = _to(dev, theta, cf)
    lp, el, O, fl = ctx.evaluate(th, sm)
    dth, diag = ctx.minsr_step(O, sm, el, eps=eps, rcond=1e-12)
    torch.cuda.synchronize()
    g = peps.Geometry(Lx, Ly, 2, D)
    _, ora_e, ora_Oc = oracle_eval(theta, Lx, Ly, D, chi, cf, model=CHIRAL, want_O=True)
    Ofull = np.array([peps.expand_compact(ora_Oc[i], g, cf[i]) for i in range(n)])
    ref, info = OM.minsr_eigh(Ofull, ora_e, eps, 1e-12)
    got = dth.cpu().numpy()
    assert diag.cpu().numpy()[3] == 0.0
    tol = 1e-8 if dtype == "c128" else 1e-3
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"{dtype} minSR relative error {err:.2e}")
    assert err <= tol


def test_complex_vjp_matches_finite_differences(dev):
    # exact contraction (3x3, D=2, chi=4): the autograd gradient of
    # sum_s g_s ln|Psi(S_s)| w.r.t. complex parameters (PyTorch's
    # d/dRe + i d/dIm) against central differences of the oracle's ln|Psi|
    Lx, Ly, D, chi = 3, 3, 2, 4
    theta = synth.theta(Lx, Ly, 2, D, seed=12, cplx=True)
    cf = synth.sz0_configs(Lx * Ly - 1, 6, seed=13)
    cf = np.concatenate([cf, np.zeros((6, 1), dtype=np.uint8)], axis=1)
    g = np.random.default_rng(14).standard_normal(6)
    ctx = _ctx(Lx, Ly, D, chi, "c128")
    th = torch.from_numpy(theta).to(dev).requires_grad_(True)
    sm = torch.from_numpy(cf).to(dev)
    lp = ctx.log_abs_psi(th, sm)
    (lp * torch.from_numpy(g).to(dev)).sum().backward()
    grad = th.grad.cpu().numpy()

    def f(t):
        lpo = oracle_eval(t, Lx, Ly, D, chi, cf)[0]
        return float(np.sum(g * np.real(lpo)))

    rng = np.random.default_rng(15)
    idx = rng.choice(theta.size, 12, replace=False)
    h = 1e-6
    for k in idx:
        for unit in (1.0, 1j):
            tp, tm = theta.copy(), theta.copy()
            tp[k] += h * unit
            tm[k] -= h * unit
            fd = (f(tp) - f(tm)) / (2 * h)
            got = grad[k].real if unit == 1.0 else grad[k].imag
            assert abs(got - fd) <= 1e-6 * max(1.0, abs(fd)), (k, unit, got, fd)