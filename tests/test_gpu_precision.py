"""FP32, complex64 and BF16 modes against the FP64 oracle on identical inputs.

FP32: random sign-indefinite tensors; the bound 1e-3 on the relative error
of Psi, E_loc and O covers the FP32 unit roundoff (6e-8) amplified by the
cancellation inside the contraction of uniformly drawn configurations.
BF16 (every contraction operand rounded to bfloat16, 8 mantissa bits, FP32
accumulation): on rank-one positive tensors nothing cancels and the error
stays at a few bfloat16 roundings per row (bound 5e-2). On random tensors
the bfloat16 roundings are amplified by the same cancellation as FP32's,
2^16 times larger: the bounds below are stated from measurement with about
a factor of three of margin, and show that BF16 operands are not accurate
enough for sign-indefinite tensors (Psi off by O(1) at 12x12), while tensors
of mean 0.5 keep Psi within about 0.1. The minSR direction dtheta (FP64
solve) is compared, through the whole path, with the oracle's. With
identical physical slices every amplitude is the same number in any
precision, so ratios are exactly 1."""
import numpy as np
import pytest

import synth
from tests.gpu_util import oracle_eval, product_ham, rel_amp_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

J1J2 = ("j1j2", dict(J1=1.0, J2=0.5))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _run(dev, dtype, theta, Lx, Ly, D, chi, cf):
    from paper_2503_12557_amd import Context
    ctx = Context(Lx, Ly, D, chi, dtype)
    ctx.set_hamiltonian(product_ham(J1J2, Lx, Ly))
    lp, el, O, fl = ctx.evaluate(torch.from_numpy(theta).to(dev), torch.from_numpy(cf).to(dev))
    torch.cuda.synchronize()
    e = el.cpu().numpy()
    return lp.cpu().numpy(), e[:, 0] + 1j * e[:, 1], O.cpu().numpy()


def _errs(dev, dtype, theta, Lx, Ly, D, chi, cf):
    lp, el, O = _run(dev, dtype, theta, Lx, Ly, D, chi, cf)
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=J1J2, want_O=True)
    e_psi = rel_amp_err(lp, olp).max()
    e_el = (np.abs(el - oel) / np.maximum(1, np.abs(oel))).max()
    e_O = (np.abs(O - oO) / np.maximum(1, np.abs(oO).max(1, keepdims=True))).max()
    return e_psi, e_el, e_O


def test_fp32_random_tensors(dev):
    Lx, Ly, D, chi = 6, 6, 3, 6
    theta = synth.theta(Lx, Ly, 2, D, seed=21, mu=0.5)
    cf = synth.sz0_configs(Lx * Ly, 8, seed=4)
    e = _errs(dev, "f32", theta, Lx, Ly, D, chi, cf)
    print("f32 psi %.2e eloc %.2e O %.2e" % e)
    assert max(e) < 1e-3


def test_bf16_rank_one_tensors(dev):
    Lx, Ly, D, chi = 6, 6, 3, 4
    theta, _ = synth.product_theta(Lx, Ly, 2, D, seed=5)
    cf = synth.sz0_configs(Lx * Ly, 8, seed=4)
    e = _errs(dev, "bf16", theta, Lx, Ly, D, chi, cf)
    print("bf16 rank-one psi %.2e eloc %.2e O %.2e" % e)
    assert max(e) < 5e-2


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_uniform_amplitude_ratios_exact(dev, dtype):
    Lx, Ly, D, chi = 5, 6, 3, 4
    theta = synth.uniform_tensor_theta(Lx, Ly, 2, D, seed=2)
    cf = synth.sz0_configs(Lx * Ly, 8, seed=3)
    lp, el, O = _run(dev, dtype, theta, Lx, Ly, D, chi, cf)
    n_nn = Lx * (Ly - 1) + (Lx - 1) * Ly
    n_nnn = 2 * (Lx - 1) * (Ly - 1)
    assert np.abs(lp - lp[0]).max() == 0.0
    assert np.abs(el - (n_nn + 0.5 * n_nnn) / 4).max() < 1e-12


def test_bf16_random_tensors_reported(dev):
    Lx, Ly, D, chi = 6, 6, 3, 6
    theta = synth.theta(Lx, Ly, 2, D, seed=21, mu=0.5)
    cf = synth.sz0_configs(Lx * Ly, 8, seed=4)
    e = _errs(dev, "bf16", theta, Lx, Ly, D, chi, cf)
    print("bf16 random psi %.2e eloc %.2e O %.2e" % e)
    # measured 1.5, 0.36, 0.38
    assert e[0] < 5.0 and e[1] < 1.0 and e[2] < 1.0


# ---------------------------------------------------------------------------
# Reduced precision through the whole path to the minSR direction: Psi,
# E_loc and O from the reduced-precision contractions, then the FP64 minSR
# solve, against the oracle's FP64 (complex128) path and eigendecomposition
# solve on the same configurations.
# ---------------------------------------------------------------------------
def _dtheta_err(dev, dtype, theta, Lx, Ly, D, chi, cf, model, cplx):
    from oracle import minsr as OM
    from oracle import peps
    from paper_2503_12557_amd import Context
    ctx = Context(Lx, Ly, D, chi, dtype)
    ctx.set_hamiltonian(product_ham(model, Lx, Ly))
    th = torch.from_numpy(theta).to(dev)
    sm = torch.from_numpy(cf).to(dev)
    lp, el, O, fl = ctx.evaluate(th, sm)
    dth, diag = ctx.minsr_step(O, sm, el, eps=1e-4, rcond=1e-12)
    torch.cuda.synchronize()
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True)
    g = peps.Geometry(Lx, Ly, 2, D)
    Of = np.array([peps.expand_compact(oO[i], g, cf[i]) for i in range(len(cf))])
    ref, _ = OM.minsr_eigh(Of, oel if cplx else oel.real, 1e-4, 1e-12)
    got = dth.cpu().numpy()
    e = el.cpu().numpy()
    return (np.abs(got - ref).max() / np.abs(ref).max(),
            np.linalg.norm(got - ref) / np.linalg.norm(ref),
            rel_amp_err(lp.cpu().numpy(), olp).max(),
            (np.abs(e[:, 0] + 1j * e[:, 1] - oel) / np.maximum(1, np.abs(oel))).max(),
            diag.cpu().numpy()[3])


# measured (relative 2-norm of dtheta): 2.7e-4, 3.2e-6, 5.5e-6
@pytest.mark.parametrize("dtype,shape,mu,bound", [
    ("f32", (8, 8, 4, 16), 0.0, 2e-3), ("f32", (8, 8, 4, 16), 0.5, 5e-5),
    ("c64", (6, 6, 3, 6), 0.0, 1e-4)])
def test_dtheta_error_reduced_precision(dev, dtype, shape, mu, bound):
    Lx, Ly, D, chi = shape
    cplx = dtype == "c64"
    model = ("chiral", dict(J1=1.0, J2=0.5, Jchi=0.2)) if cplx else J1J2
    theta = synth.theta(Lx, Ly, 2, D, seed=71, mu=mu, cplx=cplx)
    cf = synth.sz0_configs(Lx * Ly, 40, seed=72)
    e_max, e_2, e_psi, e_el, cert = _dtheta_err(dev, dtype, theta, Lx, Ly, D, chi, cf, model, cplx)
    print(f"{dtype} {shape} mu={mu}: dtheta max-rel {e_max:.2e} 2-norm-rel {e_2:.2e} "
          f"(psi {e_psi:.2e}, E_loc {e_el:.2e})")
    assert cert == 0.0
    assert e_2 <= bound


# bounds (psi, E_loc, O, dtheta); measured 1.14 / 0.19 / 28 / 0.80 with
# N(0,1) tensors and 0.12 / 0.040 / 0.22 / 0.019 with N(0.5,1)
@pytest.mark.parametrize("mu,bound", [(0.0, (5.0, 1.0, 100.0, 2.0)),
                                      (0.5, (0.4, 0.15, 1.0, 0.06))])
def test_bf16_12x12_rydberg_bounded(dev, mu, bound):
    # BF16 operands with FP32 accumulation on the 12x12 D=4 chi=16 Rydberg
    # array against the FP64 oracle on 8 configurations (single-flip sector:
    # independent bits), with bounds on Psi, E_loc, O and dtheta
    from oracle import minsr as OM
    from oracle import peps
    from paper_2503_12557_amd import Context
    Lx, Ly, D, chi = 12, 12, 4, 16
    RYD = ("rydberg", dict(Omega=1.0, Delta=3.0, V=1.7 ** 6))
    theta = synth.theta(Lx, Ly, 2, D, seed=81, mu=mu)
    cf = synth.bit_configs(Lx * Ly, 8, seed=82)
    ctx = Context(Lx, Ly, D, chi, "bf16")
    ctx.set_hamiltonian(product_ham(RYD, Lx, Ly))
    th = torch.from_numpy(theta).to(dev)
    sm = torch.from_numpy(cf).to(dev)
    lp, el, O, fl = ctx.evaluate(th, sm)
    dth, diag = ctx.minsr_step(O, sm, el, eps=1e-4, rcond=1e-12)
    torch.cuda.synchronize()
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=RYD, want_O=True)
    e = el.cpu().numpy()
    e_psi = rel_amp_err(lp.cpu().numpy(), olp)
    e_el = np.abs(e[:, 0] - oel.real) / np.maximum(1, np.abs(oel))
    On = O.cpu().numpy()
    e_O = np.abs(On - oO).max(1) / np.maximum(1, np.abs(oO).max(1))
    g = peps.Geometry(Lx, Ly, 2, D)
    Of = np.array([peps.expand_compact(oO[i], g, cf[i]) for i in range(len(cf))])
    ref, _ = OM.minsr_eigh(Of, oel.real, 1e-4, 1e-12)
    got = dth.cpu().numpy()
    e_dth = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"bf16 12x12 mu={mu}: psi max {e_psi.max():.2e} median {np.median(e_psi):.2e}; "
          f"E_loc max {e_el.max():.2e} median {np.median(e_el):.2e}; O max {e_O.max():.2e}; "
          f"dtheta {e_dth:.2e}")
    assert e_psi.max() < bound[0] and e_el.max() < bound[1]
    assert e_O.max() < bound[2] and e_dth < bound[3]
