"""FP32 and BF16 modes against the FP64 oracle on identical inputs.

FP32: random sign-indefinite tensors; the bound 1e-3 on the relative error
of Psi, E_loc and O covers the FP32 unit roundoff (6e-8) amplified by the
cancellation inside the contraction of uniformly drawn configurations.
BF16 (every contraction operand rounded to bfloat16, 8 mantissa bits):
measured on rank-one positive tensors, where nothing cancels and the error
stays at the level of a few bfloat16 roundings per row; on random tensors
the error is printed, not bounded. With identical physical slices every
amplitude is the same number in any precision, so ratios are exactly 1."""
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
    assert all(np.isfinite(e))
