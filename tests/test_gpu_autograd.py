"""The hand-written adjoint behind torch.autograd.Function: exact-regime
gradient against finite differences of the forward value, and at the 8x8
D=4 chi=16 shape the library's O against central finite differences
(h = 1e-6, FP64) of the oracle's strip amplitude on 20 random active
parameters plus one inactive one."""
import numpy as np
import pytest

import synth
from oracle import peps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_autograd_matches_finite_differences_exact_regime(dev):
    from paper_2503_12557_amd import Context
    Lx, Ly, D, chi, n = 4, 4, 2, 4, 16
    theta = synth.theta(Lx, Ly, 2, D, seed=6)
    cf = synth.sz0_configs(16, n, seed=1)
    ctx = Context(Lx, Ly, D, chi, "f64")
    th = torch.from_numpy(theta).to(dev).requires_grad_(True)
    sm = torch.from_numpy(cf).to(dev)
    c = torch.linspace(0.5, 1.5, n, dtype=torch.float64, device=dev)
    f = (c * ctx.log_abs_psi(th, sm)).sum()
    (g,) = torch.autograd.grad(f, th)
    g = g.cpu().numpy()
    rng = np.random.default_rng(0)
    h = 1e-6
    for k in rng.choice(len(theta), 20, replace=False):
        vals = []
        for sgn in (1, -1):
            t2 = theta.copy()
            t2[k] += sgn * h
            lp, _ = ctx.amplitude(torch.from_numpy(t2).to(dev), sm)
            vals.append((c * lp[:, 0]).sum().item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k]))


def test_logderiv_against_oracle_finite_differences_8x8(dev):
    from paper_2503_12557_amd import Context
    Lx, Ly, D, chi = 8, 8, 4, 16
    g8 = peps.Geometry(Lx, Ly, 2, D)
    theta = synth.theta(Lx, Ly, 2, D, seed=2)
    cf = synth.sz0_configs(64, 8, seed=3)
    ctx = Context(Lx, Ly, D, chi, "f64")
    O = ctx.logderiv(torch.from_numpy(theta).to(dev), torch.from_numpy(cf).to(dev)).cpu().numpy()
    rng = np.random.default_rng(7)
    h = 1e-6
    picks = [(int(rng.integers(8)), None) for _ in range(20)] + [(0, "inactive")]
    for (i, kind) in picks:
        s = cf[i]
        full = peps.expand_compact(O[i], g8, s)
        if kind is None:
            k = int(rng.choice(np.nonzero(full)[0]))
        else:
            k = int(np.nonzero(full == 0)[0][0])
        x = [xx for (xx, yy), off in g8.offset.items()
             if off <= k < off + 2 * g8.block[(xx, yy)]][0]
        vals = []
        for sgn in (1, -1):
            t2 = theta.copy()
            t2[k] += sgn * h
            sc = peps.SampleContraction(peps.site_tensors(t2, g8), g8, s, chi)
            vals.append(sc.strip1(x).value)
        base = peps.SampleContraction(peps.site_tensors(theta, g8), g8, s, chi).strip1(x).value
        fd = (vals[0] - vals[1]) / (2 * h) / base
        assert abs(fd - full[k]) <= 1e-6 * max(1.0, abs(full[k])), (k, fd, full[k])
