"""The allocation-free minSR entry point (minsr_step_noalloc) against
minsr_step on the same inputs, through the C-ABI: two calls in a row on one
context, the second with fewer samples (the shared device workspace keeps
the first call's contents), real and complex parameters; both also against
the oracle's eigendecomposition solve (the FP64 bar of the minSR step,
1e-8 relative). Sizes beyond the fixed workspace are rejected, and a
non-finite local energy is reported on the device."""
import numpy as np
import pytest

import synth
from oracle import minsr as OM
from oracle import peps
from tests.gpu_util import product_ham

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_12557_amd import load
    load()
    return torch.device("cuda:0")


def _setup(dev, cplx, n, seed):
    from paper_2503_12557_amd import Context
    Lx, Ly, D, chi = 4, 4, 2, 4
    model = ("chiral", dict(J1=1.0, J2=0.5, Jchi=0.2)) if cplx else ("j1j2", dict(J1=1.0, J2=0.5))
    ctx = Context(Lx, Ly, D, chi, "c128" if cplx else "f64")
    ctx.set_hamiltonian(product_ham(model, Lx, Ly))
    theta = synth.theta(Lx, Ly, 2, D, seed=seed, cplx=cplx)
    cf = synth.sz0_configs(Lx * Ly, n, seed=seed + 1)
    th = torch.from_numpy(theta).to(dev)
    sm = torch.from_numpy(cf).to(dev)
    _, el, O, _ = ctx.evaluate(th, sm)
    torch.cuda.synchronize()
    return ctx, O, sm, el, cf


def _oracle_dtheta(ctx, O, cf, el, cplx):
    g = peps.Geometry(4, 4, 2, 2)
    On = O.cpu().numpy()
    Of = np.array([peps.expand_compact(On[i], g, cf[i]) for i in range(len(cf))])
    e = el.cpu().numpy()
    E = e[:, 0] + 1j * e[:, 1] if cplx else e[:, 0]
    ref, _ = OM.minsr_eigh(Of, E, 1e-4, 1e-12)
    return ref


@pytest.mark.parametrize("cplx", [False, True])
def test_noalloc_equals_minsr_step_two_calls(dev, cplx):
    for n, seed in ((96, 3), (40, 7)):   # second call smaller
        ctx, O, sm, el, cf = _setup(dev, cplx, n, seed)
        d1, g1 = ctx.minsr_step(O, sm, el, eps=1e-4, rcond=1e-12)
        d2, g2 = ctx.minsr_step_noalloc(O, sm, el, eps=1e-4, rcond=1e-12)
        torch.cuda.synchronize()
        a, b = d1.cpu().numpy(), d2.cpu().numpy()
        assert np.isfinite(b).all()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
        assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())
        assert g2[3].item() == 0.0 and g2[6].item() == n
        ref = _oracle_dtheta(ctx, O, cf, el, cplx)
        assert np.abs(b - ref).max() <= 1e-8 * np.abs(ref).max()


def test_noalloc_rejects_oversize_and_flags_nonfinite(dev):
    from paper_2503_12557_amd.binding import PepsError
    ctx, O, sm, el, cf = _setup(dev, False, 64, 11)
    big = 2600   # T alone: 2600^2 x 8 bytes > 48 MiB
    Ob = O.repeat(big // 64 + 1, 1)[:big].contiguous()
    sb = sm.repeat(big // 64 + 1, 1)[:big].contiguous()
    eb = el.repeat(big // 64 + 1, 1)[:big].contiguous()
    with pytest.raises(PepsError) as ex:
        ctx.minsr_step_noalloc(Ob, sb, eb)
    assert "scratch" in str(ex.value)
    bad = el.clone()
    bad[5, 0] = float("nan")
    d, g = ctx.minsr_step_noalloc(O, sm, bad)
    torch.cuda.synchronize()
    assert g[3].item() == 2.0
    assert torch.isnan(d).all()
    # the next call on the shared workspace is clean again
    d, g = ctx.minsr_step_noalloc(O, sm, el)
    torch.cuda.synchronize()
    assert g[3].item() == 0.0 and torch.isfinite(d).all()
