"""minSR step (Eqs. tdvp, tdvp_fast) at the full 4x4 D=2 workload size
(1024 samples, 320 parameters) and on a complex multi-tile batch whose size
is not a multiple of the 64-row tiles: the FP64 matrix-core Gram, blocked
Cholesky and blocked triangular solves against the oracle's eigenvalue
solve of the same step."""
import numpy as np
import pytest

import synth
from oracle import minsr as OM
from oracle import peps
from tests.gpu_util import oracle_eval, product_ham

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HEIS = ("j1j2", dict(J1=1.0, J2=0.0))
CHIRAL = ("chiral", dict(J1=1.0, J2=0.5, Jchi=0.2))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_12557_amd import load
    load()
    return torch.device("cuda:0")


def _step(dev, dtype, model, n, seed_t, seed_c, eps, rcond):
    from paper_2503_12557_amd import Context
    Lx, Ly, D, chi = 4, 4, 2, 4
    cplx = dtype.startswith("c")
    theta = synth.theta(Lx, Ly, 2, D, seed=seed_t, cplx=cplx)
    cf = synth.sz0_configs(Lx * Ly, n, seed=seed_c)
    ctx = Context(Lx, Ly, D, chi, dtype)
    ctx.set_hamiltonian(product_ham(model, Lx, Ly))
    th = torch.from_numpy(theta).to(dev)
    sm = torch.from_numpy(cf).to(dev)
    lp, el, O, fl = ctx.evaluate(th, sm)
    dth, diag = ctx.minsr_step(O, sm, el, eps=eps, rcond=rcond)
    torch.cuda.synchronize()
    g = peps.Geometry(Lx, Ly, 2, D)
    _, ora_e, ora_Oc = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True)
    Ofull = np.array([peps.expand_compact(ora_Oc[i], g, cf[i]) for i in range(n)])
    E = ora_e if cplx else ora_e.real
    ref, info = OM.minsr_eigh(Ofull, E, eps, rcond)
    return dth.cpu().numpy(), diag.cpu().numpy(), ref, info


def test_minsr_full_size_real(dev):
    # 1024 samples, rank of the centred O at most 320: T is singular up to
    # eps, the regime the regularisation is for
    got, diag, ref, info = _step(dev, "f64", HEIS, 1024, 1, 5, 1e-4, 1e-12)
    assert diag[3] == 0.0
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"n=1024 real minSR relative error {err:.2e} (lambda_max {info['lam_max']:.3g})")
    assert err <= 1e-8


def test_minsr_complex_ragged_multi_tile(dev):
    # 520 = 8 * 64 + 8 rows: a short last tile and block of the solves
    got, diag, ref, info = _step(dev, "c128", CHIRAL, 520, 3, 9, 1e-4, 1e-12)
    assert diag[3] == 0.0
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"n=520 complex minSR relative error {err:.2e}")
    assert err <= 1e-8
