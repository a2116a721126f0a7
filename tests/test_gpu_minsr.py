"""minSR step (Eqs. tdvp, tdvp_fast) at the full 4x4 D=2 workload size
(1024 samples, 320 parameters) and on a complex multi-tile batch whose size
is not a multiple of the 64-row tiles: the FP64 matrix-core Gram, blocked
Cholesky and blocked triangular solves, and the eigendecomposition solve
(alone, and as the fallback of a failed certificate), each against the
oracle's eigenvalue solve of the same step."""
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
_CACHE = {}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_12557_amd import load
    load()
    return torch.device("cuda:0")


def _case(dev, dtype, model, n, seed_t, seed_c):
    """Library O and E_loc on the device and the oracle's O (expanded) and E
    for the same seeded 4x4 D=2 chi=4 inputs, computed once per case."""
    key = (dtype, model[0], n, seed_t, seed_c)
    if key in _CACHE:
        return _CACHE[key]
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
    torch.cuda.synchronize()
    g = peps.Geometry(Lx, Ly, 2, D)
    _, ora_e, ora_Oc = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True)
    Ofull = np.array([peps.expand_compact(ora_Oc[i], g, cf[i]) for i in range(n)])
    E = ora_e if cplx else ora_e.real
    _CACHE[key] = (ctx, sm, el, O, Ofull, E)
    return _CACHE[key]


def _run(case, solver, eps, rcond):
    ctx, sm, el, O, Ofull, E = case
    ctx.set_minsr_solver(solver)
    dth, diag = ctx.minsr_step(O, sm, el, eps=eps, rcond=rcond)
    torch.cuda.synchronize()
    ctx.set_minsr_solver("cholesky")
    return dth.cpu().numpy(), diag.cpu().numpy()


def _err(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


def _spectrum(Ofull, E, eps):
    Ob, _ = OM.centre(Ofull, E)
    return np.linalg.eigvalsh(OM.gram(Ob) + eps * np.eye(Ob.shape[0]))


def _gap_rcond(w):
    """rcond at the geometric middle of the widest gap of the spectrum w
    (ascending), so that which eigenvalues are dropped is not decided by
    rounding."""
    ratio = w[1:] / np.maximum(w[:-1], 1e-300)
    i = int(np.argmax(ratio))
    return np.sqrt(w[i] * w[i + 1]) / w[-1], i + 1


def test_minsr_full_size_real(dev):
    # 1024 samples, rank of the centred O at most 320: T is singular up to
    # eps, the regime the regularisation is for
    case = _case(dev, "f64", HEIS, 1024, 1, 5)
    got, diag = _run(case, "cholesky", 1e-4, 1e-12)
    ref, info = OM.minsr_eigh(case[4], case[5], 1e-4, 1e-12)
    assert diag[3] == 0.0
    err = _err(got, ref)
    print(f"n=1024 real minSR (Cholesky) relative error {err:.2e} "
          f"(lambda_max {info['lam_max']:.3g})")
    assert err <= 1e-8


def test_minsr_complex_ragged_multi_tile(dev):
    # 520 = 8 * 64 + 8 rows: a short last tile and block of the solves
    case = _case(dev, "c128", CHIRAL, 520, 3, 9)
    got, diag = _run(case, "cholesky", 1e-4, 1e-12)
    ref, _ = OM.minsr_eigh(case[4], case[5], 1e-4, 1e-12)
    assert diag[3] == 0.0
    err = _err(got, ref)
    print(f"n=520 complex minSR (Cholesky) relative error {err:.2e}")
    assert err <= 1e-8


@pytest.mark.parametrize("dtype,model,n,st,sc", [("f64", HEIS, 1024, 1, 5),
                                                 ("c128", CHIRAL, 520, 3, 9)])
def test_eigh_solver_matches_oracle(dev, dtype, model, n, st, sc):
    # the eigendecomposition path on its own: with the 704 (real) / 200
    # (complex) eigenvalues equal to eps forming one cluster that is kept
    case = _case(dev, dtype, model, n, st, sc)
    got, diag = _run(case, "eigh", 1e-4, 1e-12)
    ref, info = OM.minsr_eigh(case[4], case[5], 1e-4, 1e-12)
    assert diag[3] == 0.0 and diag[2] == info["n_cut"] == 0
    err = _err(got, ref)
    print(f"{dtype} n={n} eigh solver relative error {err:.2e}")
    assert err <= 1e-8


@pytest.mark.parametrize("dtype,model,n,st,sc", [("f64", HEIS, 1024, 1, 5),
                                                 ("c128", CHIRAL, 520, 3, 9)])
def test_auto_solver_after_a_failed_certificate(dev, dtype, model, n, st, sc):
    # rcond inside the widest gap of the spectrum: eigenvalues are dropped,
    # the trace certificate fails, the Cholesky solver returns NaN and the
    # automatic one the oracle's pseudo-inverse step
    case = _case(dev, dtype, model, n, st, sc)
    eps = 1e-4
    w = _spectrum(case[4], case[5], eps)
    rcond, n_cut = _gap_rcond(w)
    assert n_cut > 0
    got_c, diag_c = _run(case, "cholesky", eps, rcond)
    assert diag_c[3] == 1.0 and np.isnan(got_c).all()
    got, diag = _run(case, "auto", eps, rcond)
    ref, info = OM.minsr_eigh(case[4], case[5], eps, rcond)
    assert info["n_cut"] == n_cut
    assert diag[3] == 0.0 and diag[2] == n_cut
    err = _err(got, ref)
    print(f"{dtype} n={n} rcond={rcond:.3g}: {n_cut} dropped, auto solver relative error "
          f"{err:.2e}")
    assert err <= 1e-8


def test_auto_solver_equals_cholesky_when_certified(dev):
    case = _case(dev, "f64", HEIS, 1024, 1, 5)
    a, da = _run(case, "cholesky", 1e-4, 1e-12)
    b, db = _run(case, "auto", 1e-4, 1e-12)
    assert np.array_equal(a, b) and np.array_equal(da, db)


def test_eigh_solver_at_zero_shift(dev):
    # eps = 0: T itself is singular (rank <= 320 of 1024); the pseudo-inverse
    # drops its null space, giving the minimum-norm least-squares step
    case = _case(dev, "f64", HEIS, 1024, 1, 5)
    got, diag = _run(case, "eigh", 0.0, 1e-10)
    ref, info = OM.minsr_eigh(case[4], case[5], 0.0, 1e-10)
    assert diag[3] == 0.0 and diag[2] == info["n_cut"] >= 1024 - 320
    err = _err(got, ref)
    print(f"eps=0 eigh solver: {int(diag[2])} dropped, relative error {err:.2e}")
    assert err <= 1e-8


def test_eigh_solver_rejects_large_batches(dev):
    from paper_2503_12557_amd import Context
    from paper_2503_12557_amd.binding import PepsError
    ctx = Context(4, 4, 2, 4, "f64")
    ctx.set_minsr_solver("eigh")
    n = 3073
    O = torch.zeros(n, ctx.n_compact, dtype=torch.float64, device=dev)
    sm = torch.zeros(n, 16, dtype=torch.uint8, device=dev)
    el = torch.zeros(n, 2, dtype=torch.float64, device=dev)
    with pytest.raises(PepsError):
        ctx.minsr_step(O, sm, el)
