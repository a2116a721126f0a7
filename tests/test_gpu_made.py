"""The learned proposal on the GPU against the FP64 oracle: loss, gradient,
ln q and the Adam step (FP32 kernels, 1e-5 relative), the sampler's
distribution (chi-square against q enumerated over the S^z = 0 sector), the
independence-MH chain's distribution (chi-square against |Psi|^2), and what
training buys: the trained proposal's IMH acceptance rises above the
untrained one's and agrees with the exact acceptance computed by
enumeration."""
import numpy as np
import pytest
from scipy import stats

import synth
from oracle import made as OM
from oracle import peps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _made(N, H, n_up, bf16=False):
    from paper_2503_12557_amd.binding import Made
    return Made(N, H, n_up, bf16)


@pytest.mark.parametrize("N,H,n_up,B", [(16, 32, 8, 64), (36, 100, 18, 200), (64, 256, -1, 130)])
def test_loss_grad_logq_match_oracle(dev, N, H, n_up, B):
    nu = None if n_up < 0 else n_up
    p = OM.init_params(N, H, seed=N, scale=0.3)
    if nu is None:
        x = synth.bit_configs(N, B, seed=2)
    else:
        x = synth.sz0_configs(N, B, seed=2)
    m = _made(N, H, nu)
    pt = torch.tensor(p, dtype=torch.float32, device=dev)
    xt = torch.from_numpy(x).to(dev)
    loss, g = m.loss_grad(pt, xt)
    lq = m.logq(pt, xt)
    torch.cuda.synchronize()
    p32 = pt.double().cpu().numpy()  # the oracle sees the FP32-rounded parameters
    ref_loss, ref_g = OM.loss_and_grad(p32, x, N, H, nu)
    ref_lq = OM.log_q(p32, x, N, H, nu)
    assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss)
    assert np.abs(g.double().cpu().numpy() - ref_g).max() <= 1e-5 * np.abs(ref_g).max()
    assert np.abs(lq.cpu().numpy() - ref_lq).max() <= 1e-5 * np.abs(ref_lq).max()


def test_adam_step_matches_oracle(dev):
    N, H = 16, 32
    m = _made(N, H, 8)
    rng = np.random.default_rng(1)
    n = m.n_params
    p, g = rng.standard_normal(n), rng.standard_normal(n)
    mo, v = rng.random(n) * 0.1, rng.random(n) * 0.01
    t = lambda a: torch.tensor(a, dtype=torch.float32, device=dev)
    pt, gt, mt, vt = t(p), t(g), t(mo), t(v)
    m.adam(pt, gt, mt, vt, 7, lr=1e-3)
    # the kernel holds the hyper-parameters in FP32; the oracle gets the same values
    f = lambda z: float(np.float32(z))
    ref, rm, rv = OM.adam(t(p).double().cpu().numpy(), t(g).double().cpu().numpy(),
                          t(mo).double().cpu().numpy(), t(v).double().cpu().numpy(), 7,
                          lr=f(1e-3), b1=f(0.9), b2=f(0.999), eps=f(1e-8))
    assert np.abs(pt.double().cpu().numpy() - ref).max() < 1e-6
    assert np.abs(mt.double().cpu().numpy() - rm).max() < 1e-6
    assert np.abs(vt.double().cpu().numpy() - rv).max() < 1e-6 * np.abs(rv).max()


def test_sampler_distribution_and_logq(dev):
    N, H, n_up = 8, 16, 4
    p = OM.init_params(N, H, seed=5, scale=1.0)
    m = _made(N, H, n_up)
    pt = torch.tensor(p, dtype=torch.float32, device=dev)
    s, lq = m.sample(pt, 40000, seed=3)
    lq2 = m.logq(pt, s)
    torch.cuda.synchronize()
    sn = s.cpu().numpy()
    assert (np.sum(sn == 0, axis=1) == n_up).all()
    assert np.abs(lq.cpu().numpy() - lq2.cpu().numpy()).max() < 1e-5
    confs = OM.enumerate_sector(N, n_up)
    q = np.exp(OM.log_q(pt.double().cpu().numpy(), confs, N, H, n_up))
    idx = {tuple(c): i for i, c in enumerate(confs.tolist())}
    counts = np.zeros(len(confs))
    for row in sn.tolist():
        counts[idx[tuple(row)]] += 1
    exp = q * len(sn)
    keep = exp > 5
    c = np.append(counts[keep], counts[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    assert stats.chisquare(c, e).pvalue > 1e-3


def test_imh_chain_distribution(dev):
    from paper_2503_12557_amd import Context
    from paper_2503_12557_amd.binding import run_imh
    Lx, Ly, D, chi = 2, 3, 2, 4
    N = Lx * Ly
    theta = synth.theta(Lx, Ly, 2, D, seed=3)
    ctx = Context(Lx, Ly, D, chi, "f64")
    m = _made(N, 16, 3)
    pt = torch.tensor(OM.init_params(N, 16, seed=1, scale=0.5), dtype=torch.float32, device=dev)
    th = torch.from_numpy(theta).to(dev)
    # chains start from local-Metropolis samples of |Psi|^2, so every step of
    # an exact IMH chain is distributed as |Psi|^2
    init, _ = ctx.sample(th, "exchange", n_chains=512, per_chain=1, burn_in=30, seed=2)
    _, hist, acc = run_imh(ctx, th, m, pt, n_chains=512, n_steps=30, seed=11, record=True,
                           init=init)
    visited = hist[2::6].reshape(-1, N).cpu().numpy()
    confs = OM.enumerate_sector(N, 3)
    psi = peps.exact_amplitudes(theta, peps.Geometry(Lx, Ly, 2, D), confs)
    pr = np.abs(psi) ** 2
    pr /= pr.sum()
    idx = {tuple(c): i for i, c in enumerate(confs.tolist())}
    counts = np.zeros(len(confs))
    for row in visited.tolist():
        counts[idx[tuple(row)]] += 1
    exp = pr * len(visited)
    keep = exp > 5
    c = np.append(counts[keep], counts[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        c, e = c[:-1], e[:-1]
    assert stats.chisquare(c, e).pvalue > 1e-3


def test_training_raises_imh_acceptance(dev):
    # 4x4 exact contraction: train q on the PEPS sampler's configurations and
    # compare the IMH acceptance before and after with the exact acceptance
    from paper_2503_12557_amd import Context
    from paper_2503_12557_amd.binding import run_imh
    Lx, Ly, D, chi, H = 4, 4, 2, 4, 64
    N = Lx * Ly
    theta = synth.theta(Lx, Ly, 2, D, seed=1, mu=0.3)
    th = torch.from_numpy(theta).to(dev)
    ctx = Context(Lx, Ly, D, chi, "f32")
    data, _ = ctx.sample(th, "exchange", n_chains=1024, per_chain=8, burn_in=16, thin=2, seed=4)
    m = _made(N, H, N // 2)
    p0 = torch.tensor(OM.init_params(N, H, seed=2, scale=0.05), dtype=torch.float32, device=dev)
    pt = p0.clone()
    losses = m.train(pt, data, steps=400, batch=1024, lr=3e-3, seed=0)
    torch.cuda.synchronize()
    ls = losses.cpu().numpy()
    assert ls[-20:].mean() < ls[:20].mean() - 0.5
    confs = OM.enumerate_sector(N, N // 2)
    psi = peps.exact_amplitudes(theta, peps.Geometry(Lx, Ly, 2, D), confs)
    pr = np.abs(psi) ** 2
    pr /= pr.sum()
    ct = torch.from_numpy(confs).to(dev)
    acc_exact = []
    for p in (p0, pt):
        q = np.exp(m.logq(p, ct).cpu().numpy())
        acc_exact.append(OM.exact_imh_acceptance(pr, q / q.sum()))
    _, _, acc = run_imh(ctx, th, m, pt, n_chains=1024, n_steps=20, seed=9,
                        init=data[::8].contiguous())
    emp = acc.sum().item() / (1024 * 20)
    print(f"exact acceptance untrained {acc_exact[0]:.3f} trained {acc_exact[1]:.3f}, "
          f"empirical trained {emp:.3f}")
    assert acc_exact[1] > acc_exact[0] + 0.1
    assert abs(emp - acc_exact[1]) < 0.03


def _bf16_rne(a):
    """bfloat16 rounding (round to nearest, ties to even) of FP32 values,
    returned as FP64: the top 16 bits of the IEEE single after adding
    0x7fff plus the lowest kept bit."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("N,H,n_up,B", [(16, 32, 8, 64), (64, 256, 32, 256)])
def test_bf16_weights_match_oracle_on_rounded_weights(dev, N, H, n_up, B):
    # with bf16 weights the kernels use the weights rounded to bfloat16 and
    # accumulate in FP32; the oracle in FP64 on the same rounded weights
    # must agree to FP32 accumulation (the gradient is taken at the rounded
    # weights and applied to the FP32 master copy)
    p = OM.init_params(N, H, seed=N + 1, scale=0.3)
    x = synth.sz0_configs(N, B, seed=3)
    m = _made(N, H, n_up, bf16=True)
    pt = torch.tensor(p, dtype=torch.float32, device=dev)
    xt = torch.from_numpy(x).to(dev)
    loss, g = m.loss_grad(pt, xt)
    lq = m.logq(pt, xt)
    torch.cuda.synchronize()
    p32 = pt.double().cpu().numpy()
    W1, b1, W2, b2 = OM.unpack(p32, N, H)
    pr = np.concatenate([_bf16_rne(W1).ravel(), b1.ravel(), _bf16_rne(W2).ravel(), b2.ravel()])
    assert pr.shape == p32.shape and np.abs(pr - p32).max() > 0  # the rounding acts
    ref_loss, ref_g = OM.loss_and_grad(pr, x, N, H, n_up)
    ref_lq = OM.log_q(pr, x, N, H, n_up)
    e_loss = abs(loss.item() - ref_loss) / abs(ref_loss)
    e_g = np.abs(g.double().cpu().numpy() - ref_g).max() / np.abs(ref_g).max()
    e_lq = np.abs(lq.cpu().numpy() - ref_lq).max() / np.abs(ref_lq).max()
    print(f"bf16 MADE N={N}: loss {e_loss:.2e} grad {e_g:.2e} ln q {e_lq:.2e}")
    assert e_loss <= 1e-5 and e_g <= 1e-5 and e_lq <= 1e-5


def _splitmix64_stream(seed):
    """splitmix64 (Steele, Lea and Flood; Vigna's constants) from its
    definition: state += golden gamma, then two xor-shift-multiply rounds."""
    M64 = (1 << 64) - 1
    x = seed & M64
    while True:
        x = (x + 0x9E3779B97F4A7C15) & M64
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        yield z ^ (z >> 31)


def _epoch_rows(M, steps, batch, seed):
    """Rows of every batch under the documented made_train order: epoch e
    visits row (a_e r + c_e) mod M at its position r, a_e coprime with M."""
    from math import gcd
    g = _splitmix64_stream(seed)
    epochs = steps * batch // M + 2
    tab = []
    for _ in range(epochs):
        a = next(g) % M if M > 1 else 1
        a = a or 1
        while gcd(a, M) != 1:
            a = a + 1 if a + 1 < M else 1
        tab.append((a, next(g) % M))
    rows = []
    for i in range(steps):
        pos = np.arange(i * batch, (i + 1) * batch)
        e, r = pos // M, pos % M
        rows.append(np.array([(tab[ee][0] * rr + tab[ee][1]) % M for ee, rr in zip(e, r)]))
    return rows


def test_made_train_equals_oracle_loop(dev):
    # the library's training loop (one call, five Adam steps over permuted
    # batches that cross an epoch boundary) against the oracle's loss,
    # gradient and Adam on the same batches
    N, H, n_up, M, B, steps, seed = 16, 32, 8, 200, 64, 5, 12345
    data = synth.sz0_configs(N, M, seed=9)
    p0 = OM.init_params(N, H, seed=4, scale=0.3)
    m = _made(N, H, n_up)
    pt = torch.tensor(p0, dtype=torch.float32, device=dev)
    losses = m.train(pt, torch.from_numpy(data).to(dev), steps=steps, batch=B, lr=1e-2, seed=seed)
    torch.cuda.synchronize()
    f = lambda z: float(np.float32(z))
    p = torch.tensor(p0, dtype=torch.float32).double().numpy()
    mo = np.zeros_like(p)
    v = np.zeros_like(p)
    ref_l = []
    for i, rows in enumerate(_epoch_rows(M, steps, B, seed)):
        assert len(set(rows.tolist())) == B or i * B // M != ((i + 1) * B - 1) // M
        loss, g = OM.loss_and_grad(p, data[rows], N, H, n_up)
        ref_l.append(loss)
        p, mo, v = OM.adam(p, g, mo, v, i + 1, lr=f(1e-2), b1=f(0.9), b2=f(0.999), eps=f(1e-8))
    got = pt.double().cpu().numpy()
    print("made_train: param err %.2e loss err %.2e" % (
        np.abs(got - p).max() / np.abs(p).max(),
        np.abs(losses.cpu().numpy() - ref_l).max() / np.abs(ref_l).max()))
    assert np.abs(losses.cpu().numpy() - np.array(ref_l)).max() <= 1e-5 * np.abs(ref_l).max()
    assert np.abs(got - p).max() <= 1e-4 * np.abs(p).max()


def test_tau_int_kernel_matches_oracle(dev):
    # the library's tau_int (peps_tau_int) against the oracle's direct sums,
    # plain and on the oracle's rank-normalised series; ties in the data
    # (sticky chains repeat values) exercise the average ranks
    from paper_2503_12557_amd import analysis
    rng = np.random.default_rng(3)
    C, T, a = 32, 300, 0.6
    x = np.zeros((C, T))
    e = rng.standard_normal((C, T))
    for t in range(1, T):
        x[:, t] = a * x[:, t - 1] + e[:, t]
    p = 0.67
    y = np.empty((256, 64))
    y[:, 0] = rng.standard_cauchy(256)
    for t in range(1, 64):
        keep = rng.random(256) < p
        y[:, t] = np.where(keep, y[:, t - 1], rng.standard_cauchy(256))
    for s in (x, y):
        got, ref = analysis.tau_int(s), OM.integrated_autocorr(s)
        assert abs(got - ref) <= 1e-9 * ref
        got_r, ref_r = analysis.tau_int_ranked(s), OM.integrated_autocorr(OM.rank_normalise(s))
        print(f"tau_int {got:.6f} / {ref:.6f}; ranked {got_r:.6f} / {ref_r:.6f}")
        assert abs(got_r - ref_r) <= 1e-9 * ref_r


def test_imh_sampler_kind_equals_its_building_blocks(dev):
    # peps_sample with the IMH kind against the same chain assembled from
    # made_sample, peps_amplitude and imh_step: identical states, ln Psi and
    # acceptance counts; the local kinds' ln Psi output equals peps_amplitude
    from paper_2503_12557_amd import Context
    from paper_2503_12557_amd.binding import imh_step
    Lx, Ly, D, chi = 3, 4, 2, 4
    N = Lx * Ly
    theta = synth.theta(Lx, Ly, 2, D, seed=8)
    th = torch.from_numpy(theta).to(dev)
    ctx = Context(Lx, Ly, D, chi, "f64")
    m = _made(N, 32, N // 2)
    pt = torch.tensor(OM.init_params(N, 32, seed=3, scale=0.5), dtype=torch.float32, device=dev)
    init, _, lp_init = ctx.sample(th, "exchange", n_chains=64, per_chain=1, burn_in=10, seed=5,
                                  want_logpsi=True)
    ref_lp, _ = ctx.amplitude(th, init)
    torch.cuda.synchronize()
    assert torch.equal(lp_init, ref_lp)
    s, acc, lp = ctx.sample(th, "imh", n_chains=64, per_chain=3, burn_in=2, thin=2, seed=9,
                            offset=4, proposal=(m, pt, init), want_logpsi=True)
    # the same chain by hand
    state = init.clone()
    st_lq = m.logq(pt, state)
    st_lp, _ = ctx.amplitude(th, state)
    acc2 = torch.zeros(64, dtype=torch.int32, device=dev)
    rec, rec_lp = [], []
    for t in range(1, 2 + 3 * 2 + 1):
        prop, pr_lq = m.sample(pt, 64, seed=9, offset=4 + t)
        pr_lp, _ = ctx.amplitude(th, prop)
        imh_step(state, st_lp, st_lq, prop, pr_lp, pr_lq, 9, 4 + t, acc2)
        if t > 2 and (t - 2) % 2 == 0:
            rec.append(state.clone())
            rec_lp.append(st_lp.clone())
    torch.cuda.synchronize()
    want = torch.stack(rec, 1).reshape(64 * 3, N)
    want_lp = torch.stack(rec_lp, 1).reshape(64 * 3, 2)
    assert torch.equal(s, want) and torch.equal(lp, want_lp) and torch.equal(acc, acc2)
    assert acc.sum().item() > 0
