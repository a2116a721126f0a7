"""Pins of the learned-proposal oracle (CPU only): normalisation of q over the
S^z = 0 sector, the autoregressive property of the masks, gradients against
central finite differences and torch's FP64 autograd, exact IMH acceptance
against a brute-force double sum, and tau_int of an AR(1) series."""
import itertools

import numpy as np
import pytest

from oracle import made


@pytest.mark.parametrize("n_up", [None, 8])
def test_q_is_normalised(n_up):
    N, H = 16, 24
    p = made.init_params(N, H, seed=1, scale=0.5)
    x = made.enumerate_sector(N, n_up)
    q = np.exp(made.log_q(p, x, N, H, n_up))
    assert abs(q.sum() - 1) < 1e-12


def test_autoregressive_masks():
    # logit_n must not depend on inputs n' >= n
    N, H = 10, 16
    p = made.init_params(N, H, seed=2, scale=1.0)
    rng = np.random.default_rng(0)
    x = rng.integers(0, 2, (1, N)).astype(np.uint8)
    _, _, l0 = made.forward(p, x, N, H)
    for j in range(N):
        x2 = x.copy()
        x2[0, j] ^= 1
        _, _, l1 = made.forward(p, x2, N, H)
        assert np.abs(l1[0, :j + 1] - l0[0, :j + 1]).max() == 0.0


def test_gradient_finite_differences():
    N, H, n_up = 8, 12, 4
    p = made.init_params(N, H, seed=3, scale=0.7)
    x = made.enumerate_sector(N, n_up)[::3]
    loss, g = made.loss_and_grad(p, x, N, H, n_up)
    rng = np.random.default_rng(1)
    for k in rng.choice(len(p), 25, replace=False):
        e = np.zeros_like(p)
        e[k] = 1e-6
        fd = (made.loss_and_grad(p + e, x, N, H, n_up)[0]
              - made.loss_and_grad(p - e, x, N, H, n_up)[0]) / 2e-6
        assert abs(fd - g[k]) < 1e-7 * max(1, abs(g[k]))


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    N, H, n_up = 12, 20, 6
    p = made.init_params(N, H, seed=4, scale=0.5)
    rng = np.random.default_rng(2)
    x = np.array([rng.permutation([0] * 6 + [1] * 6) for _ in range(32)], dtype=np.uint8)
    loss, g = made.loss_and_grad(p, x, N, H, n_up)
    M1, M2 = made.masks(N, H)
    pt = torch.tensor(p, requires_grad=True)
    W1 = pt[:H * N].reshape(H, N)
    b1 = pt[H * N:H * N + H]
    W2 = pt[H * N + H:H * N + H + N * H].reshape(N, H)
    b2 = pt[H * N + H + N * H:]
    xt = torch.tensor(x, dtype=torch.float64)
    h = torch.relu(xt @ (W1 * torch.tensor(M1)).T + b1)
    logit = h @ (W2 * torch.tensor(M2)).T + b2
    f = torch.tensor(made.free_mask(x, n_up))
    ll = xt * torch.nn.functional.logsigmoid(logit) + (1 - xt) * torch.nn.functional.logsigmoid(-logit)
    lt = -(f * ll).sum() / len(x)
    lt.backward()
    assert abs(lt.item() - loss) < 1e-12
    assert np.abs(pt.grad.numpy() - g).max() < 1e-12


def test_exact_imh_acceptance_brute_force():
    rng = np.random.default_rng(3)
    m = 30
    p = rng.random(m)
    p /= p.sum()
    q = rng.random(m)
    q /= q.sum()
    ref = 0.0
    for i, j in itertools.product(range(m), range(m)):
        ref += p[i] * q[j] * min(1.0, (p[j] / q[j]) / (p[i] / q[i]))
    assert abs(made.exact_imh_acceptance(p, q) - ref) < 1e-12
    # a perfect proposal is always accepted
    assert abs(made.exact_imh_acceptance(p, p) - 1) < 1e-12


def test_tau_int_of_ar1_series():
    # AR(1) with coefficient a has tau_int = (1 + a) / (1 - a)
    a = 0.8
    rng = np.random.default_rng(4)
    C, T = 64, 4000
    x = np.zeros((C, T))
    e = rng.standard_normal((C, T))
    for t in range(1, T):
        x[:, t] = a * x[:, t - 1] + e[:, t]
    tau = made.integrated_autocorr(x[:, 200:])
    assert abs(tau - 9.0) < 1.0


def test_adam_first_step_is_sign_step():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.1, 0.0])
    p2, m, v = made.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=1e-3)
    assert np.allclose(p2[:2], p[:2] - 1e-3 * np.sign(g[:2]), atol=1e-9)
    assert p2[2] == p[2]


def test_tau_int_of_ar1_closed_form():
    # AR(1) x_t = a x_{t-1} + e_t started stationary: rho(t) = a^t and
    # tau_int = (1 + a) / (1 - a) = 4 for a = 0.6
    rng = np.random.default_rng(9)
    C, T, a = 64, 2000, 0.6
    x = np.zeros((C, T))
    e = rng.standard_normal((C, T))
    x[:, 0] = e[:, 0] / np.sqrt(1 - a * a)
    for t in range(1, T):
        x[:, t] = a * x[:, t - 1] + e[:, t]
    assert abs(made.integrated_autocorr(x) - (1 + a) / (1 - a)) < 0.25


def test_tau_int_of_short_sticky_chains():
    # an independence chain that keeps its value with probability p has
    # rho(t) = p^t, tau_int = (1 + p) / (1 - p); short chains started from
    # the stationary law (T = 64, as in the sampler comparison)
    p, C, T = 0.67, 4096, 64
    rng = np.random.default_rng(5)
    x = np.empty((C, T))
    x[:, 0] = rng.standard_normal(C)
    for t in range(1, T):
        keep = rng.random(C) < p
        x[:, t] = np.where(keep, x[:, t - 1], rng.standard_normal(C))
    tau = made.integrated_autocorr(x)
    assert abs(tau - (1 + p) / (1 - p)) < 0.3


def test_ranked_tau_int_is_robust_to_heavy_tails():
    # the sticky chains above with Cauchy values: the ranked estimate keeps
    # the closed form, and for Gaussian AR(1) values it agrees with the
    # plain estimate
    p, C, T = 0.67, 4096, 64
    rng = np.random.default_rng(6)
    x = np.empty((C, T))
    x[:, 0] = rng.standard_cauchy(C)
    for t in range(1, T):
        keep = rng.random(C) < p
        x[:, t] = np.where(keep, x[:, t - 1], rng.standard_cauchy(C))
    assert abs(made.integrated_autocorr(made.rank_normalise(x)) - (1 + p) / (1 - p)) < 0.3
    a = 0.6
    y = np.zeros((64, 800))
    e = rng.standard_normal(y.shape)
    y[:, 0] = e[:, 0] / np.sqrt(1 - a * a)
    for t in range(1, y.shape[1]):
        y[:, t] = a * y[:, t - 1] + e[:, t]
    assert abs(made.integrated_autocorr(made.rank_normalise(y)) - made.integrated_autocorr(y)) < 0.2
    # normal scores of distinct values: symmetric about zero, increasing
    z = made.rank_normalise(np.array([[3.0, -1.0, 7.0, 0.5]]))
    assert np.allclose(np.sort(z[0]), -np.sort(z[0])[::-1]) and z[0, 2] > z[0, 0] > z[0, 3] > z[0, 1]
