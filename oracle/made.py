"""Oracle for the learned proposal: a masked autoregressive network (MADE)
over the N sites in raster order, its loss, gradients and Adam step, the
independence Metropolis-Hastings acceptance and integrated autocorrelation.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). Plain numpy FP64.

The paper samples its PEPS directly and corrects approximate samples by
importance weights (App. "direct sampling of PEPS"); the learned proposal is
an extension: the PEPS stays the arbiter through the Metropolis-Hastings
acceptance |Psi(S')|^2 q(S) / (|Psi(S)|^2 q(S')).

Model (one hidden layer of width H, ReLU):
  hidden degree m(k) = (k mod (N-1)) + 1,
  M1[k, n] = [m(k) >= n + 1],  M2[n, k] = [n + 1 > m(k)],
  h = relu(b1 + (W1 * M1) x),  logit_n = b2_n + ((W2 * M2) h)_n,
  p(s_n = 1 | s_<n) = sigmoid(logit_n), input x_n = s_n in {0, 1}.
With a fixed number n_up of zeros (spin up, S^z = 0 sector) a site is
forced once the zeros or the ones are used up; forced sites contribute a
factor 1 to q and nothing to the loss.
Parameter vector: W1 [H][N], b1 [H], W2 [N][H], b2 [N] (C order).
"""
from __future__ import annotations

import math

import numpy as np


def masks(N, H):
    k = np.arange(H)
    mk = (k % (N - 1)) + 1
    n = np.arange(N)
    M1 = (mk[:, None] >= n[None, :] + 1).astype(np.float64)
    M2 = (n[:, None] + 1 > mk[None, :]).astype(np.float64)
    return M1, M2


def unpack(p, N, H):
    o = 0
    W1 = p[o:o + H * N].reshape(H, N); o += H * N
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + N * H].reshape(N, H); o += N * H
    b2 = p[o:o + N]
    return W1, b1, W2, b2


def n_params(N, H):
    return 2 * N * H + N + H


def free_mask(x, n_up):
    """1 where site n is sampled, 0 where the S^z constraint forces it."""
    B, N = x.shape
    if n_up is None or n_up < 0:
        return np.ones((B, N))
    n_dn = N - n_up
    zeros = np.cumsum(x == 0, axis=1) - (x == 0)   # zeros before n
    ones = np.cumsum(x == 1, axis=1) - (x == 1)
    forced = (zeros >= n_up) | (ones >= n_dn)
    return (~forced).astype(np.float64)


def forward(p, x, N, H):
    W1, b1, W2, b2 = unpack(p, N, H)
    M1, M2 = masks(N, H)
    xf = x.astype(np.float64)
    a = xf @ (W1 * M1).T + b1
    h = np.maximum(a, 0.0)
    logit = h @ (W2 * M2).T + b2
    return a, h, logit


def _log_sigmoid(z):
    return -np.logaddexp(0.0, -z)


def log_q(p, x, N, H, n_up):
    _, _, logit = forward(p, x, N, H)
    f = free_mask(x, n_up)
    xf = x.astype(np.float64)
    ll = xf * _log_sigmoid(logit) + (1 - xf) * _log_sigmoid(-logit)
    return (f * ll).sum(axis=1)


def loss_and_grad(p, x, N, H, n_up):
    """Mean negative log-likelihood over the batch and its gradient."""
    W1, b1, W2, b2 = unpack(p, N, H)
    M1, M2 = masks(N, H)
    a, h, logit = forward(p, x, N, H)
    B = x.shape[0]
    xf = x.astype(np.float64)
    f = free_mask(x, n_up)
    ll = xf * _log_sigmoid(logit) + (1 - xf) * _log_sigmoid(-logit)
    loss = -(f * ll).sum() / B
    sig = 1.0 / (1.0 + np.exp(-logit))
    dlogit = f * (sig - xf) / B
    dW2 = (dlogit.T @ h) * M2
    db2 = dlogit.sum(axis=0)
    dh = dlogit @ (W2 * M2)
    da = dh * (a > 0)
    dW1 = (da.T @ xf) * M1
    db1 = da.sum(axis=0)
    return loss, np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2])


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba), t counted from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def imh_accept_log_ratio(lp_new, lp_old, lq_new, lq_old):
    """ln of |Psi(S')|^2 q(S) / (|Psi(S)|^2 q(S'))."""
    return 2.0 * (lp_new - lp_old) + lq_old - lq_new


def exact_imh_acceptance(p_psi, q):
    """Mean acceptance of independence MH at stationarity:
    sum_{S,S'} p(S) q(S') min(1, w(S')/w(S)) with w = p/q."""
    w = p_psi / q
    order = np.argsort(w)
    ws, ps, qs = w[order], p_psi[order], q[order]
    # for each S: sum over S' of q(S') min(1, w'/w)
    cq = np.cumsum(qs)           # q mass of S' with w' <= w (inclusive)
    cp = np.cumsum(ps)           # p mass of those
    tot = 0.0
    for i in range(len(ws)):
        below = cp[i] / ws[i]    # sum_{w' <= w} q' w'/w = sum p'/w
        above = 1.0 - cq[i]      # sum_{w' > w} q'
        tot += ps[i] * (below + above)
    return tot


def integrated_autocorr(series, c=5.0):
    """tau_int with Sokal's automatic window (smallest W >= c * tau(W)), the
    autocorrelation averaged over chains that start stationary, centred on
    the mean over all chains. series: [chains, T]."""
    x = np.asarray(series, dtype=np.float64)
    x = x - x.mean()
    C, T = x.shape
    var = (x * x).mean()
    if var == 0:
        return 1.0
    rho = np.empty(T)
    for t in range(T):
        rho[t] = (x[:, :T - t] * x[:, t:]).mean() / var
    tau = 1.0
    for W in range(1, T):
        tau = 1.0 + 2.0 * rho[1:W + 1].sum()
        if W >= c * tau:
            break
    return max(tau, 1.0)


def rank_normalise(series):
    """Normal scores Phi^-1((r - 3/8) / (S + 1/4)) of the pooled ranks r of
    a series (average ranks for ties, S values; Blom's offsets), the
    rank-normalised series of Vehtari et al. (2021), for tau_int of
    heavy-tailed local energies."""
    from scipy.special import ndtri
    from scipy.stats import rankdata
    x = np.asarray(series, dtype=np.float64)
    r = rankdata(x.ravel(), method="average").reshape(x.shape)
    return ndtri((r - 0.375) / (x.size + 0.25))


def enumerate_sector(N, n_up):
    """All configurations of N bits with exactly n_up zeros, as uint8 [M, N]."""
    out = []
    for v in range(2 ** N):
        bits = [(v >> (N - 1 - i)) & 1 for i in range(N)]
        if n_up is None or bits.count(0) == n_up:
            out.append(bits)
    return np.array(out, dtype=np.uint8)


def init_params(N, H, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(n_params(N, H))


def log1pexp(z):
    return math.log1p(math.exp(z)) if z < 30 else z
