"""Chain statistics for the sampler comparison (host side, numpy).

tau_int of a scalar series observed on many chains, with Sokal's automatic
window: the autocorrelation rho(t) is averaged over chains and the window W
is the smallest with W >= c * tau(W), tau(W) = 1 + 2 sum_{t=1..W} rho(t).
The chains start from stationary states, so the series is centred on the
mean over all chains (centring each short chain on its own mean would bias
rho(t) low). The effective sample size of chains x T observations is
chains*T / tau_int.

Local energies of unconverged states are heavy-tailed (a few near-zero
amplitudes carry almost all of the variance), which makes the plain
autocorrelation a statistic of a handful of outliers. tau_int_ranked
applies the estimator to rank-normalised values (normal scores of the
pooled ranks, Blom's offsets, as in the rank-normalised effective sample
size of Vehtari et al., 2021), which is invariant under monotone maps of
the observable.
"""
from __future__ import annotations

import numpy as np


def tau_int(series, c=5.0):
    x = np.asarray(series, dtype=np.float64)
    x = x - x.mean()
    T = x.shape[1]
    var = float((x * x).mean())
    if var == 0.0 or T < 2:
        return 1.0
    f = np.fft.rfft(x, n=2 * T, axis=1)
    ac = np.fft.irfft(f * np.conj(f), axis=1)[:, :T].mean(axis=0)
    ac /= np.arange(T, 0, -1)
    rho = ac / ac[0]
    tau = 1.0
    for W in range(1, T):
        tau = 1.0 + 2.0 * rho[1:W + 1].sum()
        if W >= c * tau:
            break
    return max(float(tau), 1.0)


def ess(series, c=5.0):
    x = np.asarray(series)
    return x.size / tau_int(x, c)


def rank_normalise(series):
    """Normal scores Phi^-1((r - 3/8) / (S + 1/4)) of the pooled ranks r
    (ties share their average rank); S = number of values."""
    from scipy.special import ndtri
    from scipy.stats import rankdata
    x = np.asarray(series, dtype=np.float64)
    r = rankdata(x.ravel(), method="average").reshape(x.shape)
    return ndtri((r - 0.375) / (x.size + 0.25))


def tau_int_ranked(series, c=5.0):
    return tau_int(rank_normalise(series), c)
