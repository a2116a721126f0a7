"""Chain statistics for the sampler comparison: the integrated
autocorrelation time and the effective sample size of a scalar series on
many chains, computed by the library's kernel (peps_tau_int: Sokal's
automatic window on the chain-averaged autocorrelation, optionally on the
rank-normalised series). Argument marshalling only."""
from __future__ import annotations


def _tau(series, ranked, c):
    import torch

    from .binding import _check, _ptr, _stream, load
    x = torch.as_tensor(series, dtype=torch.float64)
    if not x.is_cuda:
        x = x.to("cuda")
    x = x.contiguous()
    nc, T = x.shape
    work = torch.empty(nc * T + T, dtype=torch.float64, device=x.device)
    out = torch.empty(2, dtype=torch.float64, device=x.device)
    _check(load().peps_tau_int(_ptr(x), nc, T, 1 if ranked else 0, float(c), _ptr(work), _ptr(out),
                               _stream()))
    return float(out[0].item())


def tau_int(series, c=5.0):
    """tau_int of series [chains, T] (device tensor or array)."""
    return _tau(series, False, c)


def tau_int_ranked(series, c=5.0):
    """tau_int of the rank-normalised series (normal scores of pooled ranks)."""
    return _tau(series, True, c)


def ess(series, c=5.0, ranked=False):
    import torch
    x = torch.as_tensor(series)
    return x.numel() / _tau(series, ranked, c)
