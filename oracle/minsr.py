"""Oracle minSR step (Sec. "Reformulation of the imaginary-time Schroedinger
equation for sampling techniques", Eqs. tdvp, tdvp_slow, tdvp_fast).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings of the paper taken here:
  * O and E_loc are centred over the batch and scaled by 1/sqrt(N_s)
    (the normalisation term the paper mentions but does not write out);
  * eps*I is added to T = O O^dagger, eigenvalues of T + eps*I below
    rcond * (largest eigenvalue) are discarded in the pseudo-inverse;
  * the returned dtheta is the solution of O dtheta = E_loc, i.e. the
    parameters move as theta <- theta - tau * dtheta.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def centre(O, E):
    """O-bar = (O - <O>)/sqrt(Ns), eps-bar = (E - <E>)/sqrt(Ns)."""
    n = O.shape[0]
    Ob = (O - O.mean(axis=0, keepdims=True)) / np.sqrt(n)
    Eb = (E - E.mean()) / np.sqrt(n)
    return Ob, Eb


def gram(Ob):
    """T_SS' = sum_i O_Si O*_S'i (Eq. tdvp_fast)."""
    return Ob @ Ob.conj().T


def minsr_eigh(O, E, eps, rcond):
    """dtheta = O^dagger (T + eps I)^+ E by an eigenvalue decomposition of
    the N_s x N_s matrix T (the paper's solver)."""
    Ob, Eb = centre(O, E)
    T = gram(Ob)
    n = T.shape[0]
    w, V = sla.eigh(T + eps * np.eye(n))
    keep = w > rcond * w.max()
    y = V[:, keep] @ ((V[:, keep].conj().T @ Eb) / w[keep])
    return Ob.conj().T @ y, dict(lam_max=w.max(), lam_min=w.min(),
                                 n_cut=int((~keep).sum()))


def minsr_cholesky(O, E, eps):
    """Same step solved by a Cholesky factorisation of T + eps I."""
    Ob, Eb = centre(O, E)
    T = gram(Ob)
    n = T.shape[0]
    c = sla.cho_factor(T + eps * np.eye(n), lower=True)
    y = sla.cho_solve(c, Eb)
    return Ob.conj().T @ y


def sr_parameter_space(O, E, eps):
    """The conventional form (O^dagger O + eps I)^-1 O^dagger E in the
    N_p x N_p parameter space (Eq. tdvp_slow), for small N_p only."""
    Ob, Eb = centre(O, E)
    G = Ob.conj().T @ Ob
    return np.linalg.solve(G + eps * np.eye(G.shape[0]), Ob.conj().T @ Eb)
