"""Oracle optimisation loop: repeated minSR steps (Sec. "Reformulation of
the imaginary-time Schroedinger equation for sampling techniques", Eq. tdvp,
iterated as in the optimisations of Sec. "Results").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

One step: draw samples from p(S) ~ |Psi(S)|^2 with the local Metropolis
sampler (``sampler.metropolis``), evaluate E_loc and the log-derivatives on
them (``peps.evaluate``), solve the minSR system (``minsr.minsr_eigh``) and
move theta <- theta - tau * dtheta.

Readings taken here (the paper fixes neither):
  * the step size tau is a constant;
  * step k draws its random numbers at sweep offset
    offset0 + k * (burn_in + per_chain * thin), so consecutive steps use
    disjoint Philox counters, and every step restarts the chains from the
    sampler's initial states;
  * real parameters move along the real part of E_loc (as the minSR step
    does for real modes); complex parameters use the complex E_loc.
"""
from __future__ import annotations

import numpy as np

from . import minsr, peps, sampler


def step(theta, g, chi, ham, kind, n_chains, per_chain, burn_in, thin, seed, offset, tau,
         eps, rcond):
    """One minSR step. Returns the new theta, the batch mean of E_loc (real
    part), the samples and E_loc."""
    samples, _ = sampler.metropolis(theta, g, chi, kind, n_chains, per_chain, burn_in, thin,
                                    seed, offset)
    _, eloc, Oc = peps.evaluate(theta, g, samples, chi, ham, want_O=True)
    O = np.array([peps.expand_compact(Oc[i], g, samples[i]) for i in range(len(samples))])
    cplx = np.iscomplexobj(theta)
    E = eloc if cplx else eloc.real
    dth, _ = minsr.minsr_eigh(O, E, eps, rcond)
    if not cplx:
        dth = dth.real
    return theta - tau * dth, float(np.real(eloc).mean()), samples, eloc


def optimize(theta, g, chi, ham, kind, n_chains, per_chain, burn_in, thin, seed, tau, eps,
             rcond, steps, offset0=0):
    """`steps` minSR steps from theta; returns the final theta and the batch
    mean energy of every step (measured before that step's update)."""
    stride = burn_in + per_chain * thin
    energies = []
    for k in range(steps):
        theta, e, _, _ = step(theta, g, chi, ham, kind, n_chains, per_chain, burn_in, thin,
                              seed, offset0 + k * stride, tau, eps, rcond)
        energies.append(e)
    return theta, np.array(energies)
