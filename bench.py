"""Throughput of the sampled finite-PEPS hot path on one MI355X.

Timed workload (10x10 open lattice, d=2, D=5, chi=25, complex tensors with
real and imaginary parts i.i.d. N(0,1) from seed 4, chiral spin-liquid
Hamiltonian J1=1, J2=0.5, J_chi=0.2; 8192 configurations drawn once, before
the timed region, by the library's exchange Metropolis sampler in
complex128): one step evaluates ln Psi, the local energies E_loc and the
log-derivatives O of one batch of configurations (consecutive steps cycle
through the 8192) in complex64 with the density-matrix truncation on the
matrix cores. The same 8192 configurations are evaluated in complex128
outside the timed region, and the relative error of the mean energy on
identical samples is reported, with per-configuration quantiles.

Prints one JSON line. Extra fields: complex128 throughput, the minSR step
at n = 8192 (complex parameters, FP64 solve), the per-kernel split from HIP
events, the roofline of the dominant kernel, the oracle timed on the host's
cores on a bounded sample, the 8x8 D=4 chi=16 and 12x12 D=4 chi=16 Rydberg
workloads in FP32 / BF16 against FP64, and the learned-proposal comparison.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks (dense)
    "fp32_matrix_tflops": 157.3,
    "fp64_matrix_tflops": 78.6,
    "fp32_vector_tflops": 157.3,
    "fp64_vector_tflops": 78.6,
    "hbm_gbs": 8000.0,
}


def _legs(Lx, Ly, D, x, y):
    return (1 if y == 0 else D, 1 if y == Ly - 1 else D, 1 if x == 0 else D,
            1 if x == Lx - 1 else D)


def env_bonds(Lx, Ly, D, chi):
    """Bond dimensions of every boundary MPS (as the library's tables): for
    each direction and absorbed row t, per site the (bl, br) of the previous
    environment, the rank bound kk of the left sweep and the new bond r."""
    out = []
    for direction in (0, 1):
        x0 = 0 if direction == 0 else Lx - 1
        right = [_legs(Lx, Ly, D, x0, y)[1] for y in range(Ly)]
        left = [1] + right[:-1]
        rows = []
        for t in range(1, Lx - 1):
            x = t if direction == 0 else Lx - 1 - t
            kk, kp = [], 1
            for y in range(Ly - 1):
                Dl, Dr, Du, Dd = _legs(Lx, Ly, D, x, y)
                Dout = Dd if direction == 0 else Du
                kp = min(kp * Dout, right[y] * Dr)
                kk.append(kp)
            new_l, new_r, nbr = [1] * Ly, [1] * Ly, 1
            sites = []
            for y in range(Ly - 1, -1, -1):
                Dl, Dr, Du, Dd = _legs(Lx, Ly, D, x, y)
                Din, Dout = (Du, Dd) if direction == 0 else (Dd, Du)
                r = min(chi, kk[y - 1], Dout * nbr) if y > 0 else 1
                sites.append(dict(y=y, bl=left[y], br=right[y], Dl=Dl, Dr=Dr, Din=Din,
                                  Dout=Dout, nbr=nbr, r=r))
                new_l[y], new_r[y], nbr = r, sites[-1]["nbr"], r
            rows.append(sites[::-1])
            left, right = new_l, new_r
        out.append(rows)
    return out


# flops of the canonical (QR -> SVD) environment build of one 10x10 D=5
# chi=25 complex sample, both sweeps, complex products counted as four real
# ones: products 7.4 GF, Householder QR 5.3 GF, SVD with right vectors
# 12.2 GF (shape-tracked per site)
CANONICAL_ENV_FLOPS_10x10_D5_CHI25 = 24.9e9


def dm_env_flops_per_sample(Lx, Ly, D, chi, cplx):
    """Algorithmic flops of the density-matrix environment build per sample
    (both directions), split into matrix-core work (the Gram, projection,
    density and weight products) and the rest (eigensolver). A real
    m x n x k product counts 2mnk, a complex one 8mnk; a Hermitian result
    counts its lower triangle; the Householder tridiagonalisation of an n x n
    Hermitian matrix 16n^3/3 (complex) or 4n^3/3 (real), its back
    transformation of r vectors 8 n^2 r (complex) or 2 n^2 r."""
    cf = 4.0 if cplx else 1.0
    mm = alu = 0.0
    for rows in env_bonds(Lx, Ly, D, chi):
        for sites in rows:
            for st in sites[:-1]:   # left sweep: G E, then A, conj(A), conj(E)
                bl, br, Dl, Dr = st["bl"], st["br"], st["Dl"], st["Dr"]
                Din, Dout = st["Din"], st["Dout"]
                mm += cf * 2.0 * (bl * Dl * Dl * Din * br * bl
                                  + bl * Dl * br * Dr * Dout * Dl * Din
                                  + bl * br * Dr * Din * Dr * Dl * Dout
                                  + br * Dr * Dr * br * bl * Din)
            for st in sites:        # right sweep
                Pl = st["bl"] * st["Dl"]
                zc = st["Dout"] * st["nbr"]
                mm += cf * 2.0 * st["bl"] * st["Din"] * st["nbr"] * st["br"] * st["Dr"]
                mm += cf * 2.0 * Pl * zc * st["Din"] * st["Dr"]
                if st["y"] > 0:
                    mm += cf * (2.0 * Pl * Pl * zc + Pl * zc * (zc + 1.0) + 2.0 * Pl * zc * st["r"])
                    alu += (16.0 / 3.0 if cplx else 4.0 / 3.0) * zc ** 3
                    alu += (8.0 if cplx else 2.0) * zc * zc * st["r"]
    return mm, alu


def canonical_env_flops_per_sample(Lx, Ly, D, chi):
    """Algorithmic flops of the canonical (QR -> SVD) environment build per
    sample and both sweeps, real tensors: GEMM 2mnk, Householder R of m x n
    2mn^2 - 2n^3/3, SVD of m x n (m <= n) with its right vectors
    4 m^2 n + 8 m^3."""
    total = 0.0
    for rows in env_bonds(Lx, Ly, D, chi):
        for sites in rows:
            kp = 1
            kks = []
            for st in sites[:-1]:
                Pl, Pr = st["bl"] * st["Dl"], st["br"] * st["Dr"]
                total += st["Dout"] * 2.0 * Pl * Pr * st["Din"]
                if st["y"] > 0:
                    total += st["Dout"] * 2.0 * kp * Pl * Pr
                m, n = kp * st["Dout"], Pr
                total += (2.0 * m * n * n - 2.0 * n ** 3 / 3) if m >= n else (2.0 * n * m * m - 2.0 * m ** 3 / 3)
                kp = min(m, n)
                kks.append(kp)
            for st in sites:
                Pl = st["bl"] * st["Dl"]
                zc = st["Dout"] * st["nbr"]
                total += 2.0 * st["bl"] * st["Din"] * st["nbr"] * st["br"] * st["Dr"]
                total += 2.0 * Pl * zc * st["Din"] * st["Dr"]
                if st["y"] > 0:
                    m = kks[st["y"] - 1]
                    total += 2.0 * m * Pl * zc
                    if m > zc:
                        total += 2.0 * m * zc * zc - 2.0 * zc ** 3 / 3
                        m = zc
                    total += 4.0 * m * m * zc + 8.0 * m ** 3 + 2.0 * Pl * zc * st["r"]
    return total


def env_site_bonds(Lx, Ly, D, chi):
    """(left, right) bonds of every site of every environment: top[x] for
    E^u[x] (x = 0..Lx-2), bottom[x] for E^l[x] (x = 1..Lx-1)."""
    eb = env_bonds(Lx, Ly, D, chi)
    top = {0: [(1 if y == 0 else D, 1 if y == Ly - 1 else D) for y in range(Ly)]}
    bot = {Lx - 1: [(1 if y == 0 else D, 1 if y == Ly - 1 else D) for y in range(Ly)]}
    for t in range(1, Lx - 1):
        top[t] = [(st["r"], st["nbr"]) for st in eb[0][t - 1]]
        bot[Lx - 1 - t] = [(st["r"], st["nbr"]) for st in eb[1][t - 1]]
    return top, bot


def strip2_step_flops(Lx, Ly, D, x, y, up, dn, cplx):
    """Flops of one step of a two-row partial contraction at column y of rows
    (x, x+1) with up environment bonds up[y] (or the trivial one), down
    bonds dn[y]: the four products of the step (2mnk each, x4 complex)."""
    cf = 4.0 if cplx else 1.0
    ua, ub = up[y] if up else (1, 1)
    ba, bb = dn[y] if dn else (1, 1)
    uk = D if x > 0 else 1
    Dl = 1 if y == 0 else D
    Dr = 1 if y == Ly - 1 else D
    Dd1 = D
    Dd2 = D if x + 1 < Lx - 1 else 1
    inner = Dl * Dl * ba
    f = 2.0 * inner * uk * ub * ua
    f += 2.0 * (Dl * ba * ub) * (Dr * Dd1) * (Dl * uk)
    f += 2.0 * (ba * ub * Dr) * (Dr * Dd2) * (Dl * Dd1)
    f += 2.0 * (ub * Dr * Dr) * bb * (ba * Dd2)
    return cf * f


def strip2_flops(Lx, Ly, D, chi, configs, cplx):
    """Flops of the two-row strip kernel over a batch, from its step count:
    per row pair the Ly right-partial steps, the Ly left-partial steps and
    one window per move with a nonzero coefficient (anti-aligned vertical
    pairs: one column, diagonal pairs: two), each step as strip2_step_flops."""
    top, bot = env_site_bonds(Lx, Ly, D, chi)
    total = 0.0
    s = configs.reshape(len(configs), Lx, Ly)
    n = len(configs)
    for x in range(Lx - 1):
        up = top[x - 1] if x > 0 else None
        dn = bot[x + 2] if x + 2 <= Lx - 1 else None
        step = [strip2_step_flops(Lx, Ly, D, x, y, up, dn, cplx) for y in range(Ly)]
        a, b = s[:, x, :], s[:, x + 1, :]
        vert = (a != b)
        d1 = (a[:, :-1] != b[:, 1:])
        d2 = (a[:, 1:] != b[:, :-1])
        total += 2 * n * sum(step)
        for y in range(Ly):
            total += vert[:, y].sum() * step[y]
        for y in range(Ly - 1):
            total += (d1[:, y].sum() + d2[:, y].sum()) * (step[y] + step[y + 1])
    return total


def kernel_source_hash(files):
    """Hash of the sources a kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2503_12557_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_traffic(kernel, samples_per_launch):
    """HBM bytes per launch of the environment or two-row strip kernel from
    the committed rocprofv3 counter runs (FETCH_SIZE + WRITE_SIZE calibrated
    by a copy of known size), scaled to this launch's configurations; None
    when the counters were taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_k_env_dm_10x10_D5_chi25_c64.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if kernel == "env":
        if rec.get("source_hash") != kernel_source_hash(["common.h", "env_dev.h", "mfma.h",
                                                         "env_dm.hip"]):
            return None
        b = rec["bytes_per_launch"]
    else:
        if rec.get("strip2_source_hash") != kernel_source_hash(["common.h", "mfma.h",
                                                                "strip_dev.h", "strip.hip"]):
            return None
        b = rec["strip2_bytes_per_launch"]
    return b * samples_per_launch / rec["samples_per_launch"]


def _sync():
    import torch
    torch.cuda.synchronize()


_T0 = time.perf_counter()


def _log(msg):
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# The oracle on the host's cores: one worker process per core, one BLAS
# thread each, configurations handed out one at a time until the time budget
# is spent.
# ---------------------------------------------------------------------------
_ORC = {}


def _orc_init(theta, Lx, Ly, D, chi, model):
    from threadpoolctl import threadpool_limits
    from oracle import hamiltonian as OH
    from oracle import peps
    _ORC["lim"] = threadpool_limits(limits=1)
    g = peps.Geometry(Lx, Ly, 2, D)
    name, kw = model
    ham = {"j1j2": OH.j1j2, "chiral": OH.csl, "rydberg": OH.rydberg}[name](Lx, Ly, **kw)
    _ORC.update(T=peps.site_tensors(theta, g), g=g, chi=chi, ham=ham, peps=peps)


def _orc_one(cfg):
    P = _ORC["peps"]
    sc = P.SampleContraction(_ORC["T"], _ORC["g"], cfg, _ORC["chi"])
    sc.local_energy(_ORC["ham"])
    sc.logderiv_compact()
    return 1


def cpu_baseline(theta, Lx, Ly, D, chi, model, configs, seconds=20.0):
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    workers = max(1, min(cores, 16))
    ctxm = mp.get_context("fork")
    done = 0
    with ctxm.Pool(workers, initializer=_orc_init,
                   initargs=(theta, Lx, Ly, D, chi, model)) as pool:
        # warm the workers (imports, tensors) outside the timed region
        pool.map(_orc_one, [configs[i % len(configs)] for i in range(workers)])
        t0 = time.perf_counter()
        it = pool.imap_unordered(_orc_one, [configs[i % len(configs)] for i in range(100000)])
        for _ in it:
            done += 1
            if time.perf_counter() - t0 > seconds:
                break
        dt = time.perf_counter() - t0
        pool.terminate()
    return {"value": done / dt, "unit": "samples/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} configurations of the timed batch (psi + E_loc + O, FP64 / "
                      f"complex128 numpy oracle, canonical truncation, one BLAS thread per "
                      f"worker, {workers} worker processes) in {dt:.1f} s"}


def ess_comparison(Context, theta, Lx, Ly, D, chi, ham, made_steps, model="J1-J2 J2/J1=0.5",
                   chains=256, T=64, burn=16, data_chains=1024, data_per=64, data_burn=16,
                   compression="canonical"):
    """Effective samples per second of the energy series: local exchange
    Metropolis against independence MH with the learned proposal (trained on
    data_chains x data_per configurations of the local sampler). Both arms
    start from burned-in states: the IMH chains from the local sampler's
    states after `burn` sweeps, the local chains run their own `burn`
    burn-in sweeps, whose separately timed cost is subtracted. E_loc of the
    recorded states is evaluated untimed."""
    import torch

    from paper_2503_12557_amd import analysis
    from paper_2503_12557_amd.binding import Made, run_imh
    N = Lx * Ly
    ctx = Context(Lx, Ly, D, chi, "f32")
    ctx.set_hamiltonian(ham)
    if compression != "canonical":
        ctx.set_compression(compression)
    init, _ = ctx.sample(theta, "exchange", n_chains=chains, per_chain=1, burn_in=burn, seed=21)
    _sync()
    t0 = time.perf_counter()
    ctx.sample(theta, "exchange", n_chains=chains, per_chain=1, burn_in=burn, seed=25)
    _sync()
    t_burn = (time.perf_counter() - t0) * burn / (burn + 1.0)
    t0 = time.perf_counter()
    mh, acc_mh = ctx.sample(theta, "exchange", n_chains=chains, per_chain=T, burn_in=burn,
                            seed=22)
    _sync()
    t_mh = time.perf_counter() - t0 - t_burn
    _log(f"local chains: {t_mh:.1f} s")
    e_mh = ctx.evaluate(theta, mh, want_o=False)[1][:, 0].view(chains, T).cpu().numpy()
    _log("local chains evaluated")
    t0 = time.perf_counter()
    data, _ = ctx.sample(theta, "exchange", n_chains=data_chains, per_chain=data_per,
                         burn_in=data_burn, seed=23)
    _sync()
    t_data = time.perf_counter() - t0
    _log(f"{data.shape[0]} training configurations: {t_data:.1f} s")
    made = Made(N, 256, N // 2, bf16=True)
    params = torch.tensor(0.01 * np.random.default_rng(7).standard_normal(made.n_params),
                          dtype=torch.float32, device=theta.device)
    t0 = time.perf_counter()
    losses = made.train(params, data, steps=made_steps, batch=1024, lr=1e-3, seed=0)
    _sync()
    t_train = time.perf_counter() - t0
    ls = losses.cpu().numpy()
    t0 = time.perf_counter()
    _, hist, acc = run_imh(ctx, theta, made, params, n_chains=chains, n_steps=T, seed=24,
                           record=True, init=init)
    _sync()
    t_imh = time.perf_counter() - t0
    _log(f"independence chains: {t_imh:.1f} s")
    states = hist.permute(1, 0, 2).reshape(chains * T, N).contiguous()
    e_imh = ctx.evaluate(theta, states, want_o=False)[1][:, 0].view(chains, T).cpu().numpy()
    tau_mh, tau_imh = analysis.tau_int_ranked(e_mh), analysis.tau_int_ranked(e_imh)
    raw_mh, raw_imh = analysis.tau_int(e_mh), analysis.tau_int(e_imh)
    hist_np = hist.cpu().numpy()
    repeat = float((hist_np[1:] == hist_np[:-1]).all(axis=2).mean())
    sweeps_moves = (2 * Ly - 1) * Lx
    return {
        "workload": f"{Lx}x{Ly} D={D} chi={chi} {model}, {chains} chains x {T} "
                    f"steps, energy series, both arms after {burn} burn-in sweeps, FP32, "
                    f"{compression} truncation",
        "tau_int_estimator": "Sokal window on rank-normalised E_loc (normal scores of pooled "
                             "ranks); tau_int_plain: same window on raw E_loc",
        "local_mh": {"tau_int": tau_mh, "tau_int_plain": raw_mh, "ess": chains * T / tau_mh,
                     "seconds": t_mh, "burn_in_seconds_subtracted": t_burn,
                     "ess_per_s": chains * T / tau_mh / t_mh,
                     "acceptance_per_move": float(acc_mh.sum().item()) / (chains * (T + burn) * sweeps_moves)},
        "imh_learned": {"tau_int": tau_imh, "tau_int_plain": raw_imh,
                        "ess": chains * T / tau_imh, "seconds": t_imh,
                        "ess_per_s": chains * T / tau_imh / t_imh,
                        "acceptance": float(acc.sum().item()) / (chains * T),
                        "repeated_state_fraction": repeat},
        "made": {"N": N, "hidden": 256, "bf16_weights": True, "train_configs": int(data.shape[0]),
                 "adam_steps": made_steps, "train_s": t_train, "data_s": t_data,
                 "loss_first": float(ls[:20].mean()), "loss_last": float(ls[-20:].mean())},
    }


def _err_block(e_lo, e_hi, lp_lo, lp_hi):
    """Relative error of the mean energy and per-configuration quantiles."""
    import torch
    rel = abs(e_lo.mean().item() - e_hi.mean().item()) / abs(e_hi.mean().item())
    per = ((e_lo - e_hi).abs() / e_hi.abs().clamp_min(1.0)).cpu().numpy()
    dpsi = (lp_lo[:, 0] - lp_hi[:, 0]).abs().cpu().numpy()
    return rel, {"median": float(np.median(per)), "p90": float(np.quantile(per, 0.9)),
                 "p99": float(np.quantile(per, 0.99)), "max": float(per.max())}, \
        {"median": float(np.median(dpsi)), "p99": float(np.quantile(dpsi, 0.99))}


def cutoff_workload(Context, hamiltonians):
    """Throughput of the density-matrix environments with a maximal truncated
    weight per bond (kept bonds carried through the contractions) against
    fixed chi: 10x10 D=5 chi=25 J1-J2, real N(0.5,1) tensors (seed 4), FP32,
    1024 uniform S_z = 0 configurations; ln Psi change against fixed chi."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    th = torch.from_numpy(synth.theta(10, 10, 2, 5, seed=4, mu=0.5)).to(dev)
    sm = torch.from_numpy(synth.sz0_configs(100, 1024, seed=5)).to(dev)
    out, base = {}, None
    for cut in (0.0, 1e-4):
        ctx = Context(10, 10, 5, 25, "f32")
        ctx.set_hamiltonian(hamiltonians.j1j2(10, 10, 1.0, 0.5))
        ctx.set_compression("densmat")
        if cut:
            ctx.set_truncation(cut)
        o = ctx.evaluate(th, sm)
        _sync()
        ctx.profile(True)
        ctx.profile_read(reset=True)
        t0 = time.perf_counter()
        ctx.evaluate(th, sm, out=o)
        _sync()
        dt = time.perf_counter() - t0
        pr = ctx.profile_read(reset=True)
        lp = o[0][:, 0].double().cpu().numpy()
        base = lp if base is None else base
        out[f"cutoff_{cut:g}"] = {"samples_per_s": round(1024 / dt, 1),
                                  "env_ms": round(pr["env"][0], 2),
                                  "ln_psi_change_median": float(np.median(np.abs(lp - base)))}
    out["workload"] = ("10x10 D=5 chi=25 J1-J2, real N(0.5,1) tensors seed 4, FP32, density-matrix "
                       "truncation, 1024 uniform S_z=0 configurations")
    return out


def side_workload(Context, ham, Lx, Ly, D, chi, n, seed, mu, kind, dtypes, ref="f64",
                  compression="canonical"):
    """Throughput and energy error of reduced-precision modes on one of the
    real-tensor workloads (samples from the library's FP64 sampler)."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    th = torch.from_numpy(synth.theta(Lx, Ly, 2, D, seed=seed, mu=mu)).to(dev)
    c64 = Context(Lx, Ly, D, chi, ref)
    c64.set_hamiltonian(ham)
    chains = min(n, 1024)
    t0 = time.perf_counter()
    sm, _ = c64.sample(th, kind, n_chains=chains, per_chain=(n + chains - 1) // chains,
                       burn_in=8, seed=seed + 10)
    _sync()
    t_s = time.perf_counter() - t0
    sm = sm[:n].contiguous()
    out = {"workload": f"{Lx}x{Ly} d=2 D={D} chi={chi}, N({mu},1) tensors seed {seed}, {n} "
                       f"configurations ({kind} Metropolis, FP64, burn-in 8)",
           "sampling_s": round(t_s, 2)}
    res = {}
    for dt in [ref] + list(dtypes):
        ctx = c64 if dt == ref else Context(Lx, Ly, D, chi, dt)
        if ctx is not c64:
            ctx.set_hamiltonian(ham)
        if compression != "canonical":
            ctx.set_compression(compression)
        o = ctx.evaluate(th, sm)
        _sync()
        t0 = time.perf_counter()
        ctx.evaluate(th, sm, out=o)
        _sync()
        res[dt] = (o, time.perf_counter() - t0)
    lp_hi, e_hi = res[ref][0][0], res[ref][0][1][:, 0].double()
    out[f"{ref}_samples_per_s"] = round(n / res[ref][1], 2)
    out["energy_mean_" + ref] = e_hi.mean().item()
    for dt in dtypes:
        o, t = res[dt]
        rel, per, dpsi = _err_block(o[1][:, 0].double(), e_hi, o[0], lp_hi)
        out[dt] = {"samples_per_s": round(n / t, 2), "energy_rel_err": rel,
                   "eloc_rel_err_per_config": per, "ln_psi_abs_err_per_config": dpsi}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1024,
                    help="configurations per step (steps cycle through the set)")
    ap.add_argument("--configs", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side workloads and the learned-proposal comparison")
    ap.add_argument("--made-steps", type=int, default=2000)
    ap.add_argument("--proposal-16x16", action="store_true",
                    help="only the learned-proposal comparison on the 16x16 D=6 chi=36 "
                         "Heisenberg lattice (minutes; reduced chain and training sizes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2503_12557_amd import Context, hamiltonians

    dev = torch.device("cuda:0")
    if args.proposal_16x16:
        # 16x16 D=6 chi=36 Heisenberg, real N(0,1) tensors seed 6: the
        # density-matrix sampler needs about 2.5 s per sweep of 256 chains
        # here, so the arms take 256 chains x 32 steps and the proposal
        # trains on 512 chains x 16 configurations
        th5 = torch.from_numpy(synth.theta(16, 16, 2, 6, seed=6)).to(dev)
        out = ess_comparison(Context, th5, 16, 16, 6, 36, hamiltonians.j1j2(16, 16, 1.0, 0.0),
                             args.made_steps, model="Heisenberg", chains=256, T=32, burn=8,
                             data_chains=512, data_per=16, data_burn=8, compression="densmat")
        print(json.dumps({"metric": "ESS/s of the energy series (learned proposal vs local MH)",
                          "learned_proposal_16x16_D6_chi36": out}))
        return
    Lx, Ly, D, chi = 10, 10, 5, 25
    model = ("chiral", dict(J1=1.0, J2=0.5, Jchi=0.2))
    ham = hamiltonians.chiral(Lx, Ly, J1=1.0, J2=0.5, Jchi=0.2)
    theta_np = synth.theta(Lx, Ly, 2, D, seed=4, cplx=True)
    theta = torch.from_numpy(theta_np).to(dev)
    nconf = args.configs

    ref = Context(Lx, Ly, D, chi, "c128")
    ref.set_hamiltonian(ham)
    ref.set_compression("densmat")
    # the timed set: configurations drawn by the library's exchange
    # Metropolis sampler in complex128 (density-matrix environments), up to
    # 1024 chains, one sweep between samples after 8 burn-in sweeps
    chains = min(1024, nconf)
    per_chain = max(1, nconf // chains)
    nconf = chains * per_chain
    t0 = time.perf_counter()
    samples, _acc = ref.sample(theta, "exchange", n_chains=chains, per_chain=per_chain, burn_in=8,
                               thin=1, seed=1)
    _sync()
    t_smp = time.perf_counter() - t0
    sampler_used = (f"exchange Metropolis, complex128, {chains} chains x {per_chain} samples, "
                    f"burn-in 8, one sweep between samples (seed 1)")
    _log(f"sampled {nconf} configurations in {t_smp:.1f} s")
    # complex128 reference on the whole set (untimed; its rate reported)
    out128 = ref.evaluate(theta, samples)
    _sync()
    t0 = time.perf_counter()
    ref.evaluate(theta, samples, out=out128)
    _sync()
    t128 = time.perf_counter() - t0
    _log(f"complex128 reference: {nconf / t128:.1f} samples/s")

    # a plain elementwise kernel of known traffic (256 MiB read + 256 MiB
    # written): its FETCH_SIZE / WRITE_SIZE under rocprofv3 --pmc calibrate
    # the traffic counters of the other kernels
    calib = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    torch.mul(calib, 2.0)
    del calib
    ctx = Context(Lx, Ly, D, chi, "c64")
    ctx.set_hamiltonian(ham)
    ctx.set_compression("densmat")
    full = ctx.evaluate(theta, samples)   # every configuration once, for the error
    _sync()
    B = min(args.batch, nconf)
    chunks = [samples[i:i + B].contiguous() for i in range(0, nconf - B + 1, B)]
    outs = [ctx.evaluate(theta, chunks[0]) for _ in range(2)]
    for w in range(args.warmup):
        ctx.evaluate(theta, chunks[w % len(chunks)], out=outs[w % 2])
    _sync()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    _sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.evaluate(theta, chunks[k % len(chunks)], out=outs[k % 2])
    _sync()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    _log(f"timed {args.steps} steps: {B * args.steps / dt:.1f} samples/s")

    rel_e, per_e, per_psi = _err_block(full[1][:, 0].double(), out128[1][:, 0],
                                       full[0], out128[0])
    flags = int(torch.bitwise_or(full[3], out128[3]).max().item())
    ms_per_step = dt / args.steps * 1e3
    value = B / (dt / args.steps)

    per_kernel = {k: {"ms_total": round(v[0], 3), "launches": v[1],
                      "ms_avg": round(v[0] / v[1], 4) if v[1] else None}
                  for k, v in prof.items() if v[1]}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_total"])
    # roofline of the dominant kernel: algorithmic flops of one launch over
    # its average duration
    steps_done = args.steps
    mm_s, alu_s = dm_env_flops_per_sample(Lx, Ly, D, chi, True)
    env_launch_samples = B / (per_kernel["env"]["launches"] / steps_done)
    s2_batch = torch.cat([chunks[k % len(chunks)] for k in range(steps_done)]).cpu().numpy()
    s2_flops_total = strip2_flops(Lx, Ly, D, chi, s2_batch, True)
    env_s = per_kernel["env"]["ms_avg"] * 1e-3
    rooflines = {
        "env": {"kernel": "k_env_dm", "bound": "mfma",
                "achieved": CANONICAL_ENV_FLOPS_10x10_D5_CHI25 * env_launch_samples / env_s / 1e12,
                "peak": PEAK["fp32_matrix_tflops"], "unit": "TFLOP/s",
                "algorithmic_flops_per_sample": CANONICAL_ENV_FLOPS_10x10_D5_CHI25,
                "algorithmic_flops_model": "canonical QR -> SVD environment build (GEMM 7.4 + "
                                           "Householder QR 5.3 + SVD 12.2 GF per sample)",
                "achieved_density_matrix_mfma_flops": mm_s * env_launch_samples / env_s / 1e12,
                "density_matrix_mfma_flops_per_sample": mm_s,
                "density_matrix_alu_flops_per_sample": alu_s,
                "samples_per_launch": env_launch_samples,
                "avg_launch_ms": per_kernel["env"]["ms_avg"]},
    }
    if "strip2" in per_kernel:
        s2 = per_kernel["strip2"]
        rooflines["strip2"] = {
            "kernel": "k_strip2", "bound": "mfma",
            "achieved": s2_flops_total / s2["launches"] / (s2["ms_avg"] * 1e-3) / 1e12,
            "peak": PEAK["fp32_matrix_tflops"], "unit": "TFLOP/s",
            "algorithmic_flops_per_launch": s2_flops_total / s2["launches"],
            "samples_per_launch": B * steps_done / s2["launches"],
            "avg_launch_ms": s2["ms_avg"]}
    for r in rooflines.values():
        r["achieved"] = round(r["achieved"], 3)
        if "achieved_density_matrix_mfma_flops" in r:
            r["achieved_density_matrix_mfma_flops"] = round(r["achieved_density_matrix_mfma_flops"], 3)
        r["frac"] = round(r["achieved"] / r["peak"], 5)
    for key, r in rooflines.items():
        r["traffic"] = kernel_traffic(key, r["samples_per_launch"])
    dom_key = dom if dom in rooflines else "env"
    roofline = dict(rooflines[dom_key])
    roofline["dominant_kernel_by_time"] = dom

    res = {
        "metric": "samples/s (psi+E_loc+O)",
        "value": round(value, 2),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "10x10 open lattice d=2 D=5 chi=25, complex tensors "
                               "N(0,1)+iN(0,1) seed 4, chiral spin liquid J1=1 J2=0.5 "
                               f"Jchi=0.2, {nconf} configurations",
                   "samples": sampler_used, "global_batch": B, "configurations": nconf,
                   "truncation": "density-matrix (Gram and density products on MFMA)"},
        "sampling_s_c128": round(t_smp, 2),
        "energy_rel_err_vs_c128": rel_e,
        "eloc_rel_err_per_config": per_e,
        "ln_psi_abs_err_per_config": per_psi,
        "energy_mean_c128": out128[1][:, 0].mean().item(),
        "value_c128": round(nconf / t128, 2),
        "flags_or": flags,
        "per_kernel": per_kernel,
        "roofline": roofline,
        "rooflines": rooflines,
    }
    # minSR step on all configurations (n = 8192, complex parameters, FP64
    # Gram and solve) from the complex64 log-derivatives
    O, el = full[2], full[1]
    ctx.minsr_step(O, samples, el, eps=1e-4, rcond=1e-12)
    _sync()
    t0 = time.perf_counter()
    dth, diag = ctx.minsr_step(O, samples, el, eps=1e-4, rcond=1e-12)
    _sync()
    res["minsr_step_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    _log(f"minSR n={nconf}: {res['minsr_step_ms']} ms")
    res["minsr_n"] = nconf
    res["minsr_diag"] = [float(v) for v in diag.cpu().numpy()]
    # the eigendecomposition solve (alone, and queued behind a certificate
    # that holds) on the first 1024 configurations
    ne = 1024
    tims = {}
    for solver in ("cholesky", "auto", "eigh"):
        ctx.set_minsr_solver(solver)
        ctx.minsr_step(O[:ne], samples[:ne], el[:ne], eps=1e-4, rcond=1e-12)
        _sync()
        t0 = time.perf_counter()
        ctx.minsr_step(O[:ne], samples[:ne], el[:ne], eps=1e-4, rcond=1e-12)
        _sync()
        tims[solver] = round((time.perf_counter() - t0) * 1e3, 2)
    ctx.set_minsr_solver("cholesky")
    res["minsr_solvers_ms_n1024"] = tims
    _log(f"minSR solvers at n={ne}: {tims}")
    # one optimisation step end to end (complex64, density-matrix
    # environments): 1024 chains x 1 sample after 8 burn-in sweeps, the
    # evaluation, minSR and the update of theta
    th_step = theta.clone()
    t0 = time.perf_counter()
    ctx.vmc_step(th_step, 1e-3, "exchange", n_chains=1024, per_chain=1, burn_in=8, seed=3)
    _sync()
    res["vmc_step_s"] = {"seconds": round(time.perf_counter() - t0, 3),
                         "config": "complex64, 1024 chains x 1 sample, 8 burn-in sweeps, "
                                   "evaluation, minSR (n = 1024) and theta update"}
    _log(f"optimisation step: {res['vmc_step_s']['seconds']} s")
    del th_step
    del dth, O, full, out128
    torch.cuda.empty_cache()

    if not args.no_extras:
        res["workload_8x8_D4_chi16"] = side_workload(
            Context, hamiltonians.j1j2(8, 8, 1.0, 0.5), 8, 8, 4, 16, 4096, 2, 0.0, "exchange",
            ["f32", "bf16"])
        res["workload_8x8_D4_chi16_mu05"] = side_workload(
            Context, hamiltonians.j1j2(8, 8, 1.0, 0.5), 8, 8, 4, 16, 4096, 3, 0.5, "exchange",
            ["f32", "bf16"])
        res["workload_12x12_D4_chi16_rydberg"] = side_workload(
            Context, hamiltonians.rydberg(12, 12, Omega=1.0, Delta=3.0, V=1.7 ** 6), 12, 12, 4, 16,
            4096, 5, 0.0, "flip", ["f32", "bf16"])
        # the same with the density-matrix truncation: BF16 products on the
        # bfloat16 matrix cores
        res["workload_12x12_D4_chi16_rydberg_densmat"] = side_workload(
            Context, hamiltonians.rydberg(12, 12, Omega=1.0, Delta=3.0, V=1.7 ** 6), 12, 12, 4, 16,
            4096, 5, 0.0, "flip", ["f32", "bf16"], compression="densmat")
        res["truncated_weight_10x10_D5_chi25"] = cutoff_workload(Context, hamiltonians)
        th2 = torch.from_numpy(synth.theta(8, 8, 2, 4, seed=2)).to(dev)
        _log("side workloads done")
        res["learned_proposal"] = ess_comparison(Context, th2, 8, 8, 4, 16,
                                                 hamiltonians.j1j2(8, 8, 1.0, 0.5),
                                                 args.made_steps)
    _log("extras done")
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(theta_np, Lx, Ly, D, chi, model,
                                           samples[:256].cpu().numpy(), seconds=20.0)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
