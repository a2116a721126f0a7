"""Throughput of the sampled finite-PEPS hot path on one MI355X.

Workload (8x8 open lattice, d=2, D=4, chi=16, 4096 configurations, J1-J2
Heisenberg with J2/J1 = 0.5, tensors i.i.d. N(0,1) from a fixed seed): one
step evaluates ln Psi, the local energies E_loc and the log-derivatives O of
every configuration of the batch (the samples are drawn once, before the
timed region, by the library's Metropolis sampler when it is available).
The timed precision defaults to FP32; the same batch is also evaluated in
FP64 outside the timed region and the relative error of the batch-mean
energy is reported.

Prints one JSON line. Extra fields: the FP64 throughput, the minSR step time,
one step of the optimisation loop (sample + evaluate + minSR + update), the
per-kernel split from HIP events, the roofline of the dominant kernel and
the CPU oracle timed on a bounded sample.
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

PEAK = {  # MI355X published peaks
    "fp32_vector_tflops": 157.3,
    "fp64_vector_tflops": 78.6,
    "hbm_gbs": 8000.0,
}


# ---------------------------------------------------------------------------
# Algorithmic flop model of the environment build (the canonical two-sweep
# truncation: left QR sweep, right SVD sweep), per sample and both sweeps.
#   GEMM m x k x n: 2mnk;  Householder R of m x n (m >= n): 2mn^2 - 2n^3/3;
#   SVD of an m x n block (m <= n) with its m right singular vectors:
#   4 m^2 n + 8 m^3 (Golub and Van Loan's count for the R-SVD).
# ---------------------------------------------------------------------------
def _legs(Lx, Ly, D, x, y):
    return (1 if y == 0 else D, 1 if y == Ly - 1 else D, 1 if x == 0 else D,
            1 if x == Lx - 1 else D)


def env_flops_per_sample(Lx, Ly, D, chi):
    total = 0.0
    for direction in (0, 1):
        # bonds of the first row MPS
        bonds = [_legs(Lx, Ly, D, 0 if direction == 0 else Lx - 1, y)[1] for y in range(Ly)]
        right = [1] + bonds[:-1]  # left bond of site y
        left_b = right
        right_b = bonds
        for t in range(1, Lx - 1):
            x = t if direction == 0 else Lx - 1 - t
            kk = []
            kp = 1
            for y in range(Ly - 1):
                Dl, Dr, Du, Dd = _legs(Lx, Ly, D, x, y)
                Din, Dout = (Du, Dd) if direction == 0 else (Dd, Du)
                Pl, Pr = left_b[y] * Dl, right_b[y] * Dr
                total += Dout * 2.0 * Pl * Pr * Din            # P_k
                if y > 0:
                    total += Dout * 2.0 * kp * Pl * Pr          # R P_k
                m, n = kp * Dout, Pr
                if m >= n:
                    total += 2.0 * m * n * n - 2.0 * n ** 3 / 3
                else:
                    total += 2.0 * n * m * m - 2.0 * m ** 3 / 3
                kp = min(m, n)
                kk.append(kp)
            nbr = 1
            new_left = [1] * Ly
            new_right = [1] * Ly
            for y in range(Ly - 1, -1, -1):
                Dl, Dr, Du, Dd = _legs(Lx, Ly, D, x, y)
                Din, Dout = (Du, Dd) if direction == 0 else (Dd, Du)
                bl, br = left_b[y], right_b[y]
                Pl = bl * Dl
                zc = Dout * nbr
                total += 2.0 * bl * Din * nbr * br * Dr        # T1
                total += 2.0 * Pl * zc * Din * Dr              # Z
                if y > 0:
                    kpr = kk[y - 1]
                    total += 2.0 * kpr * Pl * zc               # C = R Z
                    m = kpr
                    if m > zc:
                        total += 2.0 * m * zc * zc - 2.0 * zc ** 3 / 3
                        m = zc
                    total += 4.0 * m * m * zc + 8.0 * m ** 3   # SVD
                    r = min(chi, kpr, zc)
                    total += 2.0 * Pl * zc * r                 # W
                else:
                    r = 1
                new_left[y] = r
                new_right[y] = nbr
                nbr = r
            left_b, right_b = new_left, new_right
    return total


def kernel_source_hash():
    """Hash of the sources the environment kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("common.h", "env_dev.h", "env.hip"):
        with open(os.path.join(ROOT, "paper_2503_12557_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def env_traffic(dtype):
    """HBM bytes per k_env_sweep launch from the committed rocprofv3 counter
    runs (FETCH_SIZE + WRITE_SIZE, calibrated by a copy of known size), or
    None when they were taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_k_env_sweep.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("dtype") != dtype:
        return None
    return rec.get("bytes_per_launch")


def _sync():
    import torch
    torch.cuda.synchronize()


def cpu_baseline(theta, Lx, Ly, D, chi, configs, seconds=12.0):
    """The FP64 oracle on the host, one process and one BLAS thread, on the
    first configurations of the batch until about `seconds` have passed."""
    from threadpoolctl import threadpool_limits

    from oracle import hamiltonian as OH
    from oracle import peps
    g = peps.Geometry(Lx, Ly, 2, D)
    ham = OH.j1j2(Lx, Ly, 1.0, 0.5)
    T = peps.site_tensors(theta, g)
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while done < len(configs):
            sc = peps.SampleContraction(T, g, configs[done], chi)
            sc.local_energy(ham)
            sc.logderiv_compact()
            done += 1
            if time.perf_counter() - t0 > seconds:
                break
        dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} configurations of the same batch (psi + E_loc + O, FP64 numpy, "
                      f"1 BLAS thread), {dt:.1f} s"}


def ess_comparison(Context, theta, Lx, Ly, D, chi, ham, made_steps):
    """Effective samples per second of the energy series: local exchange
    Metropolis against independence MH with the learned proposal (trained on
    65536 configurations of the local sampler, 2000 Adam steps by default).
    Sampling time only; E_loc of the recorded states is evaluated untimed."""
    import torch

    from paper_2503_12557_amd import analysis
    from paper_2503_12557_amd.binding import Made, run_imh
    N = Lx * Ly
    ctx = Context(Lx, Ly, D, chi, "f32")
    ctx.set_hamiltonian(ham)
    chains, T = 256, 64
    init, _ = ctx.sample(theta, "exchange", n_chains=chains, per_chain=1, burn_in=16, seed=21)
    _sync()
    t0 = time.perf_counter()
    mh, acc_mh = ctx.sample(theta, "exchange", n_chains=chains, per_chain=T, burn_in=0,
                            seed=22)
    _sync()
    t_mh = time.perf_counter() - t0
    e_mh = ctx.evaluate(theta, mh, want_o=False)[1][:, 0].view(chains, T).cpu().numpy()
    t0 = time.perf_counter()
    data, _ = ctx.sample(theta, "exchange", n_chains=1024, per_chain=64, burn_in=16, seed=23)
    _sync()
    t_data = time.perf_counter() - t0
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
    states = hist.permute(1, 0, 2).reshape(chains * T, N).contiguous()
    e_imh = ctx.evaluate(theta, states, want_o=False)[1][:, 0].view(chains, T).cpu().numpy()
    # E_loc of unconverged random tensors is heavy-tailed: ESS from the
    # rank-normalised series, the plain estimate reported beside it
    tau_mh, tau_imh = analysis.tau_int_ranked(e_mh), analysis.tau_int_ranked(e_imh)
    raw_mh, raw_imh = analysis.tau_int(e_mh), analysis.tau_int(e_imh)
    hist_np = hist.cpu().numpy()
    repeat = float((hist_np[1:] == hist_np[:-1]).all(axis=2).mean())
    sweeps_moves = (2 * Ly - 1) * Lx
    return {
        "workload": f"{Lx}x{Ly} D={D} chi={chi} J1-J2 J2/J1=0.5, {chains} chains x {T} "
                    "steps, energy series, stationary starts",
        "tau_int_estimator": "Sokal window on rank-normalised E_loc (normal scores of pooled "
                             "ranks); tau_int_plain: same window on raw E_loc",
        "local_mh": {"tau_int": tau_mh, "tau_int_plain": raw_mh, "ess": chains * T / tau_mh,
                     "seconds": t_mh,
                     "ess_per_s": chains * T / tau_mh / t_mh,
                     "acceptance_per_move": float(acc_mh.sum().item()) / (chains * T * sweeps_moves)},
        "imh_learned": {"tau_int": tau_imh, "tau_int_plain": raw_imh,
                        "ess": chains * T / tau_imh, "seconds": t_imh,
                        "ess_per_s": chains * T / tau_imh / t_imh,
                        "acceptance": float(acc.sum().item()) / (chains * T),
                        "repeated_state_fraction": repeat},
        "made": {"N": N, "hidden": 256, "bf16_weights": True, "train_configs": int(data.shape[0]),
                 "adam_steps": made_steps, "train_s": t_train, "data_s": t_data,
                 "loss_first": float(ls[:20].mean()), "loss_last": float(ls[-20:].mean())},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f64"])
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sampler", default="auto", choices=["auto", "uniform", "metropolis"])
    ap.add_argument("--no-ess", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--made-steps", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2503_12557_amd import Context, hamiltonians
    from paper_2503_12557_amd.binding import PepsError

    Lx, Ly, D, chi, n = 8, 8, 4, 16, args.n
    dev = torch.device("cuda:0")
    theta_np = synth.theta(Lx, Ly, 2, D, seed=2, mu=0.0)
    theta = torch.from_numpy(theta_np).to(dev)
    ham = hamiltonians.j1j2(Lx, Ly, 1.0, 0.5)

    ctx64 = Context(Lx, Ly, D, chi, "f64")
    ctx64.set_hamiltonian(ham)
    sampler_used = "uniform S_z=0 permutations (seed 1)"
    samples = None
    t_sample = None
    if args.sampler in ("auto", "metropolis"):
        try:
            # the FP64 sampler: the batch does not move with FP32 rounding
            ctx_s = ctx64
            chains = min(n, 1024)
            per = (n + chains - 1) // chains
            t0 = time.perf_counter()
            samples, acc = ctx_s.sample(theta, "exchange", n_chains=chains, per_chain=per,
                                        burn_in=8, thin=1, seed=1)
            _sync()
            t_sample = time.perf_counter() - t0
            sampler_used = (f"local exchange Metropolis (library sampler, FP64, {chains} chains x "
                            f"{per}, burn-in 8 sweeps, seed 1)")
        except PepsError:
            if args.sampler == "metropolis":
                raise
            samples = None
    if samples is None:
        samples = torch.from_numpy(synth.sz0_configs(Lx * Ly, n, seed=1)).to(dev)
    samples = samples[:n].contiguous()

    # FP64 reference pass (untimed) on the same batch
    lp64, e64, O64, f64 = ctx64.evaluate(theta, samples)
    _sync()
    t0 = time.perf_counter()
    ctx64.evaluate(theta, samples)
    _sync()
    t64 = time.perf_counter() - t0

    # a plain elementwise kernel of known traffic (256 MiB read + 256 MiB
    # written); its FETCH_SIZE / WRITE_SIZE under rocprofv3 --pmc calibrate
    # the traffic counters
    calib = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    torch.mul(calib, 2.0)
    del calib
    ctx = ctx64 if args.dtype == "f64" else Context(Lx, Ly, D, chi, args.dtype)
    if ctx is not ctx64:
        ctx.set_hamiltonian(ham)
    out = ctx.evaluate(theta, samples)
    for _ in range(args.warmup):
        ctx.evaluate(theta, samples, out=out)
    _sync()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.evaluate(theta, samples, out=out)
    _sync()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    lp, el, O, fl = out
    e_lo = el[:, 0].double().mean().item()
    e_hi = e64[:, 0].mean().item()
    rel_e = abs(e_lo - e_hi) / abs(e_hi)
    # per-configuration errors: the batch mean of random tensors is carried
    # by a few near-zero amplitudes with huge E_loc, so report quantiles too
    per_e = ((el[:, 0].double() - e64[:, 0]).abs() / e64[:, 0].abs().clamp_min(1.0)).cpu().numpy()
    per_psi = (lp[:, 0] - lp64[:, 0]).abs().cpu().numpy()
    flags = int(torch.bitwise_or(fl, f64).max().item())

    # minSR step on the batch (FP64 solve), timed separately
    ctx.minsr_step(O, samples, el, eps=1e-4, rcond=1e-12)
    _sync()
    t0 = time.perf_counter()
    dth, diag = ctx.minsr_step(O, samples, el, eps=1e-4, rcond=1e-12)
    _sync()
    t_minsr = time.perf_counter() - t0

    ms_per_step = dt / args.steps * 1e3
    value = n / (dt / args.steps)
    per_kernel = {k: {"ms_total": round(v[0], 3), "launches": v[1],
                      "ms_avg": round(v[0] / v[1], 4) if v[1] else None}
                  for k, v in prof.items() if v[1]}
    # dominant kernel and its roofline
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_total"])
    env_avg_ms = per_kernel["env"]["ms_avg"]
    # samples one launch processes: the batch is split into equal chunks
    env_launches_per_step = per_kernel["env"]["launches"] / args.steps
    samples_per_launch = n / env_launches_per_step
    env_flops = env_flops_per_sample(Lx, Ly, D, chi) * samples_per_launch
    peak = PEAK["fp64_vector_tflops"] if args.dtype == "f64" else PEAK["fp32_vector_tflops"]
    achieved = env_flops / (env_avg_ms * 1e-3) / 1e12
    roofline = {"kernel": "k_env_sweep", "bound": "alu", "achieved": round(achieved, 3),
                "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 5),
                "traffic": env_traffic(args.dtype),
                "algorithmic_flops_per_launch": env_flops,
                "samples_per_launch": samples_per_launch,
                "avg_launch_ms": env_avg_ms, "dominant_kernel_by_time": dom}

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
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "8x8 open lattice d=2 D=4 chi=16, J1-J2 J2/J1=0.5, "
                               f"{n} configurations, tensors N(0,1) seed 2",
                   "samples": sampler_used, "global_batch": n},
        "energy_rel_err_vs_f64": rel_e,
        "eloc_rel_err_per_config": {"median": float(np.median(per_e)),
                                    "p99": float(np.quantile(per_e, 0.99)),
                                    "max": float(per_e.max())},
        "ln_psi_abs_err_per_config": {"median": float(np.median(per_psi)),
                                      "p99": float(np.quantile(per_psi, 0.99))},
        "energy_mean_f64": e_hi,
        "value_f64": round(n / t64, 2),
        "minsr_step_ms": round(t_minsr * 1e3, 2),
        "sampling_s": round(t_sample, 2) if t_sample is not None else None,
        "minsr_diag": [float(v) for v in diag.cpu().numpy()],
        "flags_or": flags,
        "per_kernel": per_kernel,
        "roofline": roofline,
    }
    # one step of the optimisation loop on the same workload, in the bench's
    # compute dtype: sample (1024 chains x 4, burn-in 8) + evaluate + minSR +
    # update, from a copy of theta
    th_opt = theta.clone()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    _sync()
    t0 = time.perf_counter()
    ctx.vmc_step(th_opt, 0.05, n_chains=1024, per_chain=max(1, n // 1024), burn_in=8, seed=9)
    _sync()
    t_vmc = time.perf_counter() - t0
    pv = ctx.profile_read(reset=True)
    ctx.profile(False)
    res["optimisation_step"] = {
        "seconds": round(t_vmc, 3), "samples": 1024 * max(1, n // 1024),
        "sampler": "local exchange Metropolis, 1024 chains, burn-in 8 sweeps",
        "ms_by_kernel_kind": {k: round(v[0], 2) for k, v in pv.items() if v[1]}}
    del th_opt
    # the same evaluation with a maximal truncated weight of 1e-4 per bond
    # (the paper's cutoff) inside chi = 16, and the relative contraction
    # error Delta psi against the fixed chi = 16 amplitudes
    ctx.set_truncation(1e-4)
    outc = ctx.evaluate(theta, samples)
    _sync()
    t0 = time.perf_counter()
    ctx.evaluate(theta, samples, out=outc)
    _sync()
    t_cut = time.perf_counter() - t0
    ctx.set_truncation(0.0)
    dpsi = (torch.exp(outc[0][:, 0] - lp[:, 0]) - 1).abs().cpu().numpy()
    res["truncated_weight_1e-4"] = {
        "samples_per_s": round(n / t_cut, 2),
        "delta_psi_median": float(np.median(dpsi)), "delta_psi_p99": float(np.quantile(dpsi, 0.99)),
        "energy_mean": float(outc[1][:, 0].double().mean().item())}
    # direct sampler (independent draws, importance weights) on the same
    # workload: 1024 draws, chi_d = D, in the bench's compute dtype
    nd = min(n, 1024)
    ctx.direct_sample(theta, 64, D, seed=12, want_logw=False)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    _sync()
    t0 = time.perf_counter()
    sd, lpd, lwd, fld = ctx.direct_sample(theta, nd, D, seed=13)
    _sync()
    t_dir = time.perf_counter() - t0
    pdir = ctx.profile_read(reset=True)
    ctx.profile(False)
    # the same draws reusing the double-layer environments just built
    _sync()
    t0 = time.perf_counter()
    ctx.direct_sample(theta, nd, D, seed=13, refresh=False)
    _sync()
    t_reuse = time.perf_counter() - t0
    wd = torch.exp(lwd - lwd.max())
    ess = (wd.sum() ** 2 / (wd * wd).sum()).item()
    # the reweighted energy of the direct draws (self-normalised importance
    # sampling) beside the Metropolis batch mean
    eld = ctx.local_energy(theta, sd)[:, 0].double()
    e_dir = ((wd * eld).sum() / wd.sum()).item()
    res["direct_sampler"] = {
        "samples": nd, "chi_double": D, "seconds": round(t_dir, 3),
        "samples_per_s": round(nd / t_dir, 2), "importance_ess": round(ess, 2),
        "ess_per_s": round(ess / t_dir, 2), "flags_or": int(fld.max().item()),
        "reweighted_energy": e_dir, "metropolis_energy_fp64": e_hi,
        "seconds_reusing_double_layer": round(t_reuse, 3),
        "samples_per_s_reusing_double_layer": round(nd / t_reuse, 2),
        "ms_by_kernel_kind": {k: round(v[0], 2) for k, v in pdir.items() if v[1]}}
    # strict local energy (every amplitude at the one cut) on the first 64
    # configurations of the batch, in the bench's compute dtype
    ks = min(n, 64)
    sk = samples[:ks].contiguous()
    es = ctx.local_energy_strict(theta, sk)
    _sync()
    t0 = time.perf_counter()
    es = ctx.local_energy_strict(theta, sk)
    _sync()
    t_strict = time.perf_counter() - t0
    res["strict_local_energy"] = {
        "samples": ks, "seconds": round(t_strict, 4),
        "samples_per_s": round(ks / t_strict, 2),
        "mean_re": float(es[:, 0].mean().item()),
        "strip_mean_re_same_samples": float(el[:ks, 0].double().mean().item())}
    # energy error on the mu = 0.5 tensors (positive mean, less cancellation)
    th5 = torch.from_numpy(synth.theta(Lx, Ly, 2, D, seed=3, mu=0.5)).to(dev)
    ctx_s5 = Context(Lx, Ly, D, chi, "f32")
    s5, _ = ctx_s5.sample(th5, "exchange", n_chains=1024, per_chain=1, burn_in=8, seed=5)
    e5_hi = ctx64.evaluate(th5, s5, want_o=False)[1][:, 0].mean().item()
    e5_lo = ctx.evaluate(th5, s5, want_o=False)[1][:, 0].double().mean().item()
    res["energy_rel_err_vs_f64_mu0.5"] = abs(e5_lo - e5_hi) / abs(e5_hi)
    res["energy_mean_f64_mu0.5"] = e5_hi
    if not args.no_ess:
        res["learned_proposal"] = ess_comparison(Context, theta, Lx, Ly, D, chi, ham,
                                                 args.made_steps)
    if not args.no_cpu:
        # a bounded sample of the batch: up to 512 configurations or ~15 s
        k = min(n, 512)
        res["cpu_baseline"] = cpu_baseline(theta_np, Lx, Ly, D, chi, samples[:k].cpu().numpy(),
                                           seconds=15.0)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
