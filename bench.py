#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.  Prints ONE JSON line.

Default workload (the headline): 2D TFIM 10x10 (N = 100, J = 1, h = 3.04), RBM
alpha = 2 (M = 200), 4096 chains, 100 burn-in + 1000 measured sweeps.  One step
is one pass of the whole path:
  downcast of the FP64 master -> chain init + MH sampling -> local energies of
  all 4.096e6 samples -> FP64 energy statistics -> log-derivatives of the last
  sweep's samples -> FP64 forces -> centred Gram matrix in sample space.
`value` = MH proposals per second of whole-step time with the sampling copy in
BF16, inputs resident in HBM.  The same step with an FP32 sampling copy is
timed beside it, and the energy difference between the two is reported with
its paired error bar.  The CPU oracle is timed on a bounded sample of the same
workload on the host cores.

Other workloads (--workload):
  heis10   2D Heisenberg 10x10, Marshall sign, FFNN 100->400->200, exchange
           moves, 16384 chains x (50 + 500) sweeps; sampling and local
           energies in the chosen dtype, O_k of the last sweep, forces.
  uneven   32 uneven 2D TFIM instances (L in 6..16, h ~ U[2,4], alpha in
           {1,2,4}), 1024 chains x (20 + 200) sweeps each: one persistent
           launch, compared with 32 separate launches (plain and graph-replayed).
  heis20   2D Heisenberg 20x20, Marshall sign, FFNN 400->1600->800->400,
           65536 chains, exchange moves through the batched-GEMM path; a step
           is --sweeps sweeps (default 1; the full 220-sweep run is ~10^3 times
           longer), local energies of 1024 of the last sweep's samples and the
           sample-space Gram matrix T of --gram-samples of them (default 4096)
           from the per-layer factors of O (P = 2,242,800 per sample, never
           held whole); --gram-chunked times the column-block path instead.
  noise    noisy-RBM study on the 16-site TFIM chain: relative bias of
           <sigma^x> and <Pi_even> against the noise sigma (exact by
           enumeration and from 2^18 samples) beside the KL and average
           bounds, and the acceptance rate against sigma for RBMs trained
           here at h/J = 0.5, 1, 5.
  rescnn   residual convolutional network: sampling time against samples and
           filters per format on the 4x4 lattice (four blocks), and one sweep
           of 4096 chains on the 10x10 lattice with 16 filters.
  crbm     complex-parameter RBM on the 10x10 TFIM (M = 200), 4096 chains x
           (10 + 100) sweeps, beside the real RBM sampler at the same shape;
           complex local energies of the emitted samples.
  srstudy  SR regularisation study (App. I.2): an RBM on the 16-site critical TFIM
           chain trained with shifts 1e-3 and 1e-1, FP32 / BF16 sampling / BF16
           local energies; energy error against the exact ground energy and the
           condition number of S + shift along the optimisation.
  peaks    achievable rates of the device (FP32 FMA, log2/exp2, matrix cores in
           BF16/FP32/FP64, HBM read and copy) next to the published peaks.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
PEAK_FP8_MFMA_TFLOPS = 5000.0
# v_log_f32 / v_exp_f32 rate measured on this device (bench.py --workload peaks)
MEASURED_EXP2_LOG2_PER_S = 1.30e13
METRIC = "MH proposals/s + E_loc samples/s, BF16 vs FP32 on 1 GPU, at stated dE vs FP64"


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tfim10", choices=["tfim10", "heis10", "uneven", "heis20", "noise", "rescnn", "crbm", "peaks", "srstudy"])
    ap.add_argument("--sweeps", type=int, default=0, help="heis20: measured sweeps per step (default 1)")
    ap.add_argument("--gram-samples", type=int, default=4096, help="heis20: samples in T (0 = skip)")
    ap.add_argument("--gram-chunked", action="store_true", help="heis20: T by parameter column blocks")
    ap.add_argument("--dtype", default="bf16", choices=["bf16", "f16", "f32", "e4m3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 comparison step")
    ap.add_argument("--headline-only", action="store_true",
                    help="tfim10: skip the one-step runs of the dense-network and uneven-batch workloads")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per chain of the RBM sampler (0 = library default)")
    ap.add_argument("--refresh", type=int, default=4, help="sweeps between full recomputes of theta = W s + b")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device three times (HBM counter calibration)")
    return ap.parse_args()


def kernel_traffic(kernel, profile, instance=None):
    """HBM bytes per launch of `kernel` (the row naming `instance`, a template instantiation, when given)
    from a committed counter summary, or None when the kernel's sources have changed since the counters
    were taken (the summary records their hash)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    want, files, nbytes = None, [], None
    for line in open(path):
        f = line.split()
        if len(f) >= 4 and f[0] == "source_sha256" and f[1] == kernel:
            want, files = f[2], f[3].split(",")
        elif f and not line.startswith("#") and (instance or kernel) in line and len(f) >= 4:
            nbytes = float(f[-1])
    if want is None or nbytes is None:
        return None
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(ROOT, "paper_2601_20782_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return nbytes if h.hexdigest() == want else None


def _events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


class Step:
    """Buffers and phases of one hot-path pass for one workload and sampling dtype."""

    phase_names = ["downcast", "sample", "local_energy", "stats", "logpsi_grad", "forces", "gram"]

    def __init__(self, nqs, torch, wl, params, dtype, lanes=0, refresh=1, eloc_dtype="f32", with_gram=True):
        self.nqs, self.torch, self.wl, self.dtype = nqs, torch, wl, dtype
        self.eloc_dtype, self.with_gram = eloc_dtype, with_gram
        dev = torch.device("cuda:0")
        self.N = N = wl.model.n_visible
        self.C, self.S, self.B = wl.n_chains, wl.n_sweeps, wl.n_burnin
        self.model = nqs.Model.from_workload(wl, params)
        self.master = torch.from_numpy(np.asarray(params, dtype=np.float64)).to(dev)
        self.ham = nqs.Hamiltonian.from_workload(wl.ham)
        self.cfg = nqs.SampleConfig(n_chains=self.C, n_sweeps=self.S, n_burnin=self.B, seed=wl.seed, dtype=dtype,
                                    lanes_per_chain=lanes, refresh_sweeps=refresh, move=wl.move)
        self.state = torch.empty(self.C, N, dtype=torch.int8, device=dev)
        self.samples = torch.empty(self.S, self.C, N, dtype=torch.int8, device=dev)
        self.acc = torch.empty(self.C, dtype=torch.int64, device=dev)
        self.eloc = torch.empty(self.S * self.C, dtype=torch.float64, device=dev)
        self.stats = torch.empty(4, dtype=torch.float64, device=dev)
        self.P = self.model.n_params
        self.O = torch.empty(self.C, self.P, dtype=torch.float32, device=dev)
        self.F = torch.empty(self.P, dtype=torch.float64, device=dev)
        self.T = torch.empty(self.C, self.C, dtype=torch.float32, device=dev) if with_gram else None

    def run(self, ev=None):
        nqs = self.nqs
        k = 0

        def mark():
            nonlocal k
            if ev is not None:
                ev[k].record()
            k += 1

        mark()
        self.model.set_params_device(self.master)          # FP64 master -> sampling copy
        self.model.prepare(self.dtype)
        mark()
        nqs.nqs_sample(self.model, self.cfg, self.state, self.samples, None, self.acc)
        mark()
        nqs.nqs_local_energy(self.model, self.ham, self.samples, self.eloc, self.eloc_dtype)
        mark()
        nqs.nqs_energy_stats(self.eloc, self.C, self.stats)
        mark()
        nqs.nqs_logpsi_grad(self.model, self.samples[self.S - 1], O=self.O)
        mark()
        nqs.nqs_forces(self.O, self.eloc[(self.S - 1) * self.C:], self.F)
        mark()
        if self.with_gram:
            # T = Obar Obar^T / n (sample space) from the factors of O, FP64 matrix cores
            nqs.nqs_sample_gram_factored(self.model, self.samples[self.S - 1], self.T)
        mark()

    def timed(self, steps, warmup):
        """Mean step time in ms (the larger of the event and wall-clock figures) and per-phase means."""
        torch = self.torch
        for _ in range(warmup):
            self.run()
        torch.cuda.synchronize()
        all_ev = [_events(torch, len(self.phase_names) + 1) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            self.run(all_ev[s])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phases = {name: 0.0 for name in self.phase_names}
        step_ms = []
        for ev in all_ev:
            for i, name in enumerate(self.phase_names):
                phases[name] += ev[i].elapsed_time(ev[i + 1]) / steps
            step_ms.append(ev[0].elapsed_time(ev[-1]))
        if not self.with_gram:
            phases.pop("gram")
        return max(float(np.mean(step_ms)), 1e3 * wall / steps), phases


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, params, budget_s=20.0, paired_chains=0, paired_sweeps=0, device_eloc=None):
    """The oracle (FP64, full forward per proposal) on a bounded sample of the workload, on every host
    thread and on one.  With paired_chains > 0 the bounded sample is the first paired_sweeps sweeps of
    paired_chains chains (no burn-in, the workload's seed), and each entry of device_eloc (format ->
    local energies [sweep][chain] of the device's run with the same configuration and seed) is paired
    with the oracle's: the mean FP64-referenced energy difference and its chain-mean standard error."""
    import oracle
    oracle.build()
    om = oracle.model_from_workload(wl, params, "f64")
    threads = oracle.num_threads()
    N = wl.model.n_visible
    if paired_chains:
        chains, sweeps = paired_chains, paired_sweeps
    else:
        # calibrate on a small run, then size the measured runs to the time budget
        c0 = max(threads, 8)
        t = time.perf_counter()
        oracle.sample(om, oracle.make_cfg(c0, 1, 0, move=wl.move, seed=wl.seed))
        per_prop = max(1e-9, (time.perf_counter() - t) / (c0 * N))
        chains = int(max(threads, min(wl.n_chains, (0.6 * budget_s) / (per_prop * N * 2))))
        sweeps = int(max(2, min(8, (0.6 * budget_s) / (per_prop * N * chains))))
    cfg = oracle.make_cfg(chains, sweeps, 0, move=wl.move, seed=wl.seed)
    t = time.perf_counter()
    _, smp, _, _ = oracle.sample(om, cfg)
    ts = time.perf_counter() - t
    props = chains * sweeps * N
    flat = smp.reshape(-1, N)
    if paired_chains:
        n_el = flat.shape[0]
    else:
        t = time.perf_counter()
        oracle.local_energy(om, wl.ham, flat[:threads])
        per_el = max(1e-9, (time.perf_counter() - t) / threads)
        n_el = int(max(threads, min(flat.shape[0], 0.4 * budget_s / per_el)))
    t = time.perf_counter()
    e64 = oracle.local_energy(om, wl.ham, flat[:n_el])
    te = time.perf_counter() - t
    out = {"value": props / ts, "unit": "proposals/s", "cores": threads, "cpu_model": _cpu_model(),
           "kind": "oracle", "eloc_samples_per_s": n_el / te,
           "sample": f"{chains} chains x {sweeps} sweeps ({props} proposals, FP64 full forward each) + "
                     f"local energies of {n_el} samples, {wl.name}"}
    # the same oracle on one thread, on a smaller bounded sample
    c1 = min(chains, 64)
    oracle.set_num_threads(1)
    try:
        t = time.perf_counter()
        _, smp1, _, _ = oracle.sample(om, oracle.make_cfg(c1, 2, 0, move=wl.move, seed=wl.seed))
        t1 = time.perf_counter() - t
        t = time.perf_counter()
        oracle.local_energy(om, wl.ham, smp1.reshape(-1, N)[:c1])
        t1e = time.perf_counter() - t
    finally:
        oracle.set_num_threads(threads)
    out["one_thread"] = {"value": c1 * 2 * N / t1, "unit": "proposals/s", "eloc_samples_per_s": c1 / t1e,
                         "sample": f"{c1} chains x 2 sweeps + local energies of {c1} samples"}
    if device_eloc:
        res = {}
        for fmt, ed in device_eloc.items():
            d = (np.asarray(ed, dtype=np.float64) - e64).reshape(sweeps, chains)
            cm = d.mean(axis=0)
            res[fmt] = {"value": float(d.mean()), "stderr_paired": float(cm.std(ddof=1) / np.sqrt(chains))}
        out["dE_vs_fp64"] = res
        out["dE_vs_fp64_setup"] = (f"{chains} chains x {sweeps} sweeps from the start states, no burn-in, seed "
                                   f"{wl.seed}: the device's local energies (FP32 ratios) of its own samples minus "
                                   f"the oracle's FP64 local energies of its own samples, per (sweep, chain); "
                                   f"chain-mean standard error")
        out["oracle_energy"] = {"mean": float(e64.mean()),
                                "stderr": float(e64.reshape(sweeps, chains).mean(axis=0).std(ddof=1)
                                                / np.sqrt(chains))}
    return out


def _device_short_run(nqs, torch, wl, params, dtype, chains, sweeps, refresh):
    """Local energies [sweep][chain] (FP32 ratios, FP64 sums) of a short device run from the start
    states (no burn-in, the workload's seed), as a host array."""
    dev = torch.device("cuda:0")
    N = wl.model.n_visible
    model = nqs.Model.from_workload(wl, params)
    cfg = nqs.SampleConfig(n_chains=chains, n_sweeps=sweeps, n_burnin=0, seed=wl.seed, dtype=dtype,
                           refresh_sweeps=refresh, move=wl.move)
    state = torch.empty(chains, N, dtype=torch.int8, device=dev)
    samples = torch.empty(sweeps, chains, N, dtype=torch.int8, device=dev)
    eloc = torch.empty(sweeps * chains, dtype=torch.float64, device=dev)
    nqs.nqs_sample(model, cfg, state, samples, None, None)
    nqs.nqs_local_energy(model, nqs.Hamiltonian.from_workload(wl.ham), samples, eloc, "f32")
    out = eloc.cpu().numpy()
    model.close()
    return out


def _common(a, wl, props, ms, phases, step, data):
    st = step.stats.cpu().numpy()
    return {
        "metric": METRIC, "value": props / (ms * 1e-3), "unit": "proposals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": a.dtype, "data": data,
        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
        "sampler_proposals_per_s": props / (phases["sample"] * 1e-3),
        "eloc_samples_per_s": wl.n_sweeps * wl.n_chains / (phases["local_energy"] * 1e-3),
        "acceptance": float(step.acc.sum().item()) / props,
        "energy": {"mean": st[0], "stderr": st[2], "var": st[1]},
    }


def _paired(nqs, torch, x, y, n_chains):
    """Mean of the paired local-energy differences x - y and its chain-mean standard error."""
    diff = (x - y).contiguous()
    dstats = torch.empty(4, dtype=torch.float64, device=diff.device)
    nqs.nqs_energy_stats(diff, n_chains, dstats)
    d = dstats.cpu().numpy()
    return {"value": float(d[0]), "stderr_paired": float(d[2])}


def _compare_fp32(a, nqs, torch, wl, params, step, ms, props, eloc_dtype, with_gram, others=()):
    ref = Step(nqs, torch, wl, params, "f32", a.lanes, a.refresh, eloc_dtype="f32", with_gram=with_gram)
    ms32, ph32 = ref.timed(a.steps, a.warmup)
    st32 = ref.stats.cpu().numpy()
    out = {"fp32": {"proposals_per_s": props / (ms32 * 1e-3), "ms_per_step": ms32,
                    "sampler_proposals_per_s": props / (ph32["sample"] * 1e-3),
                    "phases_ms": {k: round(v, 3) for k, v in ph32.items()},
                    "energy": {"mean": st32[0], "stderr": st32[2]}},
           "speedup_vs_fp32": ms32 / ms,
           "dE_vs_fp32": dict(_paired(nqs, torch, step.eloc, ref.eloc, wl.n_chains),
                              note="same seeds; chain-mean standard error of the paired local-energy differences; "
                                   "the FP32 path's accept decisions equal the FP64 oracle's outside near ties")}
    # the other sampling formats, one timed step each, same seeds
    for dt in others:
        if dt == a.dtype:
            continue
        o = Step(nqs, torch, wl, params, dt, a.lanes, a.refresh, eloc_dtype=dt if eloc_dtype != "f32" else "f32",
                 with_gram=with_gram)
        mso, pho = o.timed(a.steps, a.warmup)
        out.setdefault("other_formats", {})[dt] = {
            "ms_per_step": round(mso, 3), "sample_ms": round(pho["sample"], 3),
            "dE_vs_fp32": _paired(nqs, torch, o.eloc, ref.eloc, wl.n_chains)}
        del o
    return out


def _sr_step(nqs, torch, step, shift=1e-2, lr=1e-2):
    """The stochastic-reconfiguration step that would follow the timed step (not part of it): CG solve of
    (T + shift) y = eps - mean eps on the last sweep's samples, then the FP64 parameter update."""
    C, S = step.C, step.S
    y = torch.empty(C, dtype=torch.float64, device="cuda:0")
    master = step.master.clone()
    eps = step.eloc[(S - 1) * C:]
    nqs.nqs_sr_solve(step.T, eps, shift, y, tol=1e-8, max_iter=2000)   # warm the workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, rr = nqs.nqs_sr_solve(step.T, eps, shift, y, tol=1e-8, max_iter=2000)
    t1 = time.perf_counter()
    nqs.nqs_sr_update(step.model, step.samples[S - 1], y, lr, master)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # the same solve preconditioned by a Cholesky factor in a reduced format, refined in FP64
    mixed = {}
    ym = torch.empty_like(y)
    ref = y.abs().max().item()
    for fmt in ("f32", "bf16", "f16"):
        nqs.nqs_sr_solve_mixed(step.T, eps, shift, ym, fmt, tol=1e-8, max_iter=2000)   # warm the workspace
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        mits, mrr, fixed, used = nqs.nqs_sr_solve_mixed(step.T, eps, shift, ym, fmt, tol=1e-8, max_iter=2000)
        t4 = time.perf_counter()
        mixed[fmt] = {"ms": round(1e3 * (t4 - t3), 3), "factor_used": used, "iterations": mits,
                      "rel_residual": mrr, "pivots_replaced": fixed,
                      "max_rel_diff_vs_cg": (ym - y).abs().max().item() / ref}
    return {"samples": C, "shift": shift, "tol": 1e-8, "cg_iterations": its, "rel_residual": rr,
            "solve_ms": round(1e3 * (t1 - t0), 3), "update_ms": round(1e3 * (t2 - t1), 3),
            "mixed_solve": mixed,
            "note": "outside the timed step; T from the step's factored Gram phase"}


def run_tfim10(a, torch, nqs, workloads):
    wl = workloads.cfg2_tfim_10x10()
    params = workloads.params_for(wl)
    N, C, S, B = wl.model.n_visible, wl.n_chains, wl.n_sweeps, wl.n_burnin
    M = wl.model.widths[0]
    props = C * (S + B) * N
    step = Step(nqs, torch, wl, params, a.dtype, a.lanes, a.refresh)
    ms, phases = step.timed(a.steps, a.warmup)
    out = _common(a, wl, props, ms, phases, step, "synthetic (seeded random RBM weights, N(0, 0.02^2))")
    # the sampler computes in FP32 (product-form ratios, log-ratio, accept test) on weights rounded to the
    # sampling format; local-energy ratios FP32, their sums and every average FP64
    out["dtype"] = "f32"
    out["weights_format"] = a.dtype
    out["arith"] = (f"FP32 arithmetic on {a.dtype.upper()}-rounded weights (the (cosh 2W, sinh 2W) table is built "
                    f"from the rounded weights); FP64 local-energy sums and averages")
    out["config"] = {"workload": wl.name, "lattice": "10x10 periodic", "J": 1.0, "h": 3.04, "rbm_hidden": M,
                     "chains": C, "sweeps": S, "burnin": B, "proposals_per_step": props, "samples_per_step": S * C,
                     "refresh_sweeps": a.refresh, "lanes_per_chain": a.lanes or "default",
                     "parallelism": "single GPU"}
    # Algorithmic work of one single-flip proposal: the log-amplitude ratio of an RBM needs M log-cosh
    # evaluations of the shifted pre-activations (two transcendentals each) and about 2M multiply-adds,
    # counted as 4M operations against the FP32 vector peak.  The kernel's own arithmetic (product form,
    # no transcendental per hidden unit) is reported beside it.
    acc = out["acceptance"]
    t_k = phases["sample"] * 1e-3
    alg = 4.0 * M
    achieved = props * alg / t_k / 1e12
    impl = 4.0 * M + 3.0 * M * acc + 2.0 * M / a.refresh
    out["roofline"] = {"kernel": "rbm_sample_kernel", "bound": "alu", "achieved": round(achieved, 3),
                       "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4),
                       "traffic": kernel_traffic("rbm_sample_kernel", "tfim2d_10x10_rbm_bf16_hbm_traffic.txt",
                                                 "rbm_sample_kernel<32, 7, true, false, false>"),
                       "traffic_unit": "bytes per launch (HBM, counter-calibrated)",
                       "ops_per_proposal": alg, "ops_per_proposal_note": "M log-cosh (2M transcendentals) + 2M FMA",
                       "proposals_per_launch": props, "launch_ms": round(phases["sample"], 3),
                       "transcendental_view": {
                           "per_proposal": 2.0 * M,
                           "achieved_per_s": props * 2.0 * M / t_k,
                           "measured_rate_per_s": MEASURED_EXP2_LOG2_PER_S,
                           "frac": round(props * 2.0 * M / t_k / MEASURED_EXP2_LOG2_PER_S, 4)},
                       "implementation_count": {
                           "flops_per_proposal": round(impl, 2),
                           "note": "4M (ratio factors) + 3M x acceptance (state update) + 2M / refresh (theta)",
                           "achieved": round(props * impl / t_k / 1e12, 3),
                           "frac": round(props * impl / t_k / 1e12 / PEAK_FP32_VALU_TFLOPS, 4)}}
    out["sr_step"] = _sr_step(nqs, torch, step)
    out["detectors"] = _detectors(nqs, torch, wl, params, a.dtype, a.refresh)
    if not a.no_compare:
        out.update(_compare_fp32(a, nqs, torch, wl, params, step, ms, props, "f32", True, others=("f16", "e4m3")))
    del step
    torch.cuda.empty_cache()
    if not a.no_cpu_baseline:
        pc, ps = C, 8
        dev_el = {fmt: _device_short_run(nqs, torch, wl, params, fmt, pc, ps, a.refresh)
                  for fmt in (a.dtype, "f32")}
        out["cpu_baseline"] = cpu_baseline(wl, params, paired_chains=pc, paired_sweeps=ps, device_eloc=dev_el)
        out["dE_vs_fp64"] = out["cpu_baseline"].pop("dE_vs_fp64")
        out["dE_vs_fp64"]["setup"] = out["cpu_baseline"].pop("dE_vs_fp64_setup")
    if not a.headline_only:
        out["other_workloads"] = _other_workloads(a, torch, nqs, workloads)
    return out


def _detectors(nqs, torch, wl, params, dtype, refresh):
    """The run-time detectors on a short run of the headline workload (untimed): non-finite log-ratios, chains
    without an accepted move for 10 sweeps, and the largest drift of log psi carried by the accepted
    log-ratios against log psi recomputed at a refresh."""
    N, C, S, B = wl.model.n_visible, wl.n_chains, 20, 10
    model = nqs.Model.from_workload(wl, params)
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=wl.seed, dtype=dtype, refresh_sweeps=refresh)
    state = torch.empty(C, N, dtype=torch.int8, device="cuda")
    lp = torch.empty(S, C, dtype=torch.float32, device="cuda")
    r = nqs.nqs_sample_checked(model, cfg, state, None, lp, stuck_after=10)
    r["mean_abs_logpsi"] = round(float(lp.abs().mean().item()), 4)
    r["run"] = f"{C} chains x ({B} + {S}) sweeps, refresh every {refresh} sweeps, {dtype} copy"
    model.close()
    return r


def _antiparallel_bonds(torch, samples, L):
    """Number of antiparallel nearest-neighbour bonds summed over all samples of a periodic L x L
    lattice (each one is a connected configuration the Heisenberg local energy evaluates)."""
    tot = 0
    flat = samples.reshape(-1, L, L)
    for k in range(0, flat.shape[0], 1 << 20):
        x = flat[k:k + (1 << 20)]
        tot += int((x != torch.roll(x, 1, dims=1)).sum().item()) + int((x != torch.roll(x, 1, dims=2)).sum().item())
    return tot


def run_heis10(a, torch, nqs, workloads, compact=False):
    wl = workloads.cfg3_heis_10x10()
    params = workloads.params_for(wl)
    N, C, S, B = wl.model.n_visible, wl.n_chains, wl.n_sweeps, wl.n_burnin
    props = C * (S + B) * N
    step = Step(nqs, torch, wl, params, a.dtype, 0, a.refresh, eloc_dtype=a.dtype, with_gram=True)
    ms, phases = step.timed(a.steps, a.warmup)
    out = _common(a, wl, props, ms, phases, step, "synthetic (seeded He-initialised FFNN)")
    w1, w2 = wl.model.widths
    out["config"] = {"workload": wl.name, "lattice": "10x10 periodic", "J": 1.0, "marshall": True,
                     "ffnn": [N, w1, w2], "move": "exchange", "chains": C, "sweeps": S, "burnin": B,
                     "proposals_per_step": props, "samples_per_step": S * C, "parallelism": "single GPU"}
    out["arith"] = (f"{a.dtype.upper()} operands of both layers' products, FP32 accumulation, FP32 nonlinearities, "
                    f"log-ratio and accept test; FP64 local-energy sums")
    peak = PEAK_BF16_MFMA_TFLOPS if a.dtype != "f32" else PEAK_FP32_VALU_TFLOPS
    # dominant contraction of the sampler: layer 2 of the proposed state, 2 w1 w2 flops per evaluated
    # proposal on the matrix cores.  An exchange of two equal spins changes nothing and is not evaluated;
    # at zero magnetisation a uniform ordered pair of distinct sites differs with probability exactly
    # N / (2 (N - 1)), so that is the fraction of proposals that need the product.
    eff = N / (2.0 * (N - 1))
    fpp = 2.0 * w1 * w2 * eff
    achieved = props * fpp / (phases["sample"] * 1e-3) / 1e12
    sampler_rl = {"kernel": "ffnn_sample_reg_kernel", "bound": "mfma", "achieved": round(achieved, 2),
                  "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                  "flops_per_proposal": round(fpp, 1), "evaluated_fraction": round(eff, 4),
                  "proposals_per_launch": props, "launch_ms": round(phases["sample"], 3)}
    # local energies: every antiparallel bond of every sample is a connected configuration whose layer 2
    # (2 w1 w2 flops) runs on the matrix cores
    rows = _antiparallel_bonds(torch, step.samples, wl.ham.lattice.L)
    el_ach = rows * 2.0 * w1 * w2 / (phases["local_energy"] * 1e-3) / 1e12
    eloc_rl = {"kernel": "ffnn_eloc_reg_kernel", "bound": "mfma", "achieved": round(el_ach, 2), "peak": peak,
               "unit": "TFLOP/s", "frac": round(el_ach / peak, 4), "traffic": None,
               "rows_per_launch": rows, "flops_per_row": 2.0 * w1 * w2, "launch_ms": round(phases["local_energy"], 3),
               "note": "rows = antiparallel bonds summed over the step's samples"}
    # the dominant kernel of the step is the one that takes longer
    if phases["local_energy"] >= phases["sample"]:
        out["roofline"], out["sampler_roofline"] = eloc_rl, sampler_rl
    else:
        out["roofline"], out["eloc_roofline"] = sampler_rl, eloc_rl
    if not compact:
        out["sr_step"] = _sr_step(nqs, torch, step)
    if not a.no_compare:
        out.update(_compare_fp32(a, nqs, torch, wl, params, step, ms, props, a.dtype, not compact,
                                 others=() if compact else ("f16",)))
    if not a.no_cpu_baseline and not compact:
        out["cpu_baseline"] = cpu_baseline(wl, params, budget_s=15.0)
    return out


def _other_workloads(a, torch, nqs, workloads):
    """One timed step each (after one untimed) of the dense-network and uneven-batch workloads, in the
    same format as the headline and against FP32, so the matrix-core paths are measured in the same run."""
    import copy
    b = copy.copy(a)
    b.steps, b.warmup, b.no_cpu_baseline = 1, 1, True
    keep = ("value", "unit", "ms_per_step", "dtype", "arith", "phases_ms", "sampler_proposals_per_s",
            "eloc_samples_per_s", "acceptance", "energy", "config", "roofline", "sampler_roofline", "eloc_roofline",
            "speedup_vs_fp32", "dE_vs_fp32", "fp32", "persistent_ms", "separate_launches_ms",
            "separate_launches_graph_ms", "speedup_vs_separate", "speedup_vs_graph", "gram_T", "steps", "warmup")
    res = {}
    b8 = copy.copy(b)
    b8.dtype, b8.no_compare, b8.gram_samples = "e4m3", True, 0
    for name, fn in (("heis10", lambda: run_heis10(b, torch, nqs, workloads, compact=True)),
                     ("uneven", lambda: run_uneven(b, torch, nqs, workloads)),
                     ("heis20", lambda: run_heis20(b, torch, nqs, workloads)),
                     ("heis20_e4m3", lambda: run_heis20(b8, torch, nqs, workloads))):
        r = fn()
        res[name] = {k: v for k, v in r.items() if k in keep}
        torch.cuda.empty_cache()
    return res


def run_uneven(a, torch, nqs, workloads):
    insts = workloads.cfg4_instances()
    dev = torch.device("cuda:0")
    models, jobs = [], []
    props = 0
    alg_ops = 0.0   # per proposal: M log-cosh (2M transcendentals) + 2M FMA, as for the headline sampler
    for k, wl in enumerate(insts):
        m = nqs.Model.from_workload(wl)
        m.prepare(a.dtype)
        models.append(m)
        N = wl.model.n_visible
        cfg = nqs.SampleConfig(n_chains=wl.n_chains, n_sweeps=wl.n_sweeps, n_burnin=wl.n_burnin, seed=wl.seed,
                               dtype=a.dtype, instance_id=k, refresh_sweeps=a.refresh)
        jobs.append({"model": m, "cfg": cfg,
                     "chain_state": torch.empty(wl.n_chains, N, dtype=torch.int8, device=dev),
                     "samples": torch.empty(wl.n_sweeps, wl.n_chains, N, dtype=torch.int8, device=dev),
                     "n_accepted": torch.empty(wl.n_chains, dtype=torch.int64, device=dev)})
        props += wl.n_chains * (wl.n_sweeps + wl.n_burnin) * N
        alg_ops += wl.n_chains * (wl.n_sweeps + wl.n_burnin) * N * 4.0 * wl.model.widths[0]

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / a.steps

    ms0 = timed(lambda: nqs.nqs_sample_batched(jobs, mode=0))
    ms1 = timed(lambda: nqs.nqs_sample_batched(jobs, mode=1))
    # every instance at the tuner's choice between 32 and 64 lanes per chain (measured on the first call)
    jobs_t = [dict(j, cfg=dataclasses.replace(j["cfg"], lanes_per_chain=nqs.LANES_TUNED)) for j in jobs]
    ms_t = timed(lambda: nqs.nqs_sample_batched(jobs_t, mode=0))
    # the 32 separate launches captured once into a graph and replayed
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        nqs.nqs_sample_batched(jobs, mode=1)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            nqs.nqs_sample_batched(jobs, mode=1)
    torch.cuda.synchronize()
    ms2 = timed(g.replay)
    out = {
        "metric": METRIC, "value": props / (ms0 * 1e-3), "unit": "proposals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": a.dtype, "data": "synthetic (32 seeded uneven TFIM/RBM instances)",
        "config": {"workload": "tfim2d_uneven_32", "instances": [w.name for w in insts], "chains_each": 1024,
                   "sweeps": 200, "burnin": 20, "proposals_per_step": props, "parallelism": "single GPU"},
        "persistent_ms": ms0, "persistent_tuned_ms": ms_t, "separate_launches_ms": ms1,
        "separate_launches_graph_ms": ms2,
        "lanes_rule": "32 lanes per chain for M <= 256, else 64 (persistent_tuned_ms: the measured choice)",
        "speedup_vs_separate": ms1 / ms0, "speedup_vs_graph": ms2 / ms0,
        "arith": f"FP32 arithmetic on {a.dtype.upper()}-rounded weights",
        "roofline": {"kernel": "rbm_batched_kernel", "bound": "alu",
                     "achieved": round(alg_ops / (ms0 * 1e-3) / 1e12, 3), "peak": PEAK_FP32_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(alg_ops / (ms0 * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4),
                     "traffic": None, "ops_per_launch": alg_ops,
                     "ops_note": "sum over instances of proposals x 4M (M log-cosh + 2M FMA)"},
    }
    for m in models:
        m.close()
    return out


def run_heis20(a, torch, nqs, workloads):
    wl = workloads.cfg5_heis_20x20()
    params = workloads.params_for(wl)
    N, C = wl.model.n_visible, wl.n_chains
    sweeps = a.sweeps or 1
    dev = torch.device("cuda:0")
    model = nqs.Model.from_workload(wl, params)
    ham = nqs.Hamiltonian.from_workload(wl.ham)
    state = torch.empty(C, N, dtype=torch.int8, device=dev)
    samples = torch.empty(sweeps, C, N, dtype=torch.int8, device=dev)
    acc = torch.empty(C, dtype=torch.int64, device=dev)
    n_el = 1024
    eloc = torch.empty(n_el, dtype=torch.float64, device=dev)
    n_t = min(a.gram_samples, C)
    T = torch.empty(n_t, n_t, dtype=torch.float32, device=dev) if n_t else None
    model.prepare(a.dtype)
    props = C * sweeps * N
    res = {}
    for dt in ([a.dtype] if a.no_compare else [a.dtype, "f32"]):
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=sweeps, n_burnin=0, seed=wl.seed, dtype=dt, move="exchange")
        for _ in range(a.warmup):
            nqs.nqs_sample(model, cfg, state, samples, None, acc)
        torch.cuda.synchronize()
        def gram():
            if a.gram_chunked:
                nqs.nqs_sample_gram(model, samples[sweeps - 1, :n_t], T)
            else:
                nqs.nqs_sample_gram_factored(model, samples[sweeps - 1, :n_t], T)
        if n_t and dt == a.dtype:
            gram()   # warm the workspace
        ev = _events(torch, 4)
        t_s = t_e = t_t = 0.0
        for _ in range(a.steps):
            ev[0].record()
            nqs.nqs_sample(model, cfg, state, samples, None, acc)
            ev[1].record()
            nqs.nqs_local_energy(model, ham, samples[sweeps - 1, :n_el], eloc, dt)
            ev[2].record()
            # O and T come from the FP32 copy whatever the sampling dtype: timed once
            if n_t and dt == a.dtype:
                gram()
            ev[3].record()
            torch.cuda.synchronize()
            t_s += ev[0].elapsed_time(ev[1]) / a.steps
            t_e += ev[1].elapsed_time(ev[2]) / a.steps
            t_t += ev[2].elapsed_time(ev[3]) / a.steps
        res[dt] = {"sample_ms": t_s, "eloc_ms": t_e, "gram_ms": t_t, "acceptance": float(acc.sum().item()) / props,
                   "eloc_mean": float(eloc.mean().item())}
    w = wl.model.widths
    peak = {"f32": 157.3, "e4m3": PEAK_FP8_MFMA_TFLOPS}.get(a.dtype, PEAK_BF16_MFMA_TFLOPS)
    flops = 2.0 * (N * w[0] + w[0] * w[1] + w[1] * w[2])   # full forward per proposal
    eff = 0.5 * props   # exchange of equal spins is not evaluated
    r0 = res[a.dtype]
    achieved = eff * flops / (r0["sample_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": props / (r0["sample_ms"] * 1e-3), "unit": "proposals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": r0["sample_ms"] + r0["eloc_ms"] + r0["gram_ms"],
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": a.dtype, "data": "synthetic (seeded He-initialised FFNN)",
        "arith": (f"{a.dtype.upper()} operands of every layer's product, FP32 accumulation, FP32 nonlinearities, "
                  f"log-ratio and accept test; FP64 local-energy sums"),
        "config": {"workload": wl.name, "lattice": "20x20 periodic", "J": 1.0, "marshall": True, "ffnn": [N, *w],
                   "move": "exchange", "chains": C, "sweeps_per_step": sweeps, "burnin": 0,
                   "proposals_per_step": props, "eloc_samples": n_el, "parallelism": "single GPU"},
        "phases_ms": {"sample": round(r0["sample_ms"], 3), "local_energy": round(r0["eloc_ms"], 3),
                      ("gram_T_chunked" if a.gram_chunked else "gram_T_factored"): round(r0["gram_ms"], 3)},
        "eloc_samples_per_s": n_el / (r0["eloc_ms"] * 1e-3),
        "acceptance": r0["acceptance"],
        "roofline": {"kernel": "deep_gemm_kernel (all layers)", "bound": "mfma", "achieved": round(achieved, 2),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": None, "flops_per_effective_proposal": flops,
                     "note": "about half of the exchange proposals swap equal spins and are not evaluated"},
    }
    if "f32" in res and a.dtype != "f32":
        out["fp32"] = {"sample_ms": res["f32"]["sample_ms"], "eloc_ms": res["f32"]["eloc_ms"]}
        out["speedup_vs_fp32"] = ((res["f32"]["sample_ms"] + res["f32"]["eloc_ms"])
                                  / (r0["sample_ms"] + r0["eloc_ms"]))
    if n_t:
        P = model.n_params
        if a.gram_chunked:
            chunk = max(32, ((1 << 28) // n_t) & ~31)
            t_flops = 1.0 * n_t * (n_t + 1) * P    # 2P flops per entry of the upper triangle of the symmetric T
            tf = t_flops / (r0["gram_ms"] * 1e-3) / 1e12
            out["gram_T"] = {"path": "column blocks", "samples": n_t, "params": P, "column_block": chunk,
                             "blocks": -(-P // chunk), "ms": round(r0["gram_ms"], 3), "tflops": round(tf, 2),
                             "peak_fp32_mfma": 157.3, "frac": round(tf / 157.3, 4),
                             "note": "whole phase: per-sample factors of O once, then per column block the "
                                     "expansion of O, its column means and the contraction"}
        else:
            dsum = sum([N, *w[:-1]]) + sum(w)   # factor widths: layer inputs and deltas
            nt = -(-n_t // 64)
            fac_flops = 2.0 * (nt * (nt + 1) // 2) * 64 * 64 * dsum   # contraction of the factor Gram tiles
            param_flops = 1.0 * n_t * (n_t + 1) * P                   # the same T contracted over all P
            out["gram_T"] = {"path": "factored", "samples": n_t, "params": P, "factor_width": dsum,
                             "ms": round(r0["gram_ms"], 3),
                             "factor_contraction_tflop": round(fac_flops / 1e12, 3),
                             "parameter_space_equivalent_tflop": round(param_flops / 1e12, 2),
                             "note": "whole phase: per-sample factors (layer inputs and deltas), FP64 means, "
                                     "per-sample centring terms, FP64 matrix-core contraction of the factor "
                                     "Gram tiles"}
    return out


def _train_rbm(nqs, torch, N, M, h, iters, seed):
    """SR training of an RBM on the N-site TFIM chain (J = 1, field h, periodic); returns FP64 parameters."""
    import workloads
    dev = torch.device("cuda:0")
    ham = nqs.Hamiltonian("tfim", 1, N, 1.0, h, True)
    p = workloads.rbm_params(N, M, 0.01, seed)
    model = nqs.Model("rbm", N, (M,), p)
    master = torch.from_numpy(p.copy()).to(dev)
    C, S = 512, 4
    n = C * S
    state = torch.empty(C, N, dtype=torch.int8, device=dev)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=dev)
    eloc = torch.empty(n, dtype=torch.float64, device=dev)
    T = torch.empty(n, n, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    offset = 0
    solve_log = []
    for it in range(iters):
        model.set_params_device(master)
        model.prepare("f32")
        burn = 20 if it == 0 else 2
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=burn, seed=seed, step_offset=offset,
                               init_chains=it == 0)
        nqs.nqs_sample(model, cfg, state, samples)
        offset += (burn + S) * N
        flat = samples.reshape(n, N)
        nqs.nqs_local_energy(model, ham, flat, eloc)
        nqs.nqs_sample_gram_factored(model, flat, T)
        its, rr = nqs.nqs_sr_solve(T, eloc, 1e-2, y, tol=1e-6, max_iter=300)
        solve_log.append((its, rr))
        nqs.nqs_sr_update(model, flat, y, 0.05, master)
    model.close()
    return master.cpu().numpy(), _solve_summary(solve_log, 1e-6, 300)


def _solve_summary(log, tol, max_iter):
    """Iteration counts and final relative residuals of the SR solves of a training run; a solve that
    stops at max_iter above tol is counted as unconverged (its direction was still used)."""
    its = np.array([k for k, _ in log], dtype=np.float64)
    rr = np.array([r for _, r in log], dtype=np.float64)
    return {"solves": len(log), "iterations_mean": float(its.mean()) if len(log) else 0.0,
            "iterations_max": int(its.max()) if len(log) else 0,
            "rel_residual_max": float(rr.max()) if len(log) else 0.0, "tol": tol,
            "unconverged": int(np.sum((its >= max_iter) & (rr > tol))),
            "note": "the Jacobi solve checks its residual every 8 iterations, so counts are multiples of 8"}


def _avg_bound(sigma):
    """The average bound of Thm 3.3 (Eq. eq:avg_bound) at mu = 0, r = 0: 1 - e^{sigma^2} erfc(sigma)."""
    import scipy.special
    return float(1.0 - np.exp(sigma * sigma) * scipy.special.erfc(sigma)) if sigma > 0 else 0.0


def run_noise(a, torch, nqs, workloads):
    """Noisy-RBM study (Sec. IV.A) on the 16-site TFIM chain: the shifts of <sigma^x> and <Pi_even> that noisy
    sampling produces against sigma (2^18 samples per point, chain-mean standard errors) beside the KL
    (Pinsker) and average total-variation bounds; the acceptance rate against sigma for RBMs trained here at
    several h/J; and the law of delta over sampled configurations.  The comparison with the exact perturbed
    distribution by enumeration is tests/test_gpu_noise_bounds.py."""
    dev = torch.device("cuda:0")
    N, M = 16, 16
    sigmas = [0.0, 0.01, 0.03, 0.1, 0.3, 1.0, 2.0]
    ham_x = workloads.Hamiltonian("tfim", workloads.Lattice(1, N), 0.0, 1.0)   # eps = sum_i psi(x^i)/psi(x)
    C, S = 1024, 256                                                            # 2^18 samples
    state = torch.empty(C, N, dtype=torch.int8, device=dev)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=dev)
    acc = torch.empty(C, dtype=torch.int64, device=dev)
    ex = torch.empty(S * C, dtype=torch.float64, device=dev)
    noise_seed = 20260101

    def sample(model, sigma, seed):
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=50, seed=seed)
        nqs.nqs_sample_noisy(model, cfg, sigma, noise_seed, state, samples, None, acc)
        nqs.nqs_local_energy(model, nqs.Hamiltonian.from_workload(ham_x), samples, ex)
        sx = (ex.cpu().numpy() / N).reshape(S, C).mean(axis=0)                  # chain means
        par = (np.sum(samples.cpu().numpy() > 0, axis=2) % 2 == 0).astype(np.float64).mean(axis=0)
        rate = float(acc.sum().item()) / (C * (S + 50) * N)
        return sx, par, rate

    bias = []
    t0 = time.perf_counter()
    props = 0
    for r in range(3):   # random initialisations
        p = workloads.rbm_params(N, M, 0.25, 100 + r)
        model = nqs.Model("rbm", N, (M,), p)
        sx0, par0, _ = sample(model, 0.0, 7)
        props += C * (S + 50) * N
        for sg in sigmas[1:]:
            sx1, par1, _ = sample(model, sg, 7)
            props += C * (S + 50) * N
            row = {"init": r, "sigma": sg, "tv_bound_kl": 0.5 * sg, "tv_bound_avg_r0": _avg_bound(sg)}
            for name, x1, x0 in (("sigma_x", sx1, sx0), ("Pi_even", par1, par0)):
                shift = float(x1.mean() - x0.mean())
                se = float(np.sqrt(x1.var(ddof=1) / C + x0.var(ddof=1) / C))
                row[name] = {"mean_sigma0": float(x0.mean()), "shift": shift, "rel_shift": abs(shift / x0.mean()),
                             "shift_3se": 3.0 * se}
            bias.append(row)
        model.close()
    t_bias = time.perf_counter() - t0
    accept = []
    trained, training_solves = {}, {}
    for h in (-0.5, -1.0, -5.0):   # h/J, stoquastic sign (positive amplitudes)
        p, training_solves[abs(h)] = _train_rbm(nqs, torch, N, 2 * N, h, 150, 5)
        trained[abs(h)] = p
        model = nqs.Model("rbm", N, (2 * N,), p)
        for sg in sigmas:
            _, _, rate = sample(model, sg, 9)
            props += C * (S + 50) * N
            accept.append({"h_over_J": abs(h), "sigma": sg, "acceptance": rate})
        model.close()
    # law of delta = 2 (f_lp - f_32) (Eq. eq:pert_chain) on sampled configurations: f_lp is the log|psi| the
    # sampler reports from its reduced-precision copy, f_32 the library's evaluation with the FP32 copy
    import scipy.stats
    lp = torch.empty(S, C, dtype=torch.float32, device=dev)
    ref = torch.empty(C, dtype=torch.float32, device=dev)
    law = []
    for name, p, m in (("random", workloads.rbm_params(N, M, 0.25, 100), M), ("trained_h0.5", trained[0.5], 2 * N)):
        model = nqs.Model("rbm", N, (m,), p)
        for dt in ("bf16", "f16", "e4m3"):
            cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=50, seed=3, dtype=dt)
            nqs.nqs_sample(model, cfg, state, samples, lp)
            nqs.nqs_logpsi_grad(model, samples[S - 1].contiguous(), logpsi=ref)
            d = 2.0 * (lp[S - 1].cpu().numpy().astype(np.float64) - ref.cpu().numpy().astype(np.float64))
            sw = scipy.stats.shapiro(d[:4096]).statistic if np.std(d) > 0 else float("nan")
            law.append({"state": name, "dtype": dt, "delta_mean": float(d.mean()), "delta_std": float(d.std()),
                        "shapiro_wilk": float(sw),
                        "unit_roundoff": {"bf16": 2.0 ** -8, "f16": 2.0 ** -11, "e4m3": 2.0 ** -4}[dt]})
        model.close()
    wall = time.perf_counter() - t0
    return {
        "metric": METRIC, "value": props / wall, "unit": "proposals/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (random RBMs; RBMs trained here by SR)",
        "config": {"workload": "noisy_rbm_tfim1d_n16", "sites": N, "samples_per_point": C * S,
                   "sigmas": sigmas, "parallelism": "single GPU",
                   "note": "value = proposals/s of the whole study including training"},
        "bias_vs_sigma": bias, "acceptance_vs_sigma": accept, "delta_law": law, "bias_study_s": round(t_bias, 2),
        "training_sr_solves": {str(k): v for k, v in training_solves.items()},
    }


def run_rescnn(a, torch, nqs, workloads):
    """Residual convolutional network (App. H): sampling time against the number of samples N_s (chains
    N_s / 4, four measured sweeps each) and the number of filters on the 4 x 4 lattice with four blocks,
    per sampling format (the grid of the paper's Fig. A5), and the proposal rate of one sweep of 4096
    chains on the 10 x 10 lattice with 16 filters (the network of the paper's Fig. 3)."""
    dev = torch.device("cuda:0")
    grid = []
    ev = _events(torch, 2)

    def time_sampling(model, N, C, S, B, dt, reps):
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=1, dtype=dt)
        state = torch.empty(C, N, dtype=torch.int8, device=dev)
        samples = torch.empty(S, C, N, dtype=torch.int8, device=dev)
        nqs.nqs_sample(model, cfg, state, samples)   # warm: copies, first launch
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            nqs.nqs_sample(model, cfg, state, samples)
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    L, R = 4, 4
    for F in (8, 16, 32):
        p = workloads.rescnn_params(F, R, F)
        model = nqs.Model.rescnn(L, F, R, p)
        for ns in (1 << 12, 1 << 14, 1 << 16):
            row = {"filters": F, "samples": ns, "chains": ns // 4}
            for dt in ("f32", "bf16", "f16"):
                row[dt + "_ms"] = round(time_sampling(model, L * L, ns // 4, 4, 10, dt, 1), 3)
            row["speedup_bf16"] = round(row["f32_ms"] / row["bf16_ms"], 3)
            row["speedup_f16"] = round(row["f32_ms"] / row["f16_ms"], 3)
            grid.append(row)
        model.close()
    # the Fig. 3 network: 10 x 10, 16 filters, 4 blocks, one sweep of 4096 chains
    L, F = 10, 16
    model = nqs.Model.rescnn(L, F, R, workloads.rescnn_params(F, R, 3))
    C = 4096
    props = C * L * L
    res = {dt: time_sampling(model, L * L, C, 1, 0, dt, a.steps) for dt in ("f32", "bf16")}
    dt = a.dtype if a.dtype in res else "bf16"
    ms = res[dt]
    macs = L * L * F * 9 * (1 + 2 * R * F)                     # per forward pass
    achieved = 2.0 * macs * props / (ms * 1e-3) / 1e12
    peak = PEAK_BF16_MFMA_TFLOPS if dt != "f32" else 157.3
    return {
        "metric": METRIC, "value": props / (ms * 1e-3), "unit": "proposals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dt, "data": "synthetic (seeded random ResCNN weights)",
        "config": {"workload": "rescnn_tfim2d_10x10_f16_r4", "lattice": "10x10 periodic", "filters": F,
                   "blocks": R, "kernel": "3x3", "chains": C, "sweeps_per_step": 1, "proposals_per_step": props,
                   "parallelism": "single GPU"},
        "fp32_ms": round(res["f32"], 3), "speedup_vs_fp32": round(res["f32"] / ms, 3),
        "roofline": {"kernel": "cnn_sample_mc_kernel", "bound": "mfma", "achieved": round(achieved, 3),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": None, "flops_per_proposal": 2.0 * macs,
                     "note": "one forward pass per proposal; convolutions on the matrix cores, four chains per "
                             "workgroup on this lattice; layer norms, GELU and the embedding on the VALU"},
        "speedup_grid_4x4": grid,
    }


def run_crbm(a, torch, nqs, workloads):
    """Complex-parameter RBM (App. G with complex a, b, W) on the 10 x 10 periodic TFIM at h/J = 3.04 with
    200 hidden units: single-flip sampling of 4096 chains against the real RBM sampler at the same shape, and
    the complex local energies of the emitted samples."""
    dev = torch.device("cuda:0")
    N, M, C, S, B = 100, 200, 4096, 100, 10
    ev = _events(torch, 2)
    ham = nqs.Hamiltonian("tfim", 2, 10, 1.0, 3.04, True)

    def time_sampling(model, dt, reps):
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=1, dtype=dt)
        state = torch.empty(C, N, dtype=torch.int8, device=dev)
        samples = torch.empty(S, C, N, dtype=torch.int8, device=dev)
        n_acc = torch.empty(C, dtype=torch.int64, device=dev)
        nqs.nqs_sample(model, cfg, state, samples, None, n_acc)   # warm: copies, first launch
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            nqs.nqs_sample(model, cfg, state, samples, None, n_acc)
        ev[1].record()
        torch.cuda.synchronize()
        acc = float(n_acc.sum().item()) / (C * (S + B) * N)
        return ev[0].elapsed_time(ev[1]) / reps, samples, acc

    p = workloads.crbm_params(N, M, 0.02, 0.02, 5)
    model = nqs.Model("crbm", N, (M,), p)
    res = {dt: time_sampling(model, dt, a.steps) for dt in ("f32", "bf16")}
    dt = a.dtype if a.dtype in res else "bf16"
    ms, samples, acc = res[dt]
    flat = samples.reshape(-1, N)
    re = torch.empty(flat.shape[0], dtype=torch.float64, device=dev)
    im = torch.empty_like(re)
    nqs.nqs_local_energy_complex(model, ham, flat, re, im, eval_dtype=dt)
    torch.cuda.synchronize()
    ev[0].record()
    nqs.nqs_local_energy_complex(model, ham, flat, re, im, eval_dtype=dt)
    ev[1].record()
    torch.cuda.synchronize()
    eloc_ms = ev[0].elapsed_time(ev[1])
    # one SR step with complex parameters on the last sweep's 4096 samples: O (FP32 copy), the real
    # embedding of T (nqs_gram mode 3), the complex solve and the update
    last = samples[S - 1].contiguous()
    er, ei = re.view(S, C)[S - 1].contiguous(), im.view(S, C)[S - 1].contiguous()
    Pc = N + M + M * N
    O = torch.empty(C, 2 * Pc, dtype=torch.float32, device=dev)
    T2 = torch.empty(2 * C, 2 * C, dtype=torch.float32, device=dev)
    y2 = torch.empty(2 * C, dtype=torch.float64, device=dev)
    master = torch.from_numpy(p.copy()).to(dev)
    sr_ev = _events(torch, 5)
    sr_ev[0].record()
    nqs.nqs_logpsi_grad(model, last, None, O)
    sr_ev[1].record()
    nqs.nqs_gram(O, 3, T2)
    sr_ev[2].record()
    sr_it, sr_rr = nqs.nqs_sr_solve_complex(T2, er, ei, 1e-2, y2, tol=1e-8, max_iter=2000)
    sr_ev[3].record()
    nqs.nqs_sr_update(model, last, y2, 0.01, master)
    sr_ev[4].record()
    torch.cuda.synchronize()
    sr_phases = {k: round(sr_ev[q].elapsed_time(sr_ev[q + 1]), 3)
                 for q, k in enumerate(("logpsi_grad", "gram_T_complex", "solve", "update"))}
    del O, T2
    real = nqs.Model("rbm", N, (M,), p[:N + M + M * N])
    real_ms, _, real_acc = time_sampling(real, dt, a.steps)
    model.close()
    real.close()
    props = C * (S + B) * N
    # FP32 flops of the complex product-form single flip, per hidden unit: n = c C - s_i s S (14) with its
    # squared modulus (3) and the running product (1) on every proposal, plus the s_i S products (2); the
    # state update s <- s C - s_i c S (16) per accepted proposal; the refresh theta = W s + b (4 N M flops
    # once per sweep of N proposals).  The lane's one logarithm is not counted.
    fpp = 20.0 * M + 16.0 * M * acc + 4.0 * M
    achieved = props * fpp / (ms * 1e-3) / 1e12
    return {
        "metric": METRIC, "value": props / (ms * 1e-3), "unit": "proposals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dt, "data": "synthetic (seeded random complex RBM weights, N(0, 0.02^2) real and imaginary)",
        "config": {"workload": "crbm_tfim2d_10x10_a2", "lattice": "10x10 periodic", "J": 1.0, "h": 3.04,
                   "rbm_hidden": M, "chains": C, "sweeps": S, "burnin": B, "proposals_per_step": props,
                   "parallelism": "single GPU"},
        "acceptance": round(acc, 4), "fp32_ms": round(res["f32"][0], 3),
        "real_rbm_ms": round(real_ms, 3), "real_rbm_acceptance": round(real_acc, 4),
        "complex_vs_real_time": round(ms / real_ms, 3),
        "eloc_complex_ms": round(eloc_ms, 3), "eloc_samples": int(flat.shape[0]),
        "sr_step": {"samples": C, "params_complex": Pc, "phases_ms": sr_phases, "cg_iterations": sr_it,
                    "rel_resid": sr_rr, "shift": 1e-2,
                    "gram_tflop": round(2.0 * (2 * C) ** 2 * (2 * Pc) / 1e12, 3),
                    "note": "T embedded as the 2n x 2n real matrix [[Re T, -Im T], [Im T, Re T]]; CG on 2n unknowns"},
        "roofline": {"kernel": "crbm_sample_kernel", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4), "traffic": None,
                     "flops_per_proposal": round(fpp, 2), "proposals_per_launch": props},
    }


def run_peaks(a, torch, nqs, workloads):
    """Achievable rates of this device from the microbenchmarks of include/nqs_probe.h (best of three
    launches each), next to the published peaks that the roofline figures divide by."""
    dev = torch.device("cuda:0")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    scratch = torch.empty(cus * 16 * 256, dtype=torch.float32, device=dev)
    ev = _events(torch, 2)

    def best_rate(kind, size, src=None, dst=scratch):
        nqs.nqs_probe_rate(kind, size, src, dst)   # warm
        torch.cuda.synchronize()
        best = 0.0
        for _ in range(3):
            ev[0].record()
            w = nqs.nqs_probe_rate(kind, size, src, dst)
            ev[1].record()
            torch.cuda.synchronize()
            best = max(best, w / (ev[0].elapsed_time(ev[1]) * 1e-3))
        return best

    got = {
        "fma_f32_tflops": best_rate("fma_f32", 4000) / 1e12,
        "log2_f32_per_s": best_rate("log_f32", 1000),
        "exp2_f32_per_s": best_rate("exp_f32", 1000),
        "mfma_bf16_16x16x16_tflops": best_rate("mfma_bf16_k16", 2000) / 1e12,
        "mfma_bf16_16x16x32_tflops": best_rate("mfma_bf16_k32", 2000) / 1e12,
        "mfma_f32_16x16x4_tflops": best_rate("mfma_f32", 1000) / 1e12,
        "mfma_f64_16x16x4_tflops": best_rate("mfma_f64", 500) / 1e12,
        # one block of 512 threads per CU (two waves per SIMD, the local-energy kernel's occupancy), one
        # accumulator chain per wave; the _lds figures read every product's B operand from LDS, issued two
        # products ahead (_lds) or where the compiler schedules it (_lds_jit)
        "mfma_bf16_32x32x16_tflops": best_rate("mfma_bf16_32", 2000) / 1e12,
        "mfma_bf16_32x32x16_lds_tflops": best_rate("mfma_bf16_32_lds", 2000) / 1e12,
        "mfma_bf16_32x32x16_lds_jit_tflops": best_rate("mfma_bf16_32_lds_jit", 2000) / 1e12,
        "lds_read_b128_gbs": best_rate("lds_read", 4000) / 1e9,
    }
    got["lds_read_bytes_per_cu_clock"] = got["lds_read_b128_gbs"] * 1e9 / (cus * 2.4e9)
    # issue rates of the vector instructions the samplers are made of, as cycles per wave64
    # instruction per SIMD at the 2.4 GHz peak clock (4 SIMDs per CU)
    simd_hz = cus * 4 * 2.4e9
    issue = {}
    for kind, iters, per_instr in (("fma_f32", 4000, 2), ("mul_f32", 4000, 1), ("xor_u32", 4000, 1),
                                   ("dpp_add_f32", 2000, 1), ("mulhi_u32", 1000, 1), ("log_f32", 1000, 1),
                                   ("exp_f32", 1000, 1), ("fma_f32_w2", 4000, 2), ("fma_f32_w1", 4000, 2),
                                   ("fma_f32_dep", 4000, 2)):
        if kind == "fma_f32":
            r = got["fma_f32_tflops"] * 1e12
        elif kind in ("log_f32", "exp_f32"):
            r = got[kind[:3] + "2_f32_per_s"]
        else:
            r = best_rate(kind, iters)
        issue[kind] = round(simd_hz / (r / 64 / per_instr), 3)
    nbytes = 2 << 30
    x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    got["hbm_read_gbs"] = best_rate("hbm_read", nbytes, x) / 1e9
    y = torch.empty_like(x)
    got["hbm_copy_gbs"] = best_rate("hbm_copy", nbytes, x, y) / 1e9
    del x, y
    published = {"fma_f32_tflops": PEAK_FP32_VALU_TFLOPS, "mfma_bf16_16x16x32_tflops": PEAK_BF16_MFMA_TFLOPS,
                 "mfma_bf16_32x32x16_tflops": PEAK_BF16_MFMA_TFLOPS, "mfma_bf16_32x32x16_lds_tflops": PEAK_BF16_MFMA_TFLOPS,
                 "mfma_bf16_32x32x16_lds_jit_tflops": PEAK_BF16_MFMA_TFLOPS,
                 "mfma_f32_16x16x4_tflops": 157.3, "mfma_f64_16x16x4_tflops": 78.6, "hbm_read_gbs": 8000.0,
                 "hbm_copy_gbs": 8000.0}
    return {
        "metric": "achievable rates (microbenchmarks)", "value": got["mfma_bf16_16x16x32_tflops"], "unit": "TFLOP/s",
        "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "mixed", "data": "synthetic",
        "config": {"workload": "peaks", "compute_units": cus, "grid": "8 blocks of 256 threads per CU",
                   "hbm_bytes": nbytes, "parallelism": "single GPU"},
        "achieved": {k: round(v, 3) for k, v in got.items()},
        "published": published,
        "frac_of_published": {k: round(got[k] / v, 4) for k, v in published.items()},
        "cycles_per_wave64_instruction": issue,
        "issue_note": "eight independent chains per thread at 8 blocks of 256 threads per CU (8 waves per SIMD); "
                      "fma_f32_w2 / _w1: two / one wave per SIMD; fma_f32_dep: one dependent chain, one wave per "
                      "SIMD (the dependent-issue latency)",
        "note": "FP32 FMA without packed FP32 (this library never issues it); log2 / exp2 in operations per second",
    }


def run_srstudy(a, torch, nqs, workloads):
    """The SR regularisation study of App. I.2 at a size exact diagonalisation reaches: an RBM (alpha = 1) on
    the 16-site TFIM chain at the critical field, trained by SR with Tikhonov shifts 1e-3 and 1e-1, three
    ways: the reference (FP32 sampling copy, FP32 local energies), BF16 sampling, BF16 local energies (the
    reduced-precision forces of the paper's study), and both in FP8 E4M3 (log-derivatives and the solve stay
    FP32 / FP64).  Per run: the relative energy error against the
    exact ground energy along the optimisation, and the condition number of S + shift (S formed in FP64 on
    the host from the library's log-derivatives every 10 steps)."""
    dev = torch.device("cuda:0")
    N, M, J, h = 16, 16, 1.0, -1.0            # h/J = 1 (critical), stoquastic sign
    steps, lr = 150, 0.05
    C, S = 256, 4
    n = C * S
    k = np.pi * (2 * np.arange(N) + 1) / N     # free-fermion ground energy of the periodic chain
    e0 = -float(np.sum(np.sqrt(J * J + h * h - 2 * J * abs(h) * np.cos(k))))
    ham = nqs.Hamiltonian("tfim", 1, N, J, h, True)
    state = torch.empty(C, N, dtype=torch.int8, device=dev)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=dev)
    eloc = torch.empty(n, dtype=torch.float64, device=dev)
    T = torch.empty(n, n, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    runs = []
    t0 = time.perf_counter()
    for shift in (1e-3, 1e-1):
        for variant, sdt, edt in (("reference", "f32", "f32"), ("bf16_sampling", "bf16", "f32"),
                                  ("bf16_local_energies", "f32", "bf16"), ("fp8_sampling_and_local_energies", "e4m3", "e4m3")):
            p = workloads.rbm_params(N, M, 0.01, 5)
            model = nqs.Model("rbm", N, (M,), p)
            P = model.n_params
            O = torch.empty(n, P, dtype=torch.float32, device=dev)
            master = torch.from_numpy(p.copy()).to(dev)
            offset, traj, kappa, iters, energies, solve_log = 0, [], [], [], [], []
            for it in range(steps):
                model.set_params_device(master)
                model.prepare(sdt)
                burn = 20 if it == 0 else 2
                cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=burn, seed=5, step_offset=offset,
                                       init_chains=it == 0, dtype=sdt)
                nqs.nqs_sample(model, cfg, state, samples)
                offset += (burn + S) * N
                flat = samples.reshape(n, N)
                nqs.nqs_local_energy(model, ham, flat, eloc, edt)
                e = float(eloc.mean().item())
                energies.append(e)
                if it % 10 == 0 or it == steps - 1:
                    nqs.nqs_logpsi_grad(model, flat, O=O)
                    Oc = O.cpu().numpy().astype(np.float64)
                    Oc -= Oc.mean(axis=0)
                    ev = np.linalg.eigvalsh(Oc.T @ Oc / n)
                    kappa.append({"step": it, "kappa": float((ev[-1] + shift) / (max(ev[0], 0.0) + shift))})
                    traj.append({"step": it, "rel_err": abs(e - e0) / abs(e0)})
                nqs.nqs_sample_gram_factored(model, flat, T)
                its, rr = nqs.nqs_sr_solve(T, eloc, shift, y, tol=1e-8, max_iter=3000)
                iters.append(its)
                solve_log.append((its, rr))
                nqs.nqs_sr_update(model, flat, y, lr, master)
            model.close()
            last = np.array(energies[-10:])
            runs.append({"shift": shift, "variant": variant,
                         "final_rel_err": abs(float(last.mean()) - e0) / abs(e0),
                         "final_rel_err_se": float(last.std(ddof=1) / np.sqrt(last.size)) / abs(e0),
                         "energy_rel_err": traj, "kappa_S_plus_shift": kappa,
                         "cg_iterations_mean": float(np.mean(iters)),
                         "sr_solves": _solve_summary(solve_log, 1e-8, 3000)})
    wall = time.perf_counter() - t0
    return {
        "metric": "SR study: relative energy error against exact diagonalisation", "value": None,
        "unit": "relative error", "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": 1e3 * wall / (len(runs) * steps),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "mixed",
        "data": "synthetic (RBM trained here by SR)",
        "config": {"workload": "sr_study_tfim1d_n16", "sites": N, "rbm_hidden": M, "h_over_J": abs(h / J),
                   "samples_per_step": n, "learning_rate": lr, "exact_ground_energy": e0,
                   "parallelism": "single GPU"},
        "runs": runs,
    }


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "only the one-GPU path is built; --gpus above 1 is not supported", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    if a.copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 4, "copies": 3}))
        return
    import paper_2601_20782_amd as nqs
    import workloads
    run = {"tfim10": run_tfim10, "heis10": run_heis10, "uneven": run_uneven, "heis20": run_heis20,
           "noise": run_noise, "rescnn": run_rescnn, "crbm": run_crbm, "peaks": run_peaks, "srstudy": run_srstudy}[a.workload]
    print(json.dumps(run(a, torch, nqs, workloads)))


if __name__ == "__main__":
    main()
