#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over the 10x10 TFIM workload (N = 100,
RBM alpha = 2, 4096 chains, 100 burn-in + 1000 measured sweeps):
  downcast of the FP64 master -> chain init + MH sampling -> local energies of
  all 4.096e6 samples -> FP64 energy statistics -> log-derivatives of the last
  sweep's samples -> FP64 forces -> centred Gram matrix (sample space).
`value` = MH proposals per second of whole-step time with the sampling copy in
BF16 (inputs resident in HBM).  The same step with an FP32 sampling copy is
timed beside it, and the energy bias between the two is reported with its
paired error bar.  The CPU oracle is timed on a bounded sample of the same
workload on the host cores.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
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
PEAK_HBM_GBS = 8000.0


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="bf16", choices=["bf16", "f16", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 comparison step")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per chain of the sampler (0 = library default)")
    ap.add_argument("--refresh", type=int, default=1, help="sweeps between full recomputes of theta = W s + b")
    return ap.parse_args()


class Step:
    """Buffers and phases of one hot-path pass for a sampling dtype."""

    def __init__(self, nqs, torch, wl, params, dtype, lanes=0, refresh=1):
        self.nqs, self.torch, self.wl, self.dtype = nqs, torch, wl, dtype
        dev = torch.device("cuda:0")
        m = wl.model
        self.N = N = m.n_visible
        self.C, self.S, self.B = wl.n_chains, wl.n_sweeps, wl.n_burnin
        self.model = nqs.Model.from_workload(wl, params)
        self.master = torch.from_numpy(np.asarray(params, dtype=np.float64)).to(dev)
        self.ham = nqs.Hamiltonian.from_workload(wl.ham)
        self.cfg = nqs.SampleConfig(n_chains=self.C, n_sweeps=self.S, n_burnin=self.B, seed=wl.seed, dtype=dtype,
                                    lanes_per_chain=lanes, refresh_sweeps=refresh)
        self.state = torch.empty(self.C, N, dtype=torch.int8, device=dev)
        self.samples = torch.empty(self.S, self.C, N, dtype=torch.int8, device=dev)
        self.acc = torch.empty(self.C, dtype=torch.int64, device=dev)
        self.eloc = torch.empty(self.S * self.C, dtype=torch.float64, device=dev)
        self.stats = torch.empty(4, dtype=torch.float64, device=dev)
        self.P = self.model.n_params
        self.O = torch.empty(self.C, self.P, dtype=torch.float32, device=dev)
        self.F = torch.empty(self.P, dtype=torch.float64, device=dev)
        self.T = torch.empty(self.C, self.C, dtype=torch.float32, device=dev)
        self.phase_names = ["downcast", "sample", "local_energy", "stats", "logpsi_grad", "forces", "gram"]

    def run(self, events=None):
        nqs, torch = self.nqs, self.torch
        ev = events
        k = 0

        def mark():
            nonlocal k
            if ev is not None:
                ev[k].record()
            k += 1

        mark()
        self.model.set_params_device(self.master)          # a1: FP64 master -> sampling copy
        self.model.prepare(self.dtype)
        mark()
        nqs.nqs_sample(self.model, self.cfg, self.state, self.samples, None, self.acc)   # a2-a6
        mark()
        nqs.nqs_local_energy(self.model, self.ham, self.samples, self.eloc, "f32")       # a7
        mark()
        nqs.nqs_energy_stats(self.eloc, self.C, self.stats)                              # a9 (energy)
        mark()
        last = self.samples[self.S - 1]
        nqs.nqs_logpsi_grad(self.model, last, O=self.O)                                  # a8
        mark()
        nqs.nqs_forces(self.O, self.eloc[(self.S - 1) * self.C:], self.F)                # a9 (forces)
        mark()
        nqs.nqs_gram(self.O, 1, self.T)                                                  # a9 (T = Obar Obar^T / n)
        mark()

    def timed(self, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.run()
        torch.cuda.synchronize()
        n_ev = len(self.phase_names) + 1
        all_ev = [[torch.cuda.Event(enable_timing=True) for _ in range(n_ev)] for _ in range(steps)]
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
        return wall, phases, step_ms


def cpu_baseline(wl, params, budget_s=20.0):
    """The oracle (FP64, full forward per proposal) on a bounded sample of the workload."""
    import oracle
    oracle.build()
    om = oracle.model_from_workload(wl, params, "f64")
    threads = oracle.num_threads()
    N = wl.model.n_visible
    # calibrate on a small run, then size the measured run to the time budget
    c0 = max(threads, 8)
    t = time.perf_counter()
    oracle.sample(om, oracle.make_cfg(c0, 1, 0, seed=wl.seed))
    per_prop = (time.perf_counter() - t) / (c0 * N)
    chains = int(max(threads, min(wl.n_chains, (0.6 * budget_s) / (per_prop * N * 2))))
    sweeps = int(max(2, min(8, (0.6 * budget_s) / (per_prop * N * chains))))
    cfg = oracle.make_cfg(chains, sweeps, 0, seed=wl.seed)
    t = time.perf_counter()
    _, smp, _, _ = oracle.sample(om, cfg)
    ts = time.perf_counter() - t
    props = chains * sweeps * N
    n_el = max(threads, min(smp.shape[0] * smp.shape[1], int(0.4 * budget_s / (per_prop * N))))
    flat = smp.reshape(-1, N)[:n_el]
    t = time.perf_counter()
    oracle.local_energy(om, wl.ham, flat)
    te = time.perf_counter() - t
    return {"value": props / ts, "unit": "proposals/s", "cores": threads, "kind": "oracle",
            "eloc_samples_per_s": n_el / te,
            "sample": f"{chains} chains x {sweeps} sweeps ({props} proposals, FP64 full forward each) + "
                      f"local energies of {n_el} samples, {wl.name}"}


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported (chains shard "
                                   "by global id, see DESIGN.md)", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import paper_2601_20782_amd as nqs
    import workloads

    wl = workloads.cfg2_tfim_10x10()
    params = workloads.params_for(wl)
    N, C, S, B = wl.model.n_visible, wl.n_chains, wl.n_sweeps, wl.n_burnin
    props = C * (S + B) * N

    main_step = Step(nqs, torch, wl, params, a.dtype, a.lanes, a.refresh)
    wall, phases, step_ms = main_step.timed(a.steps, a.warmup)
    ms = max(float(np.mean(step_ms)), 1e3 * wall / a.steps)
    st = main_step.stats.cpu().numpy()
    acc_rate = float(main_step.acc.sum().item()) / props

    # roofline of the dominant kernel (the sampler): FP32 VALU work of the
    # product-form single flip, per proposal: 3M flops (one FMA + one multiply
    # per hidden unit), 4M flops per accepted proposal (tanh update), and the
    # per-sweep refresh theta = W s + b (2 N M flops per N proposals).
    M = wl.model.widths[0]
    flops = props * (3.0 * M + 4.0 * M * acc_rate + 2.0 * M)
    sample_ms = phases["sample"]
    achieved = flops / (sample_ms * 1e-3) / 1e12
    roof = {"kernel": "rbm_sample_kernel", "bound": "alu", "achieved": round(achieved, 2),
            "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4),
            "traffic": None}

    out = {
        "metric": "MH proposals/s + E_loc samples/s, BF16 vs FP32 on 1 GPU, at stated dE vs FP64",
        "value": props / (ms * 1e-3), "unit": "proposals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": a.dtype, "data": "synthetic (seeded random RBM weights, N(0, 0.02^2))",
        "config": {"workload": wl.name, "lattice": "10x10 periodic", "J": 1.0, "h": 3.04, "rbm_hidden": M,
                   "chains": C, "sweeps": S, "burnin": B, "proposals_per_step": props,
                   "samples_per_step": S * C, "parallelism": "single GPU"},
        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
        "sampler_proposals_per_s": props / (sample_ms * 1e-3),
        "eloc_samples_per_s": S * C / (phases["local_energy"] * 1e-3),
        "acceptance": acc_rate,
        "energy": {"mean": st[0], "stderr": st[2], "var": st[1]},
        "roofline": roof,
    }

    if not a.no_compare:
        ref = Step(nqs, torch, wl, params, "f32", a.lanes, a.refresh)
        wall32, phases32, step32 = ref.timed(a.steps, a.warmup)
        ms32 = max(float(np.mean(step32)), 1e3 * wall32 / a.steps)
        st32 = ref.stats.cpu().numpy()
        diff = (main_step.eloc - ref.eloc).contiguous()
        dstats = torch.empty(4, dtype=torch.float64, device=diff.device)
        nqs.nqs_energy_stats(diff, C, dstats)
        d = dstats.cpu().numpy()
        out["fp32"] = {"proposals_per_s": props / (ms32 * 1e-3), "ms_per_step": ms32,
                       "sampler_proposals_per_s": props / (phases32["sample"] * 1e-3),
                       "phases_ms": {k: round(v, 3) for k, v in phases32.items()},
                       "energy": {"mean": st32[0], "stderr": st32[2]}}
        out["speedup_vs_fp32"] = ms32 / ms
        out["dE_vs_fp32"] = {"value": d[0], "stderr_paired": d[2],
                             "note": "same seeds: per-chain paired difference of local energies"}

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, params)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
