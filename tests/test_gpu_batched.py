"""Uneven RBM instances in one persistent launch, and the measured launch plan.

The persistent launch (mode 0) runs each instance at its own lanes per chain
(32 or 64) and must equal one launch per instance at that width (mode 1); the
traced chains of every instance are replayed against the oracle decision by
decision.  A sampler call with the measured plan must equal a call with the
plan's lanes per chain.  Every call goes through the C interface."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def nqs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20782_amd as m
    m.load()
    return m


def _say(msg):
    print(msg, flush=True)


def _job(nqs, model, wl, k, T, lanes=0):
    N = wl.model.n_visible
    cfg = nqs.SampleConfig(n_chains=wl.n_chains, n_sweeps=wl.n_sweeps, n_burnin=wl.n_burnin, seed=wl.seed,
                           dtype="bf16", instance_id=k, lanes_per_chain=lanes)
    total = (wl.n_sweeps + wl.n_burnin) * N
    return {"model": model, "cfg": cfg,
            "chain_state": torch.zeros(wl.n_chains, N, dtype=torch.int8, device=DEV),
            "samples": torch.empty(wl.n_sweeps, wl.n_chains, N, dtype=torch.int8, device=DEV),
            "logpsi": torch.empty(wl.n_sweeps, wl.n_chains, dtype=torch.float32, device=DEV),
            "n_accepted": torch.empty(wl.n_chains, dtype=torch.int64, device=DEV),
            "trace": {"n": T, "site": torch.empty(T * total, dtype=torch.int32, device=DEV),
                      "ubits": torch.empty(T * total, dtype=torch.int32, device=DEV),
                      "delta": torch.empty(T * total, dtype=torch.float32, device=DEV),
                      "accepted": torch.empty(T * total, dtype=torch.uint8, device=DEV)}}


def _batched_lanes(wl):
    M = wl.model.widths[0]
    return 32 if (M + 31) // 32 <= 8 else 64


def test_batched_instances_replay_and_equal_separate_launches(nqs):
    """12 uneven TFIM instances (6x6 to 16x16, alpha 1 to 4: 32 and 64 lanes, the table in LDS and through L2,
    K from 2 to 16), 64 chains x (2 + 3) sweeps each, 4 traced chains per instance."""
    insts = [workloads.scaled(w, n_sweeps=3, n_burnin=2) for w in workloads.cfg4_instances(seed=4, n_inst=12, chains=64)]
    assert {_batched_lanes(w) for w in insts} == {32, 64}
    T = 4
    models = [nqs.Model.from_workload(wl) for wl in insts]
    jobs0 = [_job(nqs, models[k], wl, k, T) for k, wl in enumerate(insts)]
    jobs1 = [_job(nqs, models[k], wl, k, T) for k, wl in enumerate(insts)]
    _say("batched mode 0 (persistent) / mode 1 (one launch per instance)")
    nqs.nqs_sample_batched(jobs0, mode=0)
    nqs.nqs_sample_batched(jobs1, mode=1)
    torch.cuda.synchronize()
    for a, b in zip(jobs0, jobs1):
        for key in ("samples", "logpsi", "chain_state", "n_accepted"):
            assert torch.equal(a[key], b[key]), key
        for key in ("site", "ubits", "delta", "accepted"):
            assert torch.equal(a["trace"][key], b["trace"][key]), key
    for k, wl in enumerate(insts):
        N = wl.model.n_visible
        total = (wl.n_sweeps + wl.n_burnin) * N
        j = jobs0[k]
        om = oracle.model_from_workload(wl, None, "bf16")
        ocfg = oracle.make_cfg(wl.n_chains, wl.n_sweeps, wl.n_burnin, seed=wl.seed, instance_id=k)
        starts = np.array([oracle.init_chain(N, "flip", wl.seed, c, instance=k) for c in range(T)])
        tr = {key: j["trace"][key].cpu().numpy().reshape(T, total) for key in ("site", "ubits", "delta", "accepted")}
        res = oracle.replay(om, ocfg, list(range(T)), starts, tr["site"], tr["ubits"].view(np.uint32), tr["delta"],
                            tr["accepted"], tau_rel=1e-5)
        _say(f"  {wl.name} (G = {_batched_lanes(wl)}): {res['decisions_equal']} equal, {res['near_ties']} near ties, "
             f"max |dDelta| {res['max_delta_err']:.2e}")
        assert res["site_u_mismatch"] == 0
        assert res["decision_mismatch"] == 0
        assert np.array_equal(res["end_states"], j["chain_state"].cpu().numpy()[:T])
    for m in models:
        m.close()


def test_batched_explicit_lanes_equal_single_launch(nqs):
    """An instance that would run at 32 lanes, forced to 64 in the batch, equals nqs_sample at 64 lanes."""
    wl = workloads.scaled(workloads.cfg4_instances(seed=4, n_inst=3, chains=64)[2], n_sweeps=2, n_burnin=1)
    assert _batched_lanes(wl) == 32
    m = nqs.Model.from_workload(wl)
    j = _job(nqs, m, wl, 2, 2, lanes=64)
    nqs.nqs_sample_batched([j], mode=0)
    N = wl.model.n_visible
    cfg = nqs.SampleConfig(n_chains=wl.n_chains, n_sweeps=wl.n_sweeps, n_burnin=wl.n_burnin, seed=wl.seed,
                           dtype="bf16", instance_id=2, lanes_per_chain=64)
    st = torch.zeros(wl.n_chains, N, dtype=torch.int8, device=DEV)
    sm = torch.empty(wl.n_sweeps, wl.n_chains, N, dtype=torch.int8, device=DEV)
    nqs.nqs_sample(m, cfg, st, sm)
    torch.cuda.synchronize()
    assert torch.equal(j["samples"], sm) and torch.equal(j["chain_state"], st)
    m.close()


def test_tuned_plan_is_cached_and_reproducible(nqs):
    """The measured plan for the 10x10 TFIM RBM at 4096 chains: a valid (G, K, chains per block, table placement),
    the same on the second query, and a tuned sampler call equals a call at the plan's lanes per chain."""
    wl = workloads.cfg2_tfim_10x10()
    params = workloads.params_for(wl)
    N, M = wl.model.n_visible, wl.model.widths[0]
    m = nqs.Model.from_workload(wl, params)
    cfg_t = nqs.SampleConfig(n_chains=4096, n_sweeps=2, n_burnin=1, seed=wl.seed, dtype="bf16",
                             lanes_per_chain=nqs.LANES_TUNED, refresh_sweeps=4)
    _say("tuning the 10x10 RBM sampler at 4096 chains")
    p1 = nqs.nqs_sample_plan(m, cfg_t)
    p2 = nqs.nqs_sample_plan(m, cfg_t)
    _say(f"  plan {p1}")
    assert p1 == p2 and p1["tuned"]
    G = p1["lanes_per_chain"]
    assert G in (16, 32, 64) and p1["units_per_lane"] == (M + G - 1) // G
    assert 1 <= p1["chains_per_block"] <= {16: 256, 32: 512, 64: 1024}[G] // G
    assert p1["tuned_ms"] > 0.0
    rule = nqs.nqs_sample_plan(m, nqs.SampleConfig(n_chains=4096, n_sweeps=2, dtype="bf16"))
    assert not rule["tuned"] and rule["lanes_per_chain"] == 32 and rule["table_in_lds"]
    outs = []
    for lanes in (nqs.LANES_TUNED, G):
        cfg = nqs.SampleConfig(n_chains=4096, n_sweeps=2, n_burnin=1, seed=wl.seed, dtype="bf16",
                               lanes_per_chain=lanes, refresh_sweeps=4)
        st = torch.zeros(4096, N, dtype=torch.int8, device=DEV)
        sm = torch.empty(2, 4096, N, dtype=torch.int8, device=DEV)
        lp = torch.empty(2, 4096, dtype=torch.float32, device=DEV)
        nqs.nqs_sample(m, cfg, st, sm, lp)
        outs.append((st, sm, lp))
    torch.cuda.synchronize()
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    m.close()


def test_tuned_batch_is_one_of_the_fixed_widths(nqs):
    """A batch with every instance tuned: both modes give identical results (the assignment is measured once and
    cached), and each instance equals a single launch at 32 or at 64 lanes per chain."""
    insts = [workloads.scaled(w, n_sweeps=2, n_burnin=1) for w in workloads.cfg4_instances(seed=4, n_inst=12, chains=64)]
    insts = [w for w in insts if (w.model.widths[0] + 31) // 32 <= 8][:4]   # instances that allow both widths
    models = [nqs.Model.from_workload(wl) for wl in insts]
    jobs0 = [_job(nqs, models[k], wl, k, 1, lanes=nqs.LANES_TUNED) for k, wl in enumerate(insts)]
    jobs1 = [_job(nqs, models[k], wl, k, 1, lanes=nqs.LANES_TUNED) for k, wl in enumerate(insts)]
    _say("tuned batch: mode 0 / mode 1")
    nqs.nqs_sample_batched(jobs0, mode=0)
    nqs.nqs_sample_batched(jobs1, mode=1)
    torch.cuda.synchronize()
    for k, wl in enumerate(insts):
        for key in ("samples", "logpsi", "chain_state", "n_accepted"):
            assert torch.equal(jobs0[k][key], jobs1[k][key]), key
        N = wl.model.n_visible
        match = []
        for G in (32, 64):
            cfg = nqs.SampleConfig(n_chains=wl.n_chains, n_sweeps=wl.n_sweeps, n_burnin=wl.n_burnin, seed=wl.seed,
                                   dtype="bf16", instance_id=k, lanes_per_chain=G)
            st = torch.zeros(wl.n_chains, N, dtype=torch.int8, device=DEV)
            lp = torch.empty(wl.n_sweeps, wl.n_chains, dtype=torch.float32, device=DEV)
            nqs.nqs_sample(models[k], cfg, st, None, lp)
            torch.cuda.synchronize()
            match.append(torch.equal(st, jobs0[k]["chain_state"]) and torch.equal(lp, jobs0[k]["logpsi"]))
        _say(f"  {wl.name}: equals the 32-lane launch {match[0]}, the 64-lane launch {match[1]}")
        assert any(match)
    for m in models:
        m.close()
