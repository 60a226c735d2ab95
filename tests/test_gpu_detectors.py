"""Run-time detectors of the RBM sampler (nqs_sample_checked): non-finite
log-ratios, chains that stop accepting, and the drift of the incremental state
between refreshes.  Each detector is checked against what the decision trace
of the same call, or the oracle, says.  Every call goes through the C
interface."""
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


def _buffers(C, N, S, T, total):
    return {"state": torch.empty(C, N, dtype=torch.int8, device=DEV),
            "samples": torch.empty(S, C, N, dtype=torch.int8, device=DEV),
            "logpsi": torch.empty(S, C, dtype=torch.float32, device=DEV),
            "acc": torch.empty(C, dtype=torch.int64, device=DEV),
            "nonfinite": torch.empty(C, dtype=torch.int64, device=DEV),
            "stuck": torch.empty(C, dtype=torch.int32, device=DEV),
            "drift": torch.empty(C, dtype=torch.float32, device=DEV),
            "trace": {"n": T, "site": torch.empty(T * total, dtype=torch.int32, device=DEV),
                      "ubits": torch.empty(T * total, dtype=torch.int32, device=DEV),
                      "delta": torch.empty(T * total, dtype=torch.float32, device=DEV),
                      "accepted": torch.empty(T * total, dtype=torch.uint8, device=DEV)}}


def _checked(nqs, model, cfg, b, stuck_after=0):
    return nqs.nqs_sample_checked(model, cfg, b["state"], b["samples"], b["logpsi"], b["acc"], trace=b["trace"],
                                  stuck_after=stuck_after, nonfinite=b["nonfinite"], longest_stuck=b["stuck"],
                                  drift=b["drift"])


def _longest_dry_run(accepted, N):
    """Longest run of sweeps (N proposals each) without an accepted move, from a decision trace."""
    per_sweep = accepted.reshape(-1, N).any(axis=1)
    best = run = 0
    for a in per_sweep:
        run = 0 if a else run + 1
        best = max(best, run)
    return best


def test_regular_run_is_quiet_and_unchanged(nqs):
    """The 10x10 TFIM RBM (alpha = 2, BF16 copy), 512 chains x (10 + 20) sweeps, refresh every 4 sweeps: no
    non-finite log-ratio, no stuck chain, a drift of log psi between refreshes (400 accumulated FP32 log-ratios)
    within 1e-4 max(1, |log psi|), and samples, log psi, acceptances and traces equal to nqs_sample's."""
    wl = workloads.cfg2_tfim_10x10()
    params = workloads.params_for(wl)
    N, C, S, B, T = 100, 512, 20, 10, 4
    model = nqs.Model.from_workload(wl, params)
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=wl.seed, dtype="bf16", refresh_sweeps=4)
    total = (S + B) * N
    b = _buffers(C, N, S, T, total)
    r = _checked(nqs, model, cfg, b)
    ref = _buffers(C, N, S, T, total)
    nqs.nqs_sample(model, cfg, ref["state"], ref["samples"], ref["logpsi"], ref["acc"], trace=ref["trace"])
    torch.cuda.synchronize()
    _say(f"  summary {r}; mean |log psi| {b['logpsi'].abs().mean().item():.1f}")
    assert r["status"] == 0 and r["total_nonfinite"] == 0 and r["chains_stuck"] == 0
    assert 0.0 <= r["max_drift"] <= 1e-4 * max(1.0, float(b["logpsi"].abs().max().item()))
    assert float(b["drift"].max().item()) == r["max_drift"]
    for key in ("state", "samples", "logpsi", "acc"):
        assert torch.equal(b[key], ref[key]), key
    for key in ("site", "ubits", "delta", "accepted"):
        assert torch.equal(b["trace"][key], ref["trace"][key]), key
    model.close()


def test_nonfinite_hidden_bias_is_counted_and_every_move_rejected(nqs):
    """A NaN hidden bias written into the device parameters (no host check sees it): every log-ratio is NaN, so
    every proposal is counted and rejected, the call reports NQS_ENUMERIC, and the oracle, whose log psi is NaN
    for every configuration, rejects every traced decision too."""
    N, M, C, S, B, T = 16, 16, 64, 3, 2, 4
    p = workloads.rbm_params(N, M, 0.1, 5)
    model = nqs.Model("rbm", N, (M,), p)
    bad = p.copy()
    bad[N + 3] = np.nan   # b_3
    model.set_params_device(torch.from_numpy(bad).to(DEV))
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=9, dtype="f32")
    total = (S + B) * N
    b = _buffers(C, N, S, T, total)
    r = _checked(nqs, model, cfg, b)
    torch.cuda.synchronize()
    _say(f"  summary {r}")
    assert r["status"] == 5
    assert r["total_nonfinite"] == C * total
    assert torch.all(b["nonfinite"] == total) and torch.all(b["acc"] == 0)
    start = np.array([oracle.init_chain(N, "flip", 9, c) for c in range(C)])
    assert np.array_equal(b["state"].cpu().numpy(), start)
    om = oracle.OracleModel("rbm", N, (M,), bad)
    tr = {k: b["trace"][k].cpu().numpy().reshape(T, total) for k in ("site", "ubits", "delta", "accepted")}
    res = oracle.replay(om, oracle.make_cfg(C, S, B, seed=9), list(range(T)), start[:T], tr["site"],
                        tr["ubits"].view(np.uint32), tr["delta"], tr["accepted"], tau_rel=1e-5)
    assert res["site_u_mismatch"] == 0 and res["decision_mismatch"] == 0 and res["decisions_equal"] == T * total
    assert not np.any(np.isfinite(tr["delta"]))
    model.close()


def test_chains_that_stop_accepting_are_flagged(nqs):
    """Visible biases a_i = 3 on the 16-site chain: once a chain has aligned its spins, a flip costs a factor
    e^-12 in |psi|^2 and the chain stops moving.  The longest dry run per chain equals the one read from the
    decision trace, every chain is flagged at 10 sweeps, and a weak-bias model flags none."""
    N, M, C, S, B, T = 16, 8, 128, 40, 0, 8
    p = workloads.rbm_params(N, M, 0.05, 6)
    p[:N] = 3.0
    total = (S + B) * N
    for label, params, want_all in (("strong bias", p, True), ("weak bias", workloads.rbm_params(N, M, 0.05, 6), False)):
        model = nqs.Model("rbm", N, (M,), params)
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=10, dtype="f32")
        b = _buffers(C, N, S, T, total)
        r = _checked(nqs, model, cfg, b, stuck_after=10)
        torch.cuda.synchronize()
        stuck = b["stuck"].cpu().numpy()
        acc = b["trace"]["accepted"].cpu().numpy().reshape(T, total)
        from_trace = [_longest_dry_run(acc[c], N) for c in range(T)]
        _say(f"  {label}: {r}; longest dry runs (first chains) {stuck[:T].tolist()}")
        assert stuck[:T].tolist() == from_trace
        assert r["chains_stuck"] == int((stuck >= 10).sum())
        if want_all:
            assert r["chains_stuck"] == C
        else:
            assert r["chains_stuck"] == 0
        model.close()


def test_detectors_reject_other_networks(nqs):
    wl = workloads.cfg3_heis_10x10()
    model = nqs.Model.from_workload(wl, workloads.params_for(wl))
    state = torch.empty(4, 100, dtype=torch.int8, device=DEV)
    with pytest.raises(nqs.NqsError):
        nqs.nqs_sample_checked(model, nqs.SampleConfig(n_chains=4, n_sweeps=1, move="exchange"), state)
    model.close()
