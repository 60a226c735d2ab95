"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

Each workload is sampled at its full size twice: as the benchmark runs it (no
trace) and with a decision trace of a few chains.  The two runs must give the
same samples (tracing only adds stores), the traced decisions are replayed in
FP64 by the oracle, and local energies of randomly drawn samples are computed
one by one by the oracle.  Every call goes through the C interface."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from bounds import _eloc_error_bound

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


def _sample(nqs, model, cfg, N, trace_chains=0):
    C, S = cfg.n_chains, cfg.n_sweeps
    state = torch.empty(C, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    acc = torch.empty(C, dtype=torch.int64, device=DEV)
    tr = None
    total = (cfg.n_sweeps + cfg.n_burnin) * N
    if trace_chains:
        tr = {"n": trace_chains,
              "site": torch.empty(trace_chains * total, dtype=torch.int32, device=DEV),
              "ubits": torch.empty(trace_chains * total, dtype=torch.int32, device=DEV),
              "delta": torch.empty(trace_chains * total, dtype=torch.float32, device=DEV),
              "accepted": torch.empty(trace_chains * total, dtype=torch.uint8, device=DEV)}
    nqs.nqs_sample(model, cfg, state, samples, None, acc, trace=tr)
    torch.cuda.synchronize()
    out = {"state": state, "samples": samples, "acc": acc}
    if tr:
        for k in ("site", "ubits", "delta", "accepted"):
            out["tr_" + k] = tr[k].cpu().numpy().reshape(trace_chains, total)
    return out


def _replay(wl, params, dtype, r, T, K):
    N = wl.model.n_visible
    om = oracle.model_from_workload(wl, params, dtype)
    ocfg = oracle.make_cfg(wl.n_chains, wl.n_sweeps, wl.n_burnin, move=wl.move, seed=wl.seed)
    starts = np.array([oracle.init_chain(N, wl.move, wl.seed, c) for c in range(T)])
    res = oracle.replay(om, ocfg, list(range(T)), starts, r["tr_site"][:, :K], r["tr_ubits"][:, :K].view(np.uint32),
                        r["tr_delta"][:, :K], r["tr_accepted"][:, :K], tau_rel=1e-5)
    _say(f"  replay of {T} chains x {K} proposals: {res['decisions_equal']} equal, {res['near_ties']} near ties, "
         f"max |dDelta| {res['max_delta_err']:.2e}")
    assert res["site_u_mismatch"] == 0
    assert res["decision_mismatch"] == 0
    return res


def test_tfim10_full_size(nqs):
    """10x10 TFIM, RBM alpha=2: 4096 chains x (100 + 1000) sweeps, BF16 copy, refresh every 4 sweeps."""
    wl = workloads.cfg2_tfim_10x10()
    params = workloads.params_for(wl)
    N, C, S = wl.model.n_visible, wl.n_chains, wl.n_sweeps
    model = nqs.Model.from_workload(wl, params)
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=wl.n_burnin, seed=wl.seed, dtype="bf16",
                           refresh_sweeps=4, move=wl.move)
    _say("tfim10 full size: bench run")
    a = _sample(nqs, model, cfg, N)
    _say("tfim10 full size: traced run")
    b = _sample(nqs, model, cfg, N, trace_chains=4)
    assert torch.equal(a["samples"], b["samples"]) and torch.equal(a["acc"], b["acc"])
    res = _replay(wl, params, "bf16", b, 4, (S + wl.n_burnin) * N)
    assert np.array_equal(res["end_states"], b["state"][:4].cpu().numpy())
    # local energies of all 4.1e6 samples (the bench phase), 64 checked one by one
    ham = nqs.Hamiltonian.from_workload(wl.ham)
    el = torch.empty(S * C, dtype=torch.float64, device=DEV)
    nqs.nqs_local_energy(model, ham, a["samples"], el, "f32")
    torch.cuda.synchronize()
    pick = np.random.default_rng(2).choice(S * C, 64, replace=False)
    smp = a["samples"].reshape(-1, N)[torch.from_numpy(pick).to(DEV)].cpu().numpy()
    om32 = oracle.model_from_workload(wl, params, "f32")
    ref = oracle.local_energy(om32, wl.ham, smp)
    got = el.cpu().numpy()[pick]
    bound = _eloc_error_bound(om32.params, N, wl.model.widths[0], wl.ham.h, smp)
    assert np.all(np.abs(got - ref) <= 2.0 * bound + 1e-12 * np.abs(ref))
    acc_rate = a["acc"].sum().item() / (C * (S + wl.n_burnin) * N)
    assert 0.5 < acc_rate < 1.0


def test_heis10_full_size(nqs):
    """10x10 Heisenberg, FFNN 100-400-200: 16384 chains x (50 + 500) exchange sweeps, BF16."""
    wl = workloads.cfg3_heis_10x10()
    params = workloads.params_for(wl)
    N, C, S = wl.model.n_visible, wl.n_chains, wl.n_sweeps
    model = nqs.Model.from_workload(wl, params)
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=wl.n_burnin, seed=wl.seed, dtype="bf16", move=wl.move,
                           refresh_sweeps=4)
    _say("heis10 full size: bench run")
    a = _sample(nqs, model, cfg, N)
    _say("heis10 full size: traced run")
    b = _sample(nqs, model, cfg, N, trace_chains=2)
    assert torch.equal(a["samples"], b["samples"])
    assert torch.all(a["samples"].sum(dim=2, dtype=torch.int32) == 0)
    _replay(wl, params, "bf16", b, 2, 20000)
    ham = nqs.Hamiltonian.from_workload(wl.ham)
    pick = np.random.default_rng(3).choice(S * C, 24, replace=False)
    smp_d = a["samples"].reshape(-1, N)[torch.from_numpy(pick).to(DEV)].contiguous()
    el = torch.empty(24, dtype=torch.float64, device=DEV)
    nqs.nqs_local_energy(model, ham, smp_d, el, "bf16")
    om = oracle.model_from_workload(wl, params, "bf16")
    smp = smp_d.cpu().numpy()
    ref = oracle.local_energy(om, wl.ham, smp)
    f, _ = om.logamp(smp)
    scale = np.abs(ref) + 2 * 200 + 2 * 200 * np.exp(1.0)
    assert np.all(np.abs(el.cpu().numpy() - ref) < 4e-6 * np.maximum(1.0, np.abs(f)) * scale)
    # the same run writing log|psi| of every sample: the samples are unchanged, and the values carried by the
    # incremental z1 between rebuilds (every 4 sweeps) match the oracle's forward pass of the sampled spins
    _say("heis10 full size: run with log|psi|")
    state = torch.empty(C, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    logpsi = torch.empty(S, C, dtype=torch.float32, device=DEV)
    nqs.nqs_sample(model, cfg, state, samples, logpsi)
    torch.cuda.synchronize()
    assert torch.equal(a["samples"], samples)
    lp = logpsi.reshape(-1)[torch.from_numpy(pick).to(DEV)].cpu().numpy()
    assert np.max(np.abs(lp - f) / np.maximum(1.0, np.abs(f))) < 1e-5


def test_heis20_full_size_sweep(nqs):
    """20x20 Heisenberg, FFNN 400-1600-800-400: 65536 chains, one exchange sweep (the bench step), BF16."""
    wl = workloads.scaled(workloads.cfg5_heis_20x20(), n_sweeps=1, n_burnin=0)
    params = workloads.params_for(wl)
    N, C = wl.model.n_visible, wl.n_chains
    model = nqs.Model.from_workload(wl, params)
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=1, n_burnin=0, seed=wl.seed, dtype="bf16", move=wl.move)
    _say("heis20 full size: bench run")
    a = _sample(nqs, model, cfg, N)
    _say("heis20 full size: traced run")
    b = _sample(nqs, model, cfg, N, trace_chains=2)
    assert torch.equal(a["samples"], b["samples"])
    _replay(wl, params, "bf16", b, 2, N)
    ham = nqs.Hamiltonian.from_workload(wl.ham)
    pick = np.random.default_rng(4).choice(C, 3, replace=False)
    smp_d = a["samples"][0][torch.from_numpy(pick).to(DEV)].contiguous()
    el = torch.empty(3, dtype=torch.float64, device=DEV)
    nqs.nqs_local_energy(model, ham, smp_d, el, "bf16")
    om = oracle.model_from_workload(wl, params, "bf16")
    smp = smp_d.cpu().numpy()
    ref = oracle.local_energy(om, wl.ham, smp)
    f, _ = om.logamp(smp)
    scale = np.abs(ref) + 2 * 800 + 2 * 800 * np.exp(1.0)
    assert np.all(np.abs(el.cpu().numpy() - ref) < 4e-6 * np.maximum(1.0, np.abs(f)) * scale)


@pytest.mark.parametrize("which,n", [("heis10", 16384), ("heis20", 4096)])
def test_factored_T_bench_size(nqs, which, n):
    """T of the sample set the benchmark step forms (16384 samples of the 10x10
    network, 4096 of the 20x20 one), from the factors of O: entries at sampled
    (i, j) against the oracle, whose column means are accumulated over the
    samples in batches of its FP64 log-derivatives."""
    wl = workloads.cfg3_heis_10x10() if which == "heis10" else workloads.cfg5_heis_20x20()
    params = workloads.params_for(wl)
    N, widths = wl.model.n_visible, wl.model.widths
    model = nqs.Model.from_workload(wl, params)
    smp = workloads.random_spins(n, N, 21, zero_mag=True)
    st = torch.from_numpy(smp).to(DEV)
    T = torch.empty(n, n, dtype=torch.float32, device=DEV)
    nqs.nqs_sample_gram_factored(model, st, T)
    torch.cuda.synchronize()
    _say(f"{which}: factored T of {n} samples done; oracle column means")
    om = oracle.OracleModel("ffnn", N, widths, oracle.round_to(params, "f32"), act_dtype="f32")
    mu = np.zeros(model.n_params)
    batch = max(1, (1 << 30) // (8 * model.n_params))
    for k0 in range(0, n, batch):
        _, Ob = oracle.logpsi_grad(om, smp[k0:k0 + batch])
        mu += Ob.sum(axis=0)
        del Ob
    mu /= n
    rng = np.random.default_rng(17)
    pairs = [(0, 0), (n - 1, n - 1), (0, n - 1)] + [tuple(int(v) for v in rng.choice(n, 2)) for _ in range(9)]
    idx = sorted({i for p in pairs for i in p})
    _, Orows = oracle.logpsi_grad(om, smp[idx])
    row = {k: Orows[m] - mu for m, k in enumerate(idx)}
    got = T.cpu().numpy()
    for i, j in pairs:
        ref = float(np.dot(row[i], row[j])) / n
        tol = 1e-5 * np.linalg.norm(row[i]) * np.linalg.norm(row[j]) / n + 1e-9
        assert abs(got[i, j] - ref) < tol, (i, j, got[i, j], ref, tol)
    assert np.array_equal(got[:256, :256], got[:256, :256].T)
    assert np.all(np.diag(got) >= 0)
