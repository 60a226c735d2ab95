"""FP8 (E4M3) sampling of dense networks on the FP8 matrix cores, against the oracle's E4M3 reading.

The oracle's reading: every weight tensor scaled by amax/448 and rounded to
E4M3; every hidden-layer output rounded to E4M3 after a power-of-two scale from
a bound over all configurations; products and sums in FP64.  The device adds its
products in FP32, so a layer output that lies within the FP32 accumulation error
of an E4M3 rounding midpoint can round to the neighbouring code, one E4M3 step
(1/8 to 1/16 relative) away from the oracle's.  That happens for a few of the
2400 outputs of a 20x20-network evaluation per hundred evaluations and moves log psi
by up to ~1e-3 relative; it does not bias anything.  So the checks are:
  - the proposal stream (sites, u bits) equals the oracle's bit for bit;
  - log psi of sampled configurations: most within the FP32 tolerance of the
    oracle (1e-5 relative), every one within 1e-2 relative;
  - replayed decisions equal the oracle's except for a small fraction;
  - local energies of 2048 sampled configurations: the mean signed difference
    from the oracle consistent with zero within four of its standard errors (no
    bias), and the per-sample spread of the differences below 1 % of the spread
    of the local energies.  (A flipped layer output changes a connected
    configuration's amplitude ratio by up to ~10 %, and the Heisenberg local
    energy of these unequilibrated random-network samples is dominated by a few
    very large ratios, so FP8 adds per-sample noise; the tenth-of-the-error-bar
    test of the 16-bit formats would measure that noise, not a bias.)
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import dense

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


def _sample(nqs, wl, params, C, S, B, trace=0):
    N = wl.model.n_visible
    model = nqs.Model.from_workload(wl, params)
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=wl.seed, dtype="e4m3", move=wl.move)
    st = torch.empty(C, N, dtype=torch.int8, device=DEV)
    sm = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    lp = torch.empty(S, C, dtype=torch.float32, device=DEV)
    total = (S + B) * N
    tr = None
    if trace:
        tr = {"n": trace, "site": torch.empty(trace * total, dtype=torch.int32, device=DEV),
              "ubits": torch.empty(trace * total, dtype=torch.int32, device=DEV),
              "delta": torch.empty(trace * total, dtype=torch.float32, device=DEV),
              "accepted": torch.empty(trace * total, dtype=torch.uint8, device=DEV)}
    nqs.nqs_sample(model, cfg, st, sm, lp, None, trace=tr)
    torch.cuda.synchronize()
    out = {"model": model, "samples": sm, "logpsi": lp.cpu().numpy()}
    if tr:
        for k in ("site", "ubits", "delta", "accepted"):
            out["tr_" + k] = tr[k].cpu().numpy().reshape(trace, total)
    return out


def _check_logpsi(wl, params, r, S, C, n_pick, seed, frac_fp32):
    N = wl.model.n_visible
    om = oracle.model_from_workload(wl, params, "e4m3")
    assert om.act_dtype == "e4m3" and om.act_scales
    pick = np.sort(np.random.default_rng(seed).choice(C, min(C, n_pick), replace=False))
    smp = r["samples"][S - 1].cpu().numpy()[pick]
    f = dense.logamp_rows(om.params, N, wl.model.widths, smp, act_dtype="e4m3", act_scales=om.act_scales)
    rel = np.abs(r["logpsi"][S - 1][pick] - f) / np.maximum(1.0, np.abs(f))
    _say(f"  log psi: median rel {np.median(rel):.1e}, max {rel.max():.1e}, "
         f"{(rel <= 1e-5).mean():.3f} within 1e-5")
    assert (rel <= 1e-5).mean() >= frac_fp32
    assert rel.max() <= 1e-2
    return om


def _replay(wl, params, om, r, C, S, B, T, max_frac):
    N = wl.model.n_visible
    ocfg = oracle.make_cfg(C, S, B, move=wl.move, seed=wl.seed)
    starts = np.array([oracle.init_chain(N, wl.move, wl.seed, c) for c in range(T)])
    res = oracle.replay(om, ocfg, list(range(T)), starts, r["tr_site"], r["tr_ubits"].view(np.uint32),
                        r["tr_delta"], r["tr_accepted"], tau_rel=1e-5)
    n = res["decisions_equal"] + res["decision_mismatch"] + res["near_ties"]
    _say(f"  replay: {res['decisions_equal']} equal, {res['decision_mismatch']} differ, {res['near_ties']} near ties "
         f"of {n}; max |dDelta| {res['max_delta_err']:.2e}")
    assert res["site_u_mismatch"] == 0
    assert res["decision_mismatch"] <= max_frac * n


def test_fp8_dense_small_network(nqs):
    """10x10 Heisenberg, FFNN 100-400-200, 512 chains x (2 + 2) exchange sweeps."""
    wl = workloads.cfg3_heis_10x10()
    params = workloads.params_for(wl)
    C, S, B, T = 512, 2, 2, 4
    r = _sample(nqs, wl, params, C, S, B, trace=T)
    om = _check_logpsi(wl, params, r, S, C, 256, 1, 0.9)
    _replay(wl, params, om, r, C, S, B, T, 0.01)
    assert torch.all(r["samples"].sum(dim=2, dtype=torch.int32) == 0)   # exchange moves keep the magnetisation
    r["model"].close()


def test_fp8_dense_20x20_bench_shape(nqs):
    """20x20 Heisenberg, FFNN 400-1600-800-400, 65536 chains (the benchmark's launch), four exchange sweeps;
    then the local energies of 2048 sampled configurations."""
    wl = workloads.cfg5_heis_20x20()
    params = workloads.params_for(wl)
    N, C, S, B, T = wl.model.n_visible, wl.n_chains, 1, 3, 2
    _say("heis20 e4m3: 65536 chains x (3 + 1) sweeps")
    r = _sample(nqs, wl, params, C, S, B, trace=T)
    om = _check_logpsi(wl, params, r, S, C, 256, 2, 0.7)
    _replay(wl, params, om, r, C, S, B, T, 0.01)
    # local energies in the E4M3 copy against the oracle's E4M3 reading
    pick = np.sort(np.random.default_rng(41).choice(C, 2048, replace=False))
    smp_d = r["samples"][S - 1][torch.from_numpy(pick).to(DEV)].contiguous()
    ham = nqs.Hamiltonian.from_workload(wl.ham)
    el = torch.empty(2048, dtype=torch.float64, device=DEV)
    nqs.nqs_local_energy(r["model"], ham, smp_d, el, "e4m3")
    torch.cuda.synchronize()
    got = el.cpu().numpy()
    _say("  oracle local energies (batched FP64, E4M3 reading)")
    ref = dense.local_energy(om.params, N, wl.model.widths, wl.ham, smp_d.cpu().numpy(), act_dtype="e4m3",
                             marshall=True, act_scales=om.act_scales)
    d = got - ref
    se = d.std(ddof=1) / np.sqrt(d.size)
    _say(f"  local energies: mean(device - oracle) {d.mean():.3e} (+- {se:.1e}), sd {d.std():.3e}, "
         f"sd of the local energies {ref.std():.3e}")
    assert abs(d.mean()) <= 4.0 * se
    assert d.std() <= 0.01 * ref.std()
    r["model"].close()
