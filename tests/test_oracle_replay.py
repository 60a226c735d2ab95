"""The decision-replay checker flags planted mistakes (CPU only; the mistakes are planted in a trace
written here, never on the GPU)."""
import numpy as np

import oracle
import workloads


def _python_trace(model, n, seed, chains, steps, move="flip"):
    """A step-by-step MH trace built from the oracle's generator and log-amplitude."""
    T = len(chains)
    site = np.zeros((T, steps), np.uint32)
    ubits = np.zeros((T, steps), np.uint32)
    delta = np.zeros((T, steps), np.float32)
    acc = np.zeros((T, steps), np.uint8)
    starts = np.array([oracle.init_chain(n, move, seed, c) for c in chains])
    for t, c in enumerate(chains):
        s = starts[t].copy()
        f = model.logamp(s)[0][0]
        for k in range(steps):
            r = oracle.philox([k, 0, c, 0], [seed & 0xFFFFFFFF, seed >> 32])
            i = int((int(r[0]) * n) >> 32)
            u = (int(r[2]) >> 8) * 2.0 ** -24
            y = s.copy()
            y[i] = -y[i]
            fy = model.logamp(y)[0][0]
            d = 2 * (fy - f)
            a = u < np.exp(min(d, 0.0))
            site[t, k] = i | (0xFFFF << 16)
            ubits[t, k] = int(r[2]) >> 8
            delta[t, k] = d
            acc[t, k] = a
            if a:
                s, f = y, fy
    return starts, site.view(np.int32), ubits, delta, acc


def test_replay_accepts_faithful_trace_and_flags_planted_errors(orc):
    n = 8
    p = workloads.rbm_params(n, 8, 0.5, 3)
    model = oracle.OracleModel("rbm", n, (8,), p)
    chains = [0, 3, 17]
    steps = 160
    cfg = oracle.make_cfg(n_chains=max(chains) + 1, n_sweeps=steps // n, n_burnin=0, seed=4242)
    starts, site, ubits, delta, acc = _python_trace(model, n, 4242, chains, steps)
    res = oracle.replay(model, cfg, chains, starts, site, ubits, delta, acc)
    assert res["site_u_mismatch"] == 0 and res["decision_mismatch"] == 0
    assert res["decisions_equal"] == len(chains) * steps
    assert res["max_delta_err"] < 1e-6
    # the replayed trajectory ends where the free-running oracle sampler ends
    st, _, _, _ = oracle.sample(model, cfg)
    assert np.array_equal(res["end_states"], st[chains])

    # planted mistake 1: a clear decision flipped
    gap = np.abs(np.log(np.maximum(ubits.astype(np.float64) * 2.0 ** -24, 1e-300)) - delta)
    t, k = np.unravel_index(np.argmax(gap[:, :50]), gap[:, :50].shape)
    bad = acc.copy()
    bad[t, k] ^= 1
    r2 = oracle.replay(model, cfg, chains, starts, site, ubits, delta, bad)
    assert r2["decision_mismatch"] >= 1

    # planted mistake 2: a wrong site
    bad_site = site.view(np.uint32).copy()
    bad_site[1, 7] = ((int(bad_site[1, 7]) & 0xFFFF) + 1) % n | (0xFFFF << 16)
    bad_site = bad_site.view(np.int32)
    r3 = oracle.replay(model, cfg, chains, starts, bad_site, ubits, delta, acc)
    assert r3["site_u_mismatch"] == 1

    # planted mistake 3: u bits off by one
    bad_u = ubits.copy()
    bad_u[2, 100] ^= 1
    r4 = oracle.replay(model, cfg, chains, starts, site, bad_u, delta, acc)
    assert r4["site_u_mismatch"] == 1
