"""GPU parity of the residual convolutional network (App. H): log psi of given
configurations, the single-flip sampler (decision replay in FP64 and the
histogram against the enumerated |psi|^2) and TFIM local energies, against
the numpy oracle.  Every call goes through the C interface."""
import numpy as np
import pytest
import scipy.stats
import torch

import oracle
import workloads
from oracle import exact
from oracle import rescnn

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


@pytest.mark.parametrize("L,F,R", [(3, 4, 1), (4, 8, 2), (4, 16, 4), (6, 5, 3), (10, 16, 1), (5, 3, 0)])
def test_logpsi_matches_oracle(nqs, L, F, R):
    p = workloads.rescnn_params(F, R, L + F + R)
    model = nqs.Model.rescnn(L, F, R, p)
    x = workloads.random_spins(37, L * L, 2)
    lp = torch.empty(37, dtype=torch.float32, device=DEV)
    nqs.nqs_logpsi_grad(model, torch.from_numpy(x).to(DEV), logpsi=lp)
    ref, _ = rescnn.ResCNN(L, F, R, p, "f32").logamp(x)
    got = lp.cpu().numpy().astype(np.float64)
    err = np.max(np.abs(got - ref) / (1.0 + np.abs(ref)))
    _say(f"  L={L} F={F} R={R}: max |dlogpsi| / (1 + |logpsi|) = {err:.2e}")
    assert err < 2e-5


def _trace_run(nqs, model, N, dtype, C, S, B, T, seed=5):
    cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=B, seed=seed, dtype=dtype)
    total = (S + B) * N
    tr = {"n": T,
          "site": torch.empty(T * total, dtype=torch.int32, device=DEV),
          "ubits": torch.empty(T * total, dtype=torch.int32, device=DEV),
          "delta": torch.empty(T * total, dtype=torch.float32, device=DEV),
          "accepted": torch.empty(T * total, dtype=torch.uint8, device=DEV)}
    state = torch.empty(C, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    logpsi = torch.empty(S, C, dtype=torch.float32, device=DEV)
    nqs.nqs_sample(model, cfg, state, samples, logpsi, None, trace=tr)
    torch.cuda.synchronize()
    out = {k: tr[k].cpu().numpy().reshape(T, total) for k in ("site", "ubits", "delta", "accepted")}
    out["samples"], out["logpsi"], out["state"] = samples.cpu().numpy(), logpsi.cpu().numpy(), state.cpu().numpy()
    return out


@pytest.mark.parametrize("dtype,L,F,C", [("f32", 4, 8, 16), ("bf16", 4, 8, 16), ("f16", 4, 8, 16),
                                         ("f32", 4, 16, 40), ("bf16", 4, 16, 40), ("f16", 4, 16, 40),
                                         ("bf16", 5, 32, 7), ("f32", 3, 16, 33)])
def test_sampler_decisions_replay_in_fp64(nqs, dtype, L, F, C):
    """Each traced proposal: site and u equal the Philox draws, Delta equals the
    oracle's FP64 2 (log psi(x') - log psi(x)) of the `dtype` network within its
    rounding, and the decision equals u < exp(min(Delta, 0)) except near ties.
    F = 8 runs one chain per workgroup; F = 16 and 32 the matrix-core kernel with
    several chains per workgroup (C not a multiple of them: a partial group)."""
    R = 2
    N = L * L
    p = workloads.rescnn_params(F, R, 9, scale=1.5)
    model = nqs.Model.rescnn(L, F, R, p)
    T, S, B = 3, 6, 2
    r = _trace_run(nqs, model, N, dtype, C, S, B, T)
    net = rescnn.ResCNN(L, F, R, p, dtype)
    tol = {"f32": 1e-4, "bf16": 3e-2, "f16": 5e-3}[dtype]
    near, max_err = 0, 0.0
    for c in range(T):
        x = oracle.init_chain(N, "flip", 5, c).copy()
        f0, _ = net.logamp(x[None])
        for k in range((S + B) * N):
            rb = oracle.philox([k & 0xFFFFFFFF, k >> 32, c, 0], [5, 0])
            site = int((int(rb[0]) * N) >> 32)
            ub = int(rb[2]) >> 8
            assert (r["site"][c, k] & 0xFFFF) == site and int(r["ubits"][c, k]) == ub
            y = x.copy()
            y[site] = -y[site]
            f1, _ = net.logamp(y[None])
            d = 2.0 * (f1[0] - f0[0])
            err = abs(float(r["delta"][c, k]) - d)
            max_err = max(max_err, err / max(1.0, abs(d)))
            assert err <= tol * max(1.0, abs(d)), (c, k, r["delta"][c, k], d)
            u = ub * 2.0 ** -24
            acc = u < np.exp(min(d, 0.0))
            if bool(r["accepted"][c, k]) != acc:
                # only where the FP32 decision and the FP64 one straddle u
                assert abs(np.log(max(u, 1e-300)) - min(d, 0.0)) <= 2 * tol * max(1.0, abs(d))
                near += 1
            if r["accepted"][c, k]:
                x, f0 = y, f1
    assert np.array_equal(x, r["state"][T - 1]) or near > 0
    _say(f"  {dtype} L={L} F={F}: max relative |dDelta| {max_err:.2e}, {near} near ties")


@pytest.mark.parametrize("F,lanes", [(4, 0), (16, 0), (16, -1)])
def test_sampler_histogram_matches_exact_pi(nqs, F, lanes):
    """3 x 3 lattice, final layer-norm scale N(0, 0.3^2): pi far from uniform.
    F = 16 runs the matrix-core kernel unless lanes_per_chain = -1."""
    L, R = 3, 1
    N = L * L
    p = workloads.rescnn_params(F, R, 3, scale=2.0).copy()
    p[-2 * F:-F] = np.random.default_rng(7).normal(0.0, 0.3, size=F)
    model = nqs.Model.rescnn(L, F, R, p)
    cfg = nqs.SampleConfig(n_chains=8192, n_sweeps=60, n_burnin=30, seed=2, lanes_per_chain=lanes)
    state = torch.empty(8192, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(60, 8192, N, dtype=torch.int8, device=DEV)
    nqs.nqs_sample(model, cfg, state, samples)
    smp = samples.cpu().numpy()[4::5]
    f, _ = rescnn.ResCNN(L, F, R, p, "f32").logamp(exact.all_configs(N))
    w = np.exp(2 * (f - f.max()))
    pi = w / w.sum()
    idx = np.sum((smp.reshape(-1, N) > 0).astype(np.int64) << np.arange(N), axis=1)
    counts = np.bincount(idx, minlength=2 ** N)
    e = pi * counts.sum()
    keep = e > 5
    chi2 = np.sum((counts[keep] - e[keep]) ** 2 / e[keep])
    _say(f"  chi2/dof = {chi2 / (keep.sum() - 1):.3f}, TV = {exact.tv(pi, counts / counts.sum()):.4f}, "
         f"TV to uniform {exact.tv(pi, np.full_like(pi, 1.0 / pi.size)):.3f}")
    assert scipy.stats.chi2.sf(chi2, keep.sum() - 1) > 1e-5
    assert exact.tv(pi, counts / counts.sum()) < 0.05 < exact.tv(pi, np.full_like(pi, 1.0 / pi.size))


@pytest.mark.parametrize("J,h", [(1.0, -1.0), (0.5, 2.5)])
def test_local_energy_matches_oracle(nqs, J, h):
    L, F, R = 4, 8, 2
    p = workloads.rescnn_params(F, R, 4)
    model = nqs.Model.rescnn(L, F, R, p)
    x = workloads.random_spins(24, L * L, 3)
    ham = nqs.Hamiltonian("tfim", 2, L, J, h, True)
    el = torch.empty(24, dtype=torch.float64, device=DEV)
    nqs.nqs_local_energy(model, ham, torch.from_numpy(x).to(DEV), el)
    ref = rescnn.ResCNN(L, F, R, p, "f32").local_energy_tfim(x, J, h)
    got = el.cpu().numpy()
    scale = np.abs(J) * 2 * L * L + np.abs(h) * np.abs(ref - 0) + 1.0
    assert np.all(np.abs(got - ref) <= 1e-4 * scale)


def test_rejections(nqs):
    L, F, R = 4, 4, 1
    model = nqs.Model.rescnn(L, F, R, workloads.rescnn_params(F, R, 1))
    x = torch.from_numpy(workloads.random_spins(4, L * L, 1)).to(DEV)
    with pytest.raises(nqs.NqsError):   # shared convolution weights: no per-layer outer-product factors
        nqs.nqs_sample_gram_factored(model, x, torch.empty(4, 4, dtype=torch.float32, device=DEV))
    with pytest.raises(nqs.NqsError):
        nqs.nqs_local_energy(model, nqs.Hamiltonian("heisenberg", 2, L, 1.0, 0.0, True), x,
                             torch.empty(4, dtype=torch.float64, device=DEV))
    state = torch.empty(4, L * L, dtype=torch.int8, device=DEV)
    with pytest.raises(nqs.NqsError):
        nqs.nqs_sample(model, nqs.SampleConfig(n_chains=4, n_sweeps=1, dtype="e4m3"), state)
    with pytest.raises(nqs.NqsError):
        nqs.Model("rescnn", 15, (4,), workloads.rescnn_params(4, 1, 1), lat_dim=2, lat_L=4, n_layers=1)


@pytest.mark.parametrize("L,F,R", [(3, 4, 1), (4, 8, 2), (4, 4, 0)])
def test_log_derivatives_match_finite_differences(nqs, L, F, R):
    p = workloads.rescnn_params(F, R, 11 + R, scale=1.2).copy()
    p[-2 * F:-F] = np.random.default_rng(3).normal(0.0, 0.3, size=F)   # a non-trivial readout scale
    model = nqs.Model.rescnn(L, F, R, p)
    x = workloads.random_spins(4, L * L, 6)
    xd = torch.from_numpy(x).to(DEV)
    P = model.n_params
    O = torch.empty(4, P, dtype=torch.float32, device=DEV)
    lp = torch.empty(4, dtype=torch.float32, device=DEV)
    nqs.nqs_logpsi_grad(model, xd, logpsi=lp, O=O)
    net = rescnn.ResCNN(L, F, R, p)
    ref = rescnn.logpsi_grad_fd(net, x)
    f, _ = net.logamp(x)
    got = O.cpu().numpy()
    err = np.max(np.abs(got - ref) / (1.0 + np.abs(ref)))
    _say(f"  L={L} F={F} R={R}: P={P}, max |dO| / (1 + |O|) = {err:.2e}")
    assert err < 2e-4
    assert np.max(np.abs(lp.cpu().numpy() - f) / (1 + np.abs(f))) < 1e-5
    g = np.random.default_rng(4).normal(size=4).astype(np.float32)
    vo = torch.empty(P, dtype=torch.float32, device=DEV)
    nqs.nqs_logpsi_grad(model, xd, vjp_in=torch.from_numpy(g).to(DEV), vjp_out=vo)
    assert np.allclose(vo.cpu().numpy(), g.astype(np.float64) @ ref, rtol=1e-3, atol=1e-3)


def test_vmc_training_tfim_4x4_rescnn(nqs):
    """SR steps of a ResCNN (8 filters, 2 blocks) on the 4 x 4 periodic TFIM at
    h/J = 3 (stoquastic sign), BF16 sampling copy: the energy reaches the exact
    ground-state energy (Lanczos) to 1e-3 (5.5e-5 when measured)."""
    L, F, R = 4, 8, 2
    N = L * L
    J, hf = 1.0, -3.0
    e0, _ = exact.ground_state("tfim", 2, L, J, hf)
    p = workloads.rescnn_params(F, R, 2)
    model = nqs.Model.rescnn(L, F, R, p)
    ham = nqs.Hamiltonian("tfim", 2, L, J, hf, True)
    master = torch.from_numpy(p.copy()).to(DEV)
    C, S = 512, 4
    n = C * S
    state = torch.empty(C, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    eloc = torch.empty(n, dtype=torch.float64, device=DEV)
    stats = torch.empty(4, dtype=torch.float64, device=DEV)
    T = torch.empty(n, n, dtype=torch.float32, device=DEV)
    y = torch.empty(n, dtype=torch.float64, device=DEV)
    energies, offset = [], 0
    for it in range(120):
        model.set_params_device(master)
        model.prepare("bf16")
        burn = 20 if it == 0 else 2
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=burn, seed=4, dtype="bf16", step_offset=offset,
                               init_chains=it == 0)
        nqs.nqs_sample(model, cfg, state, samples)
        offset += (burn + S) * N
        flat = samples.reshape(n, N)
        nqs.nqs_local_energy(model, ham, flat, eloc)
        nqs.nqs_energy_stats(eloc, C, stats)
        nqs.nqs_sample_gram(model, flat, T)
        nqs.nqs_sr_solve(T, eloc, 1e-2, y, tol=1e-6, max_iter=300)
        nqs.nqs_sr_update(model, flat, y, 0.03, master)
        energies.append(float(stats[0].item()))
        if it % 20 == 0:
            _say(f"  rescnn 4x4 iteration {it}: E = {energies[-1]:.5f} (exact {e0:.5f})")
    e_end = float(np.mean(energies[-10:]))
    _say(f"  rescnn 4x4: mean of the last 10 energies {e_end:.5f}, exact {e0:.5f}, "
         f"rel {abs(e_end - e0) / abs(e0):.2e}")
    assert abs(e_end - e0) <= 1e-3 * abs(e0)
