"""GPU parity of the noisy-target sampler (Sec. IV.A, Eq. eq:pert_chain): its
histogram against the exactly enumerated pi~ = pi e^zeta / Z with the oracle's
zeta(x), and its determinism.  Every call goes through the C interface."""
import numpy as np
import pytest
import scipy.stats
import torch

import oracle
import workloads
from oracle import exact

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def nqs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20782_amd as m
    m.load()
    return m


def _run(nqs, model, cfg, N, sigma, seed):
    state = torch.empty(cfg.n_chains, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(cfg.n_sweeps, cfg.n_chains, N, dtype=torch.int8, device=DEV)
    acc = torch.empty(cfg.n_chains, dtype=torch.int64, device=DEV)
    nqs.nqs_sample_noisy(model, cfg, sigma, seed, state, samples, None, acc)
    torch.cuda.synchronize()
    return samples.cpu().numpy(), acc.cpu().numpy()


@pytest.mark.parametrize("sigma,seed", [(0.5, 11), (1.0, 13), (1.5, 12)])
def test_noisy_histogram_matches_exact_perturbed_pi(nqs, sigma, seed):
    """Up to sigma = 1.5 the single-flip chains equilibrate in 40 sweeps; at
    sigma = 3 pi~ is concentrated on a few configurations separated by
    low-probability ones and chains stay where they started (the loss of
    ergodicity the paper describes for large noise), so no finite run is held
    to pi~ there."""
    n = 8
    p = workloads.rbm_params(n, 8, 0.3, 21)
    model = nqs.Model("rbm", n, (8,), p)
    # 16384 independent chains, every 10th of 100 sweeps kept: close to independent draws even
    # where the noise slows mixing
    cfg = nqs.SampleConfig(n_chains=16384, n_sweeps=100, n_burnin=40, seed=3)
    smp, _ = _run(nqs, model, cfg, n, sigma, seed)
    smp = smp[9::10]
    pi, _, _ = exact.enumerate_pi(oracle.OracleModel("rbm", n, (8,), oracle.round_to(p, "f32")))
    pit = exact.perturbed_pi(pi, oracle.noise_zeta(exact.all_configs(n), sigma, seed))
    idx = np.sum((smp.reshape(-1, n) > 0).astype(np.int64) << np.arange(n), axis=1)
    counts = np.bincount(idx, minlength=2 ** n)
    e = pit * counts.sum()
    keep = e > 5
    chi2 = np.sum((counts[keep] - e[keep]) ** 2 / e[keep])
    print(f"  sigma={sigma}: chi2/dof = {chi2 / (keep.sum() - 1):.3f}, TV(sampled, pi~) = "
          f"{exact.tv(pit, counts / counts.sum()):.4f}, TV(pi, pi~) = {exact.tv(pi, pit):.4f}", flush=True)
    assert scipy.stats.chi2.sf(chi2, keep.sum() - 1) > 1e-5
    assert exact.tv(pit, counts / counts.sum()) < 0.03
    # and it is not the noiseless distribution
    assert exact.tv(pi, pit) > 0.05 and exact.tv(pi, counts / counts.sum()) > 0.04


def test_noisy_sampler_zero_sigma_and_launch_shape(nqs):
    n, M = 20, 40
    p = workloads.rbm_params(n, M, 0.1, 2)
    model = nqs.Model("rbm", n, (M,), p)
    base = dict(n_chains=300, n_sweeps=6, n_burnin=3, seed=9)
    a, _ = _run(nqs, model, nqs.SampleConfig(**base), n, 0.0, 5)
    state = torch.empty(300, n, dtype=torch.int8, device=DEV)
    ref = torch.empty(6, 300, n, dtype=torch.int8, device=DEV)
    nqs.nqs_sample(model, nqs.SampleConfig(**base), state, ref)
    assert np.array_equal(a, ref.cpu().numpy())                       # sigma = 0 is the plain sampler
    b16, acc16 = _run(nqs, model, nqs.SampleConfig(lanes_per_chain=16, **base), n, 0.8, 5)
    b32, acc32 = _run(nqs, model, nqs.SampleConfig(lanes_per_chain=32, **base), n, 0.8, 5)
    b64, _ = _run(nqs, model, nqs.SampleConfig(lanes_per_chain=64, **base), n, 0.8, 5)
    assert np.array_equal(b16, b32) and np.array_equal(b16, b64) and np.array_equal(acc16, acc32)
    assert not np.array_equal(a, b16)


def test_noisy_sampler_rejects_unsupported(nqs):
    model = nqs.Model("rbm", 130, (8,), workloads.rbm_params(130, 8, 0.1, 1))
    state = torch.empty(4, 130, dtype=torch.int8, device=DEV)
    with pytest.raises(nqs.NqsError):
        nqs.nqs_sample_noisy(model, nqs.SampleConfig(n_chains=4, n_sweeps=1), 0.5, 1, state)
    model2 = nqs.Model("rbm", 8, (8,), workloads.rbm_params(8, 8, 0.1, 1))
    state2 = torch.empty(4, 8, dtype=torch.int8, device=DEV)
    with pytest.raises(nqs.NqsError):
        nqs.nqs_sample_noisy(model2, nqs.SampleConfig(n_chains=4, n_sweeps=1), -1.0, 1, state2)
