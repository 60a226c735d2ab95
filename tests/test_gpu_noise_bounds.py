"""The bound-validation harness on an enumerated system (Sec. IV.A, Eqs.
eq:tv_gaussian and eq:avg_bound).  For random RBMs on the 16-site TFIM chain,
the exact perturbed distribution pi~ = pi e^zeta / Z (zeta from the oracle: the
field the device sampler draws) stays within both total-variation bounds; the
exact biases of <sigma^x> and <Pi_even> stay within 2 max|f| TV; and the shift
of <sigma^x> that the device's noisy sampling estimates agrees with the exact
shift within its Monte Carlo error (chain-mean standard errors)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import exact

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
NOISE_SEED = 20260101


@pytest.fixture(scope="module")
def nqs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20782_amd as m
    m.load()
    return m


@pytest.mark.parametrize("init", [0, 1])
def test_bias_within_the_paper_bounds(nqs, init):
    N, M, C, S = 16, 16, 1024, 256
    p = workloads.rbm_params(N, M, 0.25, 100 + init)
    cfgs = exact.all_configs(N)
    om = oracle.OracleModel("rbm", N, (M,), oracle.round_to(p, "f32"))
    pi, _, _ = exact.enumerate_pi(om)
    ham_x = workloads.Hamiltonian("tfim", workloads.Lattice(1, N), 0.0, 1.0)   # eps = sum_i psi(x^i)/psi(x)
    sx = oracle.local_energy(om, ham_x, cfgs) / N
    even = (np.sum(cfgs > 0, axis=1) % 2 == 0).astype(np.float64)

    model = nqs.Model("rbm", N, (M,), p)
    state = torch.empty(C, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    ex = torch.empty(S * C, dtype=torch.float64, device=DEV)

    def chain_means(sigma):
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=50, seed=7)
        nqs.nqs_sample_noisy(model, cfg, sigma, NOISE_SEED, state, samples)
        nqs.nqs_local_energy(model, nqs.Hamiltonian.from_workload(ham_x), samples.reshape(-1, N), ex)
        return (ex.cpu().numpy() / N).reshape(S, C).mean(axis=0)

    m0 = chain_means(0.0)
    for sg in (0.01, 0.1, 0.3, 1.0):
        pit = exact.perturbed_pi(pi, oracle.noise_zeta(cfgs, sg, NOISE_SEED))
        tv = exact.tv(pi, pit)
        kl_b, avg_b = exact.pinsker_bound(sg), exact.avg_bound(sg)
        assert tv <= min(kl_b, avg_b), (sg, tv, kl_b, avg_b)
        for f in (sx, even):
            assert abs(pit @ f - pi @ f) <= 2.0 * np.max(np.abs(f)) * tv + 1e-12
        m1 = chain_means(sg)
        shift, exact_shift = m1.mean() - m0.mean(), pit @ sx - pi @ sx
        err = np.sqrt(m1.var(ddof=1) / C + m0.var(ddof=1) / C)
        print(f"  init {init} sigma {sg}: TV {tv:.4f} (bounds {kl_b:.4f}, {avg_b:.4f}); <sx> shift sampled "
              f"{shift:+.5f}, exact {exact_shift:+.5f}, s.e. {err:.5f}", flush=True)
        assert abs(shift - exact_shift) <= 4.0 * err
