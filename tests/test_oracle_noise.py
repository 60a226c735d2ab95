"""Pins of the oracle's noisy-target perturbation zeta(x) (Sec. IV.A, Eq.
eq:pert_chain): a normal of standard deviation sigma, fixed per configuration."""
import numpy as np
import scipy.stats

import oracle
from oracle import exact


def test_zeta_is_normal_over_the_hilbert_space():
    """Over all 2^16 configurations: KS against N(0, sigma^2), mean and spread."""
    cfgs = exact.all_configs(16)
    for sigma, seed in [(1.0, 7), (0.25, 123456789012345)]:
        z = oracle.noise_zeta(cfgs, sigma, seed)
        assert scipy.stats.kstest(z / sigma, "norm").pvalue > 1e-3
        assert abs(z.mean()) < 5 * sigma / np.sqrt(z.size)
        assert abs(z.std() / sigma - 1.0) < 0.02
        # Box-Muller on the 2^-24 grid: |g| <= sqrt(2 ln 2^24)
        assert np.max(np.abs(z)) <= sigma * np.sqrt(2 * 24 * np.log(2)) + 1e-12


def test_zeta_is_fixed_per_configuration():
    cfgs = exact.all_configs(10)
    a = oracle.noise_zeta(cfgs, 0.7, 3)
    assert np.array_equal(a, oracle.noise_zeta(cfgs, 0.7, 3))        # same x, same value
    assert np.array_equal(a[::-1], oracle.noise_zeta(cfgs[::-1], 0.7, 3))
    assert not np.allclose(a, oracle.noise_zeta(cfgs, 0.7, 4))       # the seed matters
    assert np.unique(a).size == a.size                               # distinct configurations differ
    # sites beyond the first word enter the counter
    rng = np.random.default_rng(1)
    x = (2 * rng.integers(0, 2, size=(1, 100)) - 1).astype(np.int8)
    y = x.copy()
    y[0, 77] = -y[0, 77]
    assert oracle.noise_zeta(x, 1.0, 5)[0] != oracle.noise_zeta(y, 1.0, 5)[0]


def test_zeta_scales_with_sigma():
    cfgs = exact.all_configs(8)
    assert np.allclose(oracle.noise_zeta(cfgs, 2.0, 9), 2.0 * oracle.noise_zeta(cfgs, 1.0, 9), rtol=1e-15, atol=0)
