"""Pins for the oracle's log-derivatives, forces, S matrix, averages and the paper's bounds (CPU only)."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import exact


def _fd_grad(make_model, params, samples, h=1e-6):
    """Central finite differences of log|psi| with respect to every parameter."""
    P = params.size
    out = np.empty((samples.shape[0], P))
    for k in range(P):
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        fp, _ = make_model(pp).logamp(samples)
        fm, _ = make_model(pm).logamp(samples)
        out[:, k] = (fp - fm) / (2 * h)
    return out


def test_rbm_logderivatives_vs_finite_differences(orc):
    n, m = 7, 9
    p = workloads.rbm_params(n, m, 0.4, 2)
    mk = lambda q: oracle.OracleModel("rbm", n, (m,), q)
    smp = workloads.random_spins(5, n, 3)
    lp, O = oracle.logpsi_grad(mk(p), smp)
    fd = _fd_grad(mk, p, smp)
    assert np.max(np.abs(O - fd)) < 1e-7
    assert np.allclose(lp, mk(p).logamp(smp)[0])


def test_ffnn_logderivatives_vs_finite_differences(orc):
    n = 8
    widths = (12, 7, 5)
    p = workloads.ffnn_params(n, widths, 4, bias_std=0.2)
    mk = lambda q: oracle.OracleModel("ffnn", n, widths, q)
    smp = workloads.random_spins(4, n, 5)
    _, O = oracle.logpsi_grad(mk(p), smp)
    fd = _fd_grad(mk, p, smp)
    # skip parameters whose finite difference straddles a ReLU kink
    ok = np.abs(O - fd) < 1e-6
    assert ok.mean() > 0.999
    assert np.max(np.abs(O - fd)[ok]) < 1e-7


def test_forces_equal_half_energy_gradient(orc):
    """Exact F (pi-weighted Eq. eq:forces) equals (1/2) dE/dtheta of the matrix energy for real psi."""
    n = 6
    p = workloads.rbm_params(n, 6, 0.3, 13)
    ham = workloads.Hamiltonian("tfim", workloads.Lattice(1, n), 1.0, 0.8)
    mk = lambda q: oracle.OracleModel("rbm", n, (6,), q)
    model = mk(p)
    cfg = exact.all_configs(n)
    pi, _, _ = exact.enumerate_pi(model)
    el = oracle.local_energy(model, ham, cfg)
    _, O = oracle.logpsi_grad(model, cfg)
    F = oracle.forces(O, el, weights=pi)
    h = 1e-5
    grad = np.empty(p.size)
    for k in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        grad[k] = (exact.exact_energy(mk(pp), "tfim", 1, n, 1.0, 0.8) -
                   exact.exact_energy(mk(pm), "tfim", 1, n, 1.0, 0.8)) / (2 * h)
    assert np.max(np.abs(2 * F - grad)) < 1e-7


def test_smatrix_equals_metric_of_normalised_state(orc):
    """S (pi-weighted Eq. eq:smat) = J^T J, J = d psi_hat / d theta of the normalised real state."""
    n = 5
    p = workloads.rbm_params(n, 4, 0.3, 14)
    mk = lambda q: oracle.OracleModel("rbm", n, (4,), q)
    cfg = exact.all_configs(n)
    pi, _, _ = exact.enumerate_pi(mk(p))
    _, O = oracle.logpsi_grad(mk(p), cfg)
    S = oracle.smatrix(O, weights=pi)
    h = 1e-6
    Jac = np.empty((2 ** n, p.size))
    for k in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        Jac[:, k] = (exact.psi_vector(mk(pp)) - exact.psi_vector(mk(pm))) / (2 * h)
    assert np.max(np.abs(S - Jac.T @ Jac)) < 1e-8
    assert np.min(np.linalg.eigvalsh(S)) > -1e-12


def test_tmatrix_shares_spectrum_with_smatrix(orc):
    rng = np.random.default_rng(1)
    O = rng.normal(size=(12, 30))
    S = oracle.smatrix(O)
    T = oracle.tmatrix(O)
    es = np.sort(np.linalg.eigvalsh(S))[::-1][:12]
    et = np.sort(np.linalg.eigvalsh(T))[::-1]
    assert np.allclose(es, et, atol=1e-10)


def test_sample_forces_match_weighted_definition_on_repeated_samples(orc):
    """Sample means with integer multiplicities equal the weighted means."""
    rng = np.random.default_rng(2)
    O = rng.normal(size=(7, 5))
    e = rng.normal(size=7)
    mult = rng.integers(1, 5, size=7)
    Orep, erep = np.repeat(O, mult, axis=0), np.repeat(e, mult)
    assert np.allclose(oracle.forces(Orep, erep), oracle.forces(O, e, weights=mult.astype(float)), atol=1e-14)
    assert np.allclose(oracle.smatrix(Orep), oracle.smatrix(O, weights=mult.astype(float)), atol=1e-14)


def test_stats_chain_mean_standard_error(orc):
    """Chain c holds the constant c: chain means 0..C-1, stderr = sqrt(C(C+1)/12)/sqrt(C)."""
    C, per = 10, 7
    e = np.tile(np.arange(C, dtype=float), per)          # layout [sweep][chain]
    st = oracle.stats(e, C)
    assert st[0] == pytest.approx((C - 1) / 2)
    assert st[2] == pytest.approx(np.sqrt(C * (C + 1) / 12.0) / np.sqrt(C))
    assert st[3] == C * per


# ---------------------------------------------------------------------------
# The paper's bounds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sigma,mu", [(0.01, 0.0), (0.1, 0.0), (0.5, 0.0), (1.0, 0.0), (0.3, 0.2),
                                      (0.8, -0.5), (2.0, 1.0)])
def test_thm33_closed_form_equals_quadrature(sigma, mu):
    assert abs(exact.avg_bound(sigma, mu) - exact.avg_bound_quadrature(sigma, mu)) < 1e-10


def test_thm33_mu_zero_is_first_order_in_sigma():
    """1 - e^{s^2} erfc(s) = 2 s / sqrt(pi) - s^2 + O(s^3): first order in sigma, not second."""
    for s in (1e-3, 1e-2):
        b = exact.avg_bound(s)
        assert abs(b - (2 * s / np.sqrt(np.pi) - s * s)) < 2 * s ** 3
    # hence it exceeds Pinsker's sigma/2 for small sigma (2/sqrt(pi) > 1/2)
    assert exact.avg_bound(0.01) > exact.pinsker_bound(0.01)


def test_lemma32_pointwise_bound():
    rng = np.random.default_rng(0)
    s = np.exp(rng.uniform(-8, 8, 10 ** 6))
    eps = rng.normal(0, 2, 10 ** 6)
    lhs = exact.acceptance_difference(s, eps)
    rhs = exact.lemma32_bound(eps)
    assert np.all(lhs <= rhs + 1e-15)
    # the bound is attained at s = e^{-eps} for eps > 0
    e = np.abs(rng.normal(0, 1, 1000))
    assert np.allclose(exact.acceptance_difference(np.exp(-e), e), exact.lemma32_bound(e), atol=1e-15)


def test_pinsker_and_bias_bound_on_enumerated_perturbation(orc):
    """Reduced-precision perturbation of an RBM: TV <= sqrt(KL/2) and |E~ f - E f| <= 2 A TV (Eq. eq:bias_gaussian)."""
    n = 12
    p = workloads.rbm_params(n, 12, 0.3, 3)
    ham = workloads.Hamiltonian("tfim", workloads.Lattice(1, n), 1.0, 1.0)
    m64 = oracle.OracleModel("rbm", n, (12,), p)
    pi, f64, _ = exact.enumerate_pi(m64)
    el = oracle.local_energy(m64, ham, exact.all_configs(n))
    A = np.max(np.abs(el))
    for fmt in ("bf16", "f16"):
        mlp = oracle.OracleModel("rbm", n, (12,), oracle.round_to(p, fmt))
        pit, flp, _ = exact.enumerate_pi(mlp)
        delta = 2 * (flp - f64)
        assert np.allclose(exact.perturbed_pi(pi, delta), pit, rtol=1e-10, atol=1e-15)
        t = exact.tv(pi, pit)
        assert t <= np.sqrt(exact.kl(pi, pit) / 2) + 1e-15
        assert abs(np.sum(pit * el) - np.sum(pi * el)) <= 2 * A * t + 1e-12
        assert t > 0
