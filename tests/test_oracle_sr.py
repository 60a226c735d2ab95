"""Pins of the oracle's stochastic-reconfiguration direction (App. I.2,
Eq. eq:smat, forces of Eq. eq:forces): the sample-space form through T, and
the exact energy decrease it produces on an enumerated system."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.mark.parametrize("n,P,shift", [(40, 90, 1e-2), (120, 30, 1e-3), (64, 64, 0.5)])
def test_sr_direction_push_through(n, P, shift):
    """delta = Obar^T (T + shift)^{-1} (eps - mean eps) / n, derived independently
    of the parameter-space solve (the matrix identity (A^T A + c)^{-1} A^T =
    A^T (A A^T + c)^{-1})."""
    rng = np.random.default_rng(n + P)
    O = rng.normal(size=(n, P)) + rng.normal(size=P)
    eps = rng.normal(-5.0, 2.0, size=n)
    ref = oracle.sr_direction(O, eps, shift)
    Ob = O - O.mean(axis=0)
    T = Ob @ Ob.T / n
    y = np.linalg.solve(T + shift * np.eye(n), eps - eps.mean())
    assert np.allclose(Ob.T @ y / n, ref, rtol=1e-8, atol=1e-10 * np.abs(ref).max())


def _exact_energy(om, ham, configs):
    f, _ = om.logamp(configs)
    w = np.exp(2.0 * (f - f.max()))
    pi = w / w.sum()
    eps = oracle.local_energy(om, ham, configs)
    return float(np.dot(pi, eps)), pi, eps


def test_sr_step_lowers_the_exact_energy():
    """On the enumerated 8-site TFIM chain with the exact |psi|^2 weights, the
    directional derivative of E along -delta is -2 F.delta < 0 (F = grad E / 2),
    checked by central differences of the exactly enumerated energy."""
    N, M = 8, 8
    ham = workloads.Hamiltonian("tfim", workloads.Lattice(1, N), 1.0, -1.0)
    p = workloads.rbm_params(N, M, 0.3, 5)
    configs = ((np.arange(2 ** N)[:, None] >> np.arange(N)) & 1) * 2 - 1
    configs = configs.astype(np.int8)
    om = oracle.OracleModel("rbm", N, (M,), p)
    E0, pi, eps = _exact_energy(om, ham, configs)
    _, O = oracle.logpsi_grad(om, configs)
    F = oracle.forces(O, eps, weights=pi)
    delta = oracle.sr_direction(O, eps, 1e-3, weights=pi)
    h = 1e-5
    Ep, _, _ = _exact_energy(oracle.OracleModel("rbm", N, (M,), p - h * delta), ham, configs)
    Em, _, _ = _exact_energy(oracle.OracleModel("rbm", N, (M,), p + h * delta), ham, configs)
    dE = (Ep - Em) / (2 * h)
    assert dE < 0
    assert abs(dE - (-2.0 * np.dot(F, delta))) < 1e-6 * max(1.0, abs(dE))
    # a finite step lowers the energy too
    E1, _, _ = _exact_energy(oracle.OracleModel("rbm", N, (M,), p - 0.05 * delta), ham, configs)
    assert E1 < E0
