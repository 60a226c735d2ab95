"""Pins of the complex-parameter RBM oracle."""
import numpy as np

import oracle
import workloads
from oracle import crbm
from oracle import exact


def test_real_parameters_reduce_to_the_real_rbm():
    N, M = 10, 14
    p = workloads.rbm_params(N, M, 0.3, 2)
    net = crbm.ComplexRBM(N, M, np.concatenate([p, np.zeros_like(p)]))
    x = workloads.random_spins(50, N, 3)
    f_ref, _ = oracle.OracleModel("rbm", N, (M,), p).logamp(x)
    lp = net.logpsi(x)
    assert np.allclose(lp.real, f_ref, atol=1e-12) and np.allclose(lp.imag, 0.0, atol=1e-12)


def test_phase_state_is_the_sx_eigenstate():
    """a_i = i pi / 2, b = W = 0: psi(x) ~ prod_i exp(i pi s_i / 2), so every flip
    ratio is -1 and eps = -h N: the all-(sigma^x = -1) eigenstate."""
    N, M = 8, 3
    P = N + M + M * N
    p = np.zeros(2 * P)
    p[P:P + N] = np.pi / 2
    net = crbm.ComplexRBM(N, M, p)
    x = workloads.random_spins(20, N, 1)
    eps = net.local_energy_tfim(x, 1, N, 0.0, 0.7)
    assert np.allclose(eps, -0.7 * N, atol=1e-12)


def test_local_energy_matches_matrix_expectation():
    for dim, L in [(1, 8), (2, 3)]:
        N, M = L if dim == 1 else L * L, 6
        net = crbm.ComplexRBM(N, M, workloads.crbm_params(N, M, 0.3, 0.5, 4 + dim))
        cfgs = exact.all_configs(N)
        lp = net.logpsi(cfgs)
        psi = np.exp(lp - lp.real.max())
        pi = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
        for J, h in [(1.0, 1.0), (-0.5, 2.0)]:
            eps = net.local_energy_tfim(cfgs, dim, L, J, h)
            H = exact.hamiltonian_matrix("tfim", dim, L, J, h, True)
            v = psi / np.linalg.norm(psi)
            e_mat = complex(np.vdot(v, H @ v))
            e_mc = complex(np.sum(pi * eps))
            assert abs(e_mc - e_mat) < 1e-10 * max(1.0, abs(e_mat))
            assert abs(e_mat.imag) < 1e-10


# ---------------------------------------------------------------------------
# Log-derivatives, forces, S and the SR direction with complex parameters
# ---------------------------------------------------------------------------

def _enumerated(net, N):
    """All 2^N configurations, |psi|^2 weights and complex TFIM local energies (chain, J = 1, h = 0.9)."""
    cfgs = exact.all_configs(N)
    lp = net.logpsi(cfgs)
    w = np.exp(2.0 * (lp.real - lp.real.max()))
    return cfgs, w / w.sum(), net.local_energy_tfim(cfgs, 1, N, 1.0, 0.9)


def test_log_derivatives_are_the_finite_differences_along_both_parts():
    """d log psi / d Re p_k = O_k and d log psi / d Im p_k = i O_k (log psi holomorphic in p), every k."""
    N, M = 6, 5
    P = N + M + M * N
    p = workloads.crbm_params(N, M, 0.3, 0.3, 11)
    x = workloads.random_spins(7, N, 12)
    O = crbm.ComplexRBM(N, M, p).logpsi_grad(x)
    assert O.shape == (7, P)
    h = 1e-6
    for k in range(2 * P):
        dp = np.zeros(2 * P)
        dp[k] = h
        d = (crbm.ComplexRBM(N, M, p + dp).logpsi(x) - crbm.ComplexRBM(N, M, p - dp).logpsi(x)) / (2 * h)
        want = O[:, k] if k < P else 1j * O[:, k - P]
        assert np.max(np.abs(d - want)) < 1e-8, k


def test_forces_are_half_the_exact_energy_gradient():
    """Over the enumerated 6-site chain, dE/dRe p_k = 2 Re F_k and dE/dIm p_k = 2 Im F_k, E the exact energy
    <psi|H|psi>/<psi|psi>: a dropped conjugate or a sign in F fails one of the two halves."""
    N, M = 6, 6
    P = N + M + M * N
    p = workloads.crbm_params(N, M, 0.2, 0.2, 21)

    def energy(q):
        net = crbm.ComplexRBM(N, M, q)
        _, w, eps = _enumerated(net, N)
        return float(np.sum(w * eps).real)

    net = crbm.ComplexRBM(N, M, p)
    cfgs, w, eps = _enumerated(net, N)
    F = crbm.forces(net.logpsi_grad(cfgs), eps, weights=w)
    h = 1e-5
    grad = np.empty(2 * P)
    for k in range(2 * P):
        dp = np.zeros(2 * P)
        dp[k] = h
        grad[k] = (energy(p + dp) - energy(p - dp)) / (2 * h)
    want = 2.0 * np.concatenate([F.real, F.imag])
    assert np.max(np.abs(grad - want)) < 1e-7 * max(1.0, np.max(np.abs(want)))


def test_s_matrix_is_the_geometric_tensor_of_the_state():
    """S of Eq. eq:smat under |psi|^2 equals <d_k psi|d_l psi>/<psi|psi> - <d_k psi|psi><psi|d_l psi>/<psi|psi>^2
    with d_k psi from finite differences of the state vector itself (no use of the O formulas)."""
    N, M = 5, 4
    P = N + M + M * N
    p = workloads.crbm_params(N, M, 0.3, 0.3, 31)
    cfgs = exact.all_configs(N)

    def state(q):
        return np.exp(crbm.ComplexRBM(N, M, q).logpsi(cfgs))

    psi = state(p)
    h = 1e-6
    D = np.empty((P, psi.size), dtype=np.complex128)
    for k in range(P):
        dp = np.zeros(2 * P)
        dp[k] = h
        D[k] = (state(p + dp) - state(p - dp)) / (2 * h)
    nrm = np.vdot(psi, psi).real
    ov = D.conj() @ psi / nrm                       # <d_k psi | psi> / <psi|psi>
    qgt = (D.conj() @ D.T) / nrm - np.outer(ov, ov.conj())
    net = crbm.ComplexRBM(N, M, p)
    w = np.abs(psi) ** 2 / nrm
    S = crbm.smatrix(net.logpsi_grad(cfgs), weights=w)
    assert np.allclose(S, S.conj().T, atol=1e-14)
    assert np.max(np.abs(S - qgt)) < 1e-7 * np.max(np.abs(S))


def test_real_parameters_reduce_to_the_real_log_derivatives_and_sr():
    """Imaginary parts zero: O, F, S and the SR direction are the real RBM's, from the C oracle."""
    N, M = 8, 6
    p = workloads.rbm_params(N, M, 0.3, 41)
    net = crbm.ComplexRBM(N, M, np.concatenate([p, np.zeros_like(p)]))
    real = oracle.OracleModel("rbm", N, (M,), p)
    x = workloads.random_spins(64, N, 42)
    _, O_ref = oracle.logpsi_grad(real, x)
    O = net.logpsi_grad(x)
    assert np.max(np.abs(O.imag)) == 0.0 and np.allclose(O.real, O_ref, atol=1e-12)
    e = workloads.random_spins(64, 1, 43).astype(np.float64).ravel() + 0.25 * np.arange(64) / 64
    assert np.allclose(crbm.forces(O, e), oracle.forces(O_ref, e), atol=1e-12)
    assert np.allclose(crbm.smatrix(O), oracle.smatrix(O_ref), atol=1e-12)
    assert np.allclose(crbm.sr_direction(O, e, 0.1), oracle.sr_direction(O_ref, e, 0.1), atol=1e-10)


def test_sample_space_solve_gives_the_parameter_space_direction():
    """(S + l) delta = F in parameter space equals Obar^H z / n with (T + l) z = eps - mean eps in sample space,
    T taken as its real 2n x 2n embedding (the push-through identity)."""
    N, M, n, lam = 6, 5, 40, 0.05
    p = workloads.crbm_params(N, M, 0.3, 0.3, 51)
    net = crbm.ComplexRBM(N, M, p)
    x = workloads.random_spins(n, N, 52)
    O = net.logpsi_grad(x)
    eps = net.local_energy_tfim(x, 1, N, 1.0, 0.9)
    delta = crbm.sr_direction(O, eps, lam)
    T2 = crbm.tmatrix_embedded(O)
    e = eps - eps.mean()
    y = np.linalg.solve(T2 + lam * np.eye(2 * n), np.concatenate([e.real, e.imag]))
    z = y[:n] + 1j * y[n:]
    Ob = O - O.mean(axis=0)
    assert np.max(np.abs(Ob.conj().T @ z / n - delta)) < 1e-10 * np.max(np.abs(delta))
