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
