"""Pins of the residual convolutional network oracle (App. H)."""
import numpy as np
import scipy.ndimage
import scipy.special

import workloads
from oracle import exact
from oracle import rescnn


def test_conv_matches_scipy_wrap_correlation():
    rng = np.random.default_rng(0)
    L, C, O = 5, 3, 4
    h = rng.normal(size=(2, L, L, C))
    W = rng.normal(size=(O, C, 9))
    b = rng.normal(size=O)
    got = rescnn.conv3x3(h, W, b)
    for n in range(2):
        for o in range(O):
            ref = np.full((L, L), b[o])
            for c in range(C):
                k = W[o, c].reshape(3, 3)   # k[dx + 1, dy + 1]
                ref += scipy.ndimage.correlate(h[n, :, :, c], k, mode="wrap")
            assert np.allclose(got[n, :, :, o], ref, atol=1e-12)


def test_layer_norm_and_gelu():
    rng = np.random.default_rng(1)
    h = rng.normal(3.0, 2.0, size=(4, 3, 3, 16))
    z = rescnn.layer_norm(h, np.ones(16), np.zeros(16))
    assert np.allclose(z.mean(axis=-1), 0.0, atol=1e-12)
    assert np.allclose(z.var(axis=-1), 1.0, atol=1e-5)
    x = np.linspace(-6, 6, 1001)
    exact_gelu = 0.5 * x * (1.0 + scipy.special.erf(x / np.sqrt(2.0)))
    assert np.max(np.abs(rescnn.gelu(x) - exact_gelu)) < 1e-3


def test_log_psi_is_translation_invariant_and_not_constant():
    L, F, R = 4, 8, 2
    net = rescnn.ResCNN(L, F, R, workloads.rescnn_params(F, R, 3))
    x = workloads.random_spins(20, L * L, 4)
    f, _ = net.logamp(x)
    g = x.reshape(-1, L, L)
    for sh in [(1, 0), (0, 1), (2, 3)]:
        ft, _ = net.logamp(np.roll(g, sh, axis=(1, 2)).reshape(-1, L * L))
        assert np.allclose(ft, f, rtol=0, atol=1e-10)
    assert np.std(f) > 1e-3


def test_local_energy_matches_matrix_expectation():
    """sum_x pi(x) eps(x) = <psi|H|psi>/<psi|psi> on the 3 x 3 periodic lattice (512 states)."""
    L, F, R = 3, 4, 1
    net = rescnn.ResCNN(L, F, R, workloads.rescnn_params(F, R, 5, scale=1.5))
    cfgs = exact.all_configs(L * L)
    f, _ = net.logamp(cfgs)
    w = np.exp(2 * (f - f.max()))
    pi = w / w.sum()
    for J, h in [(1.0, -1.0), (0.5, 2.0)]:
        eps = net.local_energy_tfim(cfgs, J, h)
        H = exact.hamiltonian_matrix("tfim", 2, L, J, h, True)
        v = np.exp(f - f.max())
        v /= np.linalg.norm(v)
        assert abs(float(pi @ eps) - float(v @ (H @ v))) < 1e-10 * max(1.0, abs(float(v @ (H @ v))))


def test_parameter_count():
    for F, R in [(4, 1), (16, 4)]:
        assert rescnn.n_params(F, R) == workloads.rescnn_params(F, R, 0).size


def test_finite_difference_gradient_is_consistent():
    """The central-difference log-derivatives of the oracle: translation
    invariance carries over (O of a translated configuration is the same), the
    final layer-norm shift has derivative L^2 exactly, and a step along O
    changes log psi to first order by |O|^2 h."""
    L, F, R = 3, 4, 1
    p = workloads.rescnn_params(F, R, 8)
    net = rescnn.ResCNN(L, F, R, p)
    x = workloads.random_spins(3, L * L, 5)
    O = rescnn.logpsi_grad_fd(net, x)
    g = x.reshape(-1, L, L)
    Ot = rescnn.logpsi_grad_fd(net, np.roll(g, (1, 2), axis=(1, 2)).reshape(-1, L * L))
    assert np.allclose(O, Ot, atol=1e-7)
    assert np.allclose(O[:, -F:], L * L, atol=1e-6)          # d/d beta_f of sum over sites
    h = 1e-4
    f0, _ = net.logamp(x[:1])
    net2 = rescnn.ResCNN(L, F, R, p + h * O[0])
    f1, _ = net2.logamp(x[:1])
    assert abs((f1[0] - f0[0]) - h * np.dot(O[0], O[0])) < 1e-3 * h * np.dot(O[0], O[0])
