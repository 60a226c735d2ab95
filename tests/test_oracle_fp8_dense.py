"""Pins of the oracle's FP8 (E4M3) reading for dense networks (CPU only).

Weights: one scale per tensor, amax / 448 (FP32), every stored value an E4M3
code times its scale.  Layer inputs h_l (outputs of the hidden layers): one
power-of-two scale per layer from the bound B_l on |h_l| over all spin
configurations (B_0 = 1, B_l = max_k sum_i |W_l[k, i]| B_{l-1} + |b_l[k]|),
so that no scaled value can exceed 448.  Pinned here:
  - every scale is an exact power of two and the first layer's bound is
    attained (by the configuration aligned with the signs of the heaviest
    row), so that scale is as small as it can be without saturation;
  - no scaled layer input exceeds 448, on random configurations, on the
    adversarial one, and on configurations sampled near the bound of layer 2;
  - the oracle model built for 'e4m3' rounds exactly the hidden-layer outputs
    (its log-amplitude equals a forward written out here with the same
    rounding), and reduces to the FP64 forward when every value is already a
    code of the format.
"""
import numpy as np

import oracle
import workloads
from oracle import dense


def _net(n, widths, seed, bias_std=0.0):
    p = workloads.ffnn_params(n, widths, seed, bias_std=bias_std)
    rounded, _ = oracle.downcast(p, "ffnn", n, widths, "e4m3")
    return rounded, oracle.e4m3_act_scales(rounded, n, widths)


def _layers(rounded, n, widths):
    off, prev, out = 0, n, []
    for w in widths:
        W = rounded[off:off + w * prev].reshape(w, prev)
        off += w * prev
        b = rounded[off:off + w]
        off += w
        out.append((W, b))
        prev = w
    return out


def test_scales_are_powers_of_two_and_layer1_bound_is_attained():
    n, widths = 400, (1600, 800, 400)          # the 20x20 network
    rounded, sc = _net(n, widths, 5)
    assert sorted(sc) == [1, 2]
    for v in sc.values():
        m, e = np.frexp(v)
        assert m == 0.5                          # exact power of two
    (W1, b1), _, _ = _layers(rounded, n, widths)
    k = int(np.argmax(np.abs(W1).sum(axis=1) + np.abs(b1)))
    s = np.where(W1[k] >= 0, 1.0, -1.0)
    B1 = float(np.abs(W1[k]).sum() + abs(b1[k]))
    assert np.isclose(W1[k] @ s + b1[k], B1, rtol=1e-14)
    assert 224.0 < B1 / sc[1] <= 448.0


def test_no_scaled_layer_input_exceeds_448():
    n, widths = 64, (96, 48, 32)
    rounded, sc = _net(n, widths, 7, bias_std=0.2)
    layers = _layers(rounded, n, widths)
    X = workloads.random_spins(300, n, 3).astype(np.float64)
    # add the configurations aligned with every row of layer 1 (each attains that row's bound)
    X = np.concatenate([X, np.where(layers[0][0] >= 0, 1.0, -1.0)])
    h = X
    for l, (W, b) in enumerate(layers[:-1]):
        z = np.maximum(h @ W.T + b, 0.0)
        assert np.max(z) / sc[l + 1] <= 448.0
        h = oracle.round_to(z / sc[l + 1], "e4m3") * sc[l + 1]


def test_e4m3_model_rounds_exactly_the_hidden_outputs():
    n, widths = 36, (48, 24, 12)
    p = workloads.ffnn_params(n, widths, 9, bias_std=0.1)
    wl = workloads.Workload("t", workloads.Hamiltonian("heisenberg", workloads.Lattice(2, 6), 1.0, 0.0, True),
                            workloads.Model("ffnn", n, widths), 4, 1, 0, "exchange", 0.0, 9)
    om = oracle.model_from_workload(wl, p, "e4m3")
    assert om.act_dtype == "e4m3" and sorted(om.act_scales) == [1, 2]
    rounded, _ = oracle.downcast(p, "ffnn", n, widths, "e4m3")
    X = workloads.random_spins(50, n, 1, zero_mag=True)
    f_c, _ = om.logamp(X)
    # written out: round each hidden output to q * scale, q an E4M3 code; no rounding of the last layer
    h = X.astype(np.float64)
    layers = _layers(rounded, n, widths)
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if l == len(layers) - 1:
            f = np.sum(dense.logcosh(z), axis=1)
        else:
            s = om.act_scales[l + 1]
            h = oracle.round_to(np.maximum(z, 0.0) / s, "e4m3") * s
    assert np.allclose(f_c, f, rtol=1e-13, atol=1e-13)
    # with unit-free codes the rounding is the identity: a network whose hidden outputs are E4M3 codes
    # times the scale gives the FP64 forward
    W1 = np.zeros((2, 4)); W1[0, 0] = 1.0; W1[1, 1] = 0.5
    W2 = np.ones((1, 2)) * 0.25
    tiny = np.concatenate([W1.ravel(), np.zeros(2), W2.ravel(), np.zeros(1)])
    sc = oracle.e4m3_act_scales(tiny, 4, (2, 1))
    assert sc == {1: 2.0 ** -8}
    om2 = oracle.OracleModel("ffnn", 4, (2, 1), tiny, act_dtype="e4m3", act_scales=sc)
    om64 = oracle.OracleModel("ffnn", 4, (2, 1), tiny)
    Xs = np.array([[1, 1, -1, 1], [-1, 1, 1, -1], [1, -1, 1, 1]], dtype=np.int8)
    assert np.array_equal(om2.logamp(Xs)[0], om64.logamp(Xs)[0])
