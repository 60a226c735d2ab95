"""Pins of the dense-network oracle (CPU only).

1. The wiring of the dense network (ReLU on every hidden layer but the last,
   log cosh on the last, sum readout; biases added before the activation) is
   evaluated here by an independent numpy forward written out in the test and
   compared with the C oracle's log-amplitude.
2. The oracle's batched local energies (oracle/dense.py, matrix products over
   all connected configurations) equal the C oracle's one-configuration-at-a-
   time local energies, for the TFIM and for the Heisenberg model with the
   Marshall sign, in FP64 and with BF16 / E4M3 layer inputs.
3. With a constant amplitude every exchange ratio is the Marshall-sign ratio,
   -1 on the bipartite lattice, so the Heisenberg local energy has a closed
   form in the numbers of parallel and antiparallel bonds; this pins the sign
   and exchange bookkeeping of the batched local energies.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import dense


def _ham(kind, L, J=1.0, h=0.0, marshall=False):
    return workloads.Hamiltonian(kind, workloads.Lattice(2, L, True), J, h, marshall)


@pytest.mark.parametrize("widths", [(32, 16), (24, 20, 12)])
def test_dense_wiring_independent_forward(widths):
    n = 16
    p = workloads.ffnn_params(n, widths, 3, bias_std=0.3)
    X = workloads.random_spins(40, n, 5)
    om = oracle.OracleModel("ffnn", n, widths, p)
    f_c, sg = om.logamp(X)
    # written out here: h = relu(W h + b) for each hidden layer, f = sum log cosh(W h + b) on the last
    h = X.astype(np.float64).T
    off, prev = 0, n
    for l, w in enumerate(widths):
        W = p[off:off + w * prev].reshape(w, prev)
        off += w * prev
        b = p[off:off + w][:, None]
        off += w
        z = W @ h + b
        if l < len(widths) - 1:
            h = np.where(z > 0, z, 0.0)
        else:
            f_np = np.sum(np.log(np.cosh(z)), axis=0)
        prev = w
    assert np.all(sg == 1)
    assert np.allclose(f_c, f_np, rtol=1e-13, atol=1e-13)
    assert np.allclose(dense.logamp_rows(p, n, widths, X), f_np, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind,act", [("heisenberg", "f64"), ("heisenberg", "bf16"), ("tfim", "f16"),
                                      ("heisenberg", "e4m3")])
def test_batched_local_energy_equals_c_oracle(kind, act):
    L = 4
    n = L * L
    widths = (48, 24)
    p = workloads.ffnn_params(n, widths, 11, bias_std=0.1)
    marshall = kind == "heisenberg"
    ham = _ham(kind, L, J=1.0, h=1.7, marshall=marshall)
    smp = workloads.random_spins(30, n, 9, zero_mag=(kind == "heisenberg"))
    scales = {1: 0.013} if act == "e4m3" else None
    om = oracle.OracleModel("ffnn", n, widths, p, act_dtype=act, marshall=marshall,
                            lattice=ham.lattice, act_scales=scales)
    ref = oracle.local_energy(om, ham, smp)
    got = dense.local_energy(p, n, widths, ham, smp, act_dtype=act, marshall=marshall, act_scales=scales, batch=7)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_batched_heisenberg_flat_state_terms():
    """A constant amplitude (zero weights in the last layer, zero bias) makes every ratio +-1: with the Marshall
    sign each antiparallel bond contributes -2J, so eps = J (n_par - n_anti) - 2 J n_anti."""
    L, n = 4, 16
    widths = (8, 4)
    p = workloads.ffnn_params(n, widths, 2)
    p[-(4 * 8 + 4):] = 0.0      # last layer: W_2 and b_2 zero, so f = 4 log cosh 0 = 0 for every input
    ham = _ham("heisenberg", L, J=1.3, marshall=True)
    smp = workloads.random_spins(12, n, 4, zero_mag=True)
    bd = oracle.bonds(2, L)
    anti = np.sum(smp[:, bd[:, 0]] != smp[:, bd[:, 1]], axis=1)
    par = bd.shape[0] - anti
    want = 1.3 * (par - anti) - 2 * 1.3 * anti
    got = dense.local_energy(p, n, widths, ham, smp, marshall=True)
    assert np.allclose(got, want, rtol=0, atol=1e-12)
