"""Batched FP64 local energies of dense networks -- TEST INFRASTRUCTURE ONLY.

The same quantities as the C oracle's dense forward and local energies
(nqs_oracle.c), evaluated for many configurations at once: every layer of
every connected configuration of a batch of samples is one matrix product,
taken with numpy's matmul (a library primitive).  The C oracle evaluates one
configuration at a time and re-reads every weight for each of them, which on
the 20x20 network (18 MB of FP64 weights, ~400 connected configurations per
sample) makes each sample take most of a second; here the weights are read
once per batch.

Definitions (as in the C oracle):
  dense network:  h_0 = s,  h_l = ReLU(W_l h_{l-1} + b_l) for l < L,
                  f(s) = sum_k log cosh((W_L h_{L-1} + b_L)_k), log|psi| = f;
                  with a reduced format each layer input h_l (l >= 1) is
                  rounded to that format (an operand of a matrix product);
  Marshall sign:  psi(s) = M(s) e^{f(s)}, M(s) = (-1)^{#up spins on A};
  local energy (App. I.1, Eq. eq:local_energies):
      TFIM        eps(s) = J sum_<ij> s_i s_j + h sum_i psi(s^i)/psi(s)
      Heisenberg  eps(s) = J sum_<ij> s_i s_j + 2J sum_{<ij>: s_i != s_j} psi(s^{ij})/psi(s)
                  (Pauli matrices, App. E).
Sums of the ratios are FP64, in bond (or site) order per sample.
"""
from __future__ import annotations

import numpy as np

from . import bonds as _bonds
from . import round_to


def logcosh(z: np.ndarray) -> np.ndarray:
    a = np.abs(z)
    return a + np.log1p(np.exp(-2.0 * a)) - np.log(2.0)


def _round_layer(h: np.ndarray, act_dtype: str, scale: float) -> np.ndarray:
    if act_dtype == "f64":
        return h
    if act_dtype == "e4m3":
        return round_to(h / scale, "e4m3") * scale
    return round_to(h, act_dtype)


def logamp_rows(params: np.ndarray, n: int, widths, X: np.ndarray, act_dtype: str = "f64",
                act_scales=None) -> np.ndarray:
    """f(x) of each row of X ([rows][n], entries +-1) for the dense network with flat FP64 parameters
    [W_1 (w_1 x n), b_1, W_2, b_2, ...]; act_scales[l] is the E4M3 scale of the input of layer l + 1."""
    h = np.asarray(X, dtype=np.float64)
    off, prev = 0, n
    L = len(widths)
    for l, w in enumerate(widths):
        W = params[off:off + w * prev].reshape(w, prev)
        off += w * prev
        b = params[off:off + w]
        off += w
        z = h @ W.T + b
        if l == L - 1:
            return logcosh(z).sum(axis=1)
        sc = 1.0 if not act_scales else act_scales.get(l + 1, 1.0)
        h = _round_layer(np.maximum(z, 0.0), act_dtype, sc)
        prev = w
    raise ValueError("network without layers")


def _sublattice_a(dim: int, L: int, n: int) -> np.ndarray:
    i = np.arange(n)
    if dim == 1:
        return i % 2 == 0
    return ((i // L + i % L) % 2) == 0


def local_energy(params, n, widths, ham, samples, act_dtype="f64", marshall=False, act_scales=None,
                 batch=8) -> np.ndarray:
    """Local energies of the rows of `samples` (int8 +-1) for the dense network (see module docstring);
    `ham` carries kind ('tfim' | 'heis'), lattice (dim, L, pbc), J and h."""
    samples = np.asarray(samples, dtype=np.int8).reshape(-1, n)
    lat = ham.lattice
    bd = _bonds(lat.dim, lat.L, lat.pbc)
    onA = _sublattice_a(lat.dim, lat.L, n)
    out = np.empty(samples.shape[0])
    for k0 in range(0, samples.shape[0], batch):
        blk = samples[k0:k0 + batch].astype(np.float64)
        rows, owner, coef = [], [], []
        diag = np.zeros(blk.shape[0])
        for b, s in enumerate(blk):
            diag[b] = ham.J * np.sum(s[bd[:, 0]] * s[bd[:, 1]])
            rows.append(s)
            owner.append(-1 - b)          # the sample itself
            coef.append(0.0)
            if ham.kind == "tfim":
                for i in range(n):
                    y = s.copy()
                    y[i] = -y[i]
                    rows.append(y)
                    owner.append(b)
                    coef.append(ham.h)
            else:
                for i, j in bd:
                    if s[i] == s[j]:
                        continue
                    y = s.copy()
                    y[i], y[j] = s[j], s[i]
                    rows.append(y)
                    owner.append(b)
                    coef.append(2.0 * ham.J)
        X = np.array(rows)
        f = logamp_rows(params, n, widths, X, act_dtype, act_scales)
        sign = np.ones(X.shape[0])
        if marshall:
            sign = np.where(np.sum((X > 0) & onA[None, :], axis=1) % 2 == 1, -1.0, 1.0)
        owner = np.array(owner)
        self_rows = np.where(owner < 0)[0]
        f0 = np.empty(blk.shape[0])
        s0 = np.empty(blk.shape[0])
        f0[-1 - owner[self_rows]] = f[self_rows]
        s0[-1 - owner[self_rows]] = sign[self_rows]
        e = diag.copy()
        for r in range(X.shape[0]):
            b = owner[r]
            if b < 0:
                continue
            e[b] += coef[r] * sign[r] * s0[b] * np.exp(f[r] - f0[b])
        out[k0:k0 + blk.shape[0]] = e
    return out
