"""CPU FP64 oracle of the complex-parameter RBM (App. G with complex a, b, W).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy complex128,
written from the definition

    log psi(x) = sum_i a_i s_i + sum_j log cosh(theta_j),  theta = W s + b,

with |psi|^2 = exp(2 Re log psi) the sampled distribution and the local
energy eps(x) = sum_x' H(x, x') psi(x') / psi(x) complex.  Parameter vector of
2P reals: the real parts of [a (N), b (M), W (M x N, row-major)], then their
imaginary parts.  Reduced precision rounds real and imaginary parts to the
format independently.
"""
from __future__ import annotations

import numpy as np

from . import round_to


def split(p: np.ndarray, N: int, M: int):
    p = np.asarray(p, dtype=np.float64)
    P = N + M + M * N
    assert p.size == 2 * P
    z = p[:P] + 1j * p[P:]
    return z[:N], z[N:N + M], z[N + M:].reshape(M, N)


def _logcosh(z):
    # log cosh z = z + log(1 + e^{-2z}) - log 2 for Re z >= 0, and log cosh(-z) = log cosh z
    w = np.where(z.real < 0, -z, z)
    return w + np.log1p(np.exp(-2.0 * w)) - np.log(2.0)


class ComplexRBM:
    def __init__(self, N: int, M: int, params, dtype: str = "f64"):
        self.n, self.N, self.M, self.dtype = N, N, M, dtype
        p = np.asarray(params, dtype=np.float64)
        self.params = p if dtype == "f64" else round_to(p, dtype)
        self.a, self.b, self.W = split(self.params, N, M)

    def logpsi(self, samples: np.ndarray) -> np.ndarray:
        s = np.asarray(samples, dtype=np.float64).reshape(-1, self.N)
        theta = s @ self.W.T + self.b
        return s @ self.a + _logcosh(theta).sum(axis=1)

    def logamp(self, samples: np.ndarray):
        lp = self.logpsi(samples)
        return lp.real, np.ones(lp.shape)

    def local_energy_tfim(self, samples: np.ndarray, dim: int, L: int, J: float, h: float, pbc: bool = True):
        """Complex eps(x) for H = J sum_<ij> sz sz + h sum_i sx (Eq. eq:TFIM) on a chain (dim 1) or
        an L x L lattice (dim 2)."""
        x = np.asarray(samples, dtype=np.int8).reshape(-1, self.N)
        g = x.astype(np.float64)
        if dim == 1:
            diag = np.sum(g[:, :L - 1] * g[:, 1:L], axis=1) + (g[:, L - 1] * g[:, 0] if pbc else 0.0)
        else:
            q = g.reshape(-1, L, L)
            if pbc:
                diag = np.sum(q * np.roll(q, -1, axis=1), axis=(1, 2)) + np.sum(q * np.roll(q, -1, axis=2), axis=(1, 2))
            else:
                diag = np.sum(q[:, :-1, :] * q[:, 1:, :], axis=(1, 2)) + np.sum(q[:, :, :-1] * q[:, :, 1:], axis=(1, 2))
        l0 = self.logpsi(x)
        off = np.zeros(x.shape[0], dtype=np.complex128)
        for i in range(self.N):
            y = x.copy()
            y[:, i] = -y[:, i]
            off += np.exp(self.logpsi(y) - l0)
        return J * diag + h * off
