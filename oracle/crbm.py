"""CPU FP64 oracle of the complex-parameter RBM (App. G with complex a, b, W).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy complex128,
written from the definition

    log psi(x) = sum_i a_i s_i + sum_j log cosh(theta_j),  theta = W s + b,

with |psi|^2 = exp(2 Re log psi) the sampled distribution and the local
energy eps(x) = sum_x' H(x, x') psi(x') / psi(x) complex.  Parameter vector of
2P reals: the real parts of [a (N), b (M), W (M x N, row-major)], then their
imaginary parts.  Reduced precision rounds real and imaginary parts to the
format independently.

Log-derivatives and stochastic reconfiguration with complex parameters
(App. I.2): O_k(x) = d log psi(x) / d p_k, the derivative with respect to the
complex parameter p_k (log psi is holomorphic in a, b, W):
    d/da_i = s_i,  d/db_j = tanh(theta_j),  d/dW_ji = tanh(theta_j) s_i;
forces F = E[O* eps] - E[O*] E[eps] (Eq. eq:forces) and
S_nm = E[O_n* O_m] - E[O_n*] E[O_m] (Eq. eq:smat), both complex; the SR step
solves (S + shift I) delta = F (Eq. eq:sr_step) and moves p -> p - lr delta,
i.e. the real parts by Re delta and the imaginary parts by Im delta.
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

    def logpsi_grad(self, samples: np.ndarray) -> np.ndarray:
        """O[n][P] complex: the derivatives of log psi with respect to the P complex parameters
        [a, b, W (row-major)], from the definitions in the module docstring."""
        s = np.asarray(samples, dtype=np.float64).reshape(-1, self.N)
        t = np.tanh(s @ self.W.T + self.b)
        dW = t[:, :, None] * s[:, None, :]
        return np.concatenate([s.astype(np.complex128), t, dW.reshape(s.shape[0], -1)], axis=1)

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


def _weights(n: int, weights):
    if weights is None:
        return np.full(n, 1.0 / n)
    w = np.asarray(weights, dtype=np.float64)
    return w / w.sum()


def forces(O: np.ndarray, eloc: np.ndarray, weights=None) -> np.ndarray:
    """F_n = E[O_n* eps] - E[O_n*] E[eps] (Eq. eq:forces), complex; E is the plain sample mean, or the
    weighted mean when weights are given (e.g. |psi|^2 over an enumeration)."""
    O = np.asarray(O, dtype=np.complex128)
    e = np.asarray(eloc, dtype=np.complex128)
    w = _weights(O.shape[0], weights)
    Oc = O.conj()
    return (w[:, None] * Oc * e[:, None]).sum(axis=0) - (w[:, None] * Oc).sum(axis=0) * (w * e).sum()


def smatrix(O: np.ndarray, weights=None) -> np.ndarray:
    """S_nm = E[O_n* O_m] - E[O_n*] E[O_m] (Eq. eq:smat), complex Hermitian."""
    O = np.asarray(O, dtype=np.complex128)
    w = _weights(O.shape[0], weights)
    mean = (w[:, None] * O).sum(axis=0)
    return (O.conj() * w[:, None]).T @ O - np.outer(mean.conj(), mean)


def sr_direction(O: np.ndarray, eloc: np.ndarray, shift: float, weights=None) -> np.ndarray:
    """delta solving (S + shift I) delta = F (Eq. eq:sr_step), FP64 complex, dense solve."""
    S = smatrix(O, weights)
    F = forces(O, eloc, weights)
    return np.linalg.solve(S + shift * np.eye(S.shape[0]), F)


def tmatrix_embedded(O: np.ndarray) -> np.ndarray:
    """The sample-space twin of S, T = Obar Obar^H / n (Obar = O minus its sample mean), as the real
    2n x 2n matrix [[Re T, -Im T], [Im T, Re T]] that acts on (Re z, Im z) as T acts on z."""
    O = np.asarray(O, dtype=np.complex128)
    Ob = O - O.mean(axis=0)
    T = Ob @ Ob.conj().T / O.shape[0]
    return np.block([[T.real, -T.imag], [T.imag, T.real]])


def sr_update(params: np.ndarray, delta: np.ndarray, lr: float) -> np.ndarray:
    """p -> p - lr delta on the real parameter vector [Re p, Im p]."""
    p = np.asarray(params, dtype=np.float64)
    return p - lr * np.concatenate([delta.real, delta.imag])
