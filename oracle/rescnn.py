"""CPU FP64 oracle of the residual convolutional network (App. H).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, FP64,
written from the definition:

    h0 = Conv(x)
    h_{l+1} = h_l + Conv(phi(Conv(phi(LN(h_l)))))      l = 0 .. R-1
    log psi(x) = sum_{i,j,c} LN(h_R)_{ijc}

Readings where the appendix is silent: 3 x 3 cross-correlation with circular
(periodic) padding and a bias per output channel; layer normalisation over the
channels of each site with a learnable scale and shift (without them the sum
readout would vanish identically) and epsilon 1e-6; phi the tanh form of GELU;
the input is the spin s = +-1 of each site, one channel.  Reduced precision
follows the reading used for the dense networks: the parameters and the input
of every convolution are rounded to the format, everything else is exact
(here FP64).

Parameter vector: [W0 (F x 9), b0 (F)], then per block [gamma (F), beta (F),
W1 (F x F x 9), b1 (F), W2 (F x F x 9), b2 (F)], then [gamma_f (F), beta_f
(F)]; W[o][c][k] with k = 3 (dx + 1) + (dy + 1) the offset of the input site
(x + dx, y + dy) (periodic), site index i = x L + y.
"""
from __future__ import annotations

import numpy as np

from . import round_to

LN_EPS = 1e-6


def n_params(F: int, R: int) -> int:
    return 10 * F + R * (2 * F + 2 * (9 * F * F + F)) + 2 * F


def unpack(p: np.ndarray, F: int, R: int):
    """Split the parameter vector into named arrays (views)."""
    p = np.asarray(p, dtype=np.float64)
    assert p.size == n_params(F, R)
    o = 0

    def take(*shape):
        nonlocal o
        n = int(np.prod(shape))
        a = p[o:o + n].reshape(shape)
        o += n
        return a

    W0, b0 = take(F, 1, 9), take(F)
    blocks = []
    for _ in range(R):
        blocks.append(dict(g=take(F), be=take(F), W1=take(F, F, 9), b1=take(F), W2=take(F, F, 9), b2=take(F)))
    gf, bef = take(F), take(F)
    return W0, b0, blocks, gf, bef


def conv3x3(h: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """h [n, L, L, C] -> [n, L, L, O]: out[x,y,o] = b[o] + sum_{c,dx,dy} W[o,c,k] h[x+dx, y+dy, c]."""
    out = np.broadcast_to(b, h.shape[:3] + (W.shape[0],)).copy()
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            k = 3 * (dx + 1) + (dy + 1)
            shifted = np.roll(h, shift=(-dx, -dy), axis=(1, 2))   # shifted[x, y] = h[x + dx, y + dy]
            out += np.einsum("nxyc,oc->nxyo", shifted, W[:, :, k])
    return out


def layer_norm(h: np.ndarray, g: np.ndarray, be: np.ndarray) -> np.ndarray:
    mu = h.mean(axis=-1, keepdims=True)
    var = ((h - mu) ** 2).mean(axis=-1, keepdims=True)
    return (h - mu) / np.sqrt(var + LN_EPS) * g + be


def gelu(x: np.ndarray) -> np.ndarray:
    return 0.5 * x * (1.0 + np.tanh(np.sqrt(2.0 / np.pi) * (x + 0.044715 * x ** 3)))


class ResCNN:
    """log|psi| of the residual convolutional network on an L x L lattice, FP64,
    parameters and convolution inputs rounded to `dtype` ("f64": no rounding)."""

    def __init__(self, L: int, F: int, R: int, params, dtype: str = "f64"):
        self.L, self.F, self.R, self.n = L, F, R, L * L
        self.dtype = dtype
        p = np.asarray(params, dtype=np.float64)
        self.params = p if dtype == "f64" else round_to(p, dtype)

    def _q(self, x):
        return x if self.dtype == "f64" else round_to(x, self.dtype)

    def logamp(self, samples: np.ndarray):
        s = np.asarray(samples, dtype=np.float64).reshape(-1, self.L, self.L, 1)
        W0, b0, blocks, gf, bef = unpack(self.params, self.F, self.R)
        h = conv3x3(s, W0, b0)
        for blk in blocks:
            t = self._q(gelu(layer_norm(h, blk["g"], blk["be"])))
            u = self._q(gelu(conv3x3(t, blk["W1"], blk["b1"])))
            h = h + conv3x3(u, blk["W2"], blk["b2"])
        f = layer_norm(h, gf, bef).sum(axis=(1, 2, 3))
        return f, np.ones_like(f)

    def local_energy_tfim(self, samples: np.ndarray, J: float, h: float) -> np.ndarray:
        """eps(x) = J sum_<ij> s_i s_j + h sum_i psi(x^i)/psi(x) on the periodic L x L lattice
        (Eq. eq:local_energies with Eq. eq:TFIM)."""
        x = np.asarray(samples, dtype=np.int8).reshape(-1, self.n)
        L = self.L
        f0, _ = self.logamp(x)
        g = x.reshape(-1, L, L).astype(np.float64)
        diag = J * (np.sum(g * np.roll(g, -1, axis=1), axis=(1, 2)) + np.sum(g * np.roll(g, -1, axis=2), axis=(1, 2)))
        off = np.zeros(x.shape[0])
        for i in range(self.n):
            y = x.copy()
            y[:, i] = -y[:, i]
            fi, _ = self.logamp(y)
            off += np.exp(fi - f0)
        return diag + h * off



def logpsi_grad_fd(net: ResCNN, samples: np.ndarray, step: float = 1e-5) -> np.ndarray:
    """O[k][p] = d log psi(x_k) / d theta_p (Eq. eq:forces) by central differences
    of the FP64 network (dtype "f64"), one parameter at a time."""
    assert net.dtype == "f64"
    base = net.params.copy()
    x = np.asarray(samples, dtype=np.int8).reshape(-1, net.n)
    O = np.empty((x.shape[0], base.size))
    for q in range(base.size):
        net.params = base.copy()
        net.params[q] += step
        fp, _ = net.logamp(x)
        net.params[q] = base[q] - step
        fm, _ = net.logamp(x)
        O[:, q] = (fp - fm) / (2.0 * step)
    net.params = base
    return O
