"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws numbers and names shapes.  It contains none of the
method's arithmetic (no network evaluation, no Hamiltonian, no sampling), so
both the CPU oracle and the HIP path can consume its arrays without sharing
any computation.

Parameter vector layouts (FP64, flat, row-major):
  RBM  (App. G):  a[N], b[M], W[M][N]           -> P = N + M + M*N
  FFNN (dense):   W1[w1][N], b1[w1], W2[w2][w1], b2[w2], ...
                  -> P = sum_l w_l * (w_{l-1} + 1)

The workloads mirror the paper's settings: random (untrained) RBM and FFNN
states on 1D chains and 2D square lattices with periodic boundaries; the
paper's trained weights are not available, so seeded random weights stand in
(random near-flat states are the paper's worst case for relative error,
App. D).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Lattice:
    dim: int          # 1 or 2
    L: int            # sites per side (1D: chain length)
    pbc: bool = True

    @property
    def n_sites(self) -> int:
        return self.L if self.dim == 1 else self.L * self.L


@dataclasses.dataclass(frozen=True)
class Hamiltonian:
    kind: str         # "tfim" | "heisenberg"
    lattice: Lattice
    J: float = 1.0
    h: float = 0.0
    marshall: bool = False


@dataclasses.dataclass(frozen=True)
class Model:
    arch: str                 # "rbm" | "ffnn"
    n_visible: int
    widths: Tuple[int, ...]   # rbm: (M,), ffnn: hidden widths, last one log-cosh

    @property
    def n_params(self) -> int:
        if self.arch == "rbm":
            (m,) = self.widths
            return self.n_visible + m + m * self.n_visible
        p, prev = 0, self.n_visible
        for w in self.widths:
            p += w * (prev + 1)
            prev = w
        return p


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    ham: Hamiltonian
    model: Model
    n_chains: int
    n_sweeps: int
    n_burnin: int
    move: str                 # "flip" | "exchange"
    weight_std: float = 0.0   # rbm: N(0, std^2); ffnn: He init when 0
    seed: int = 0


def rbm_params(n: int, m: int, std: float, seed: int) -> np.ndarray:
    """Draw RBM parameters a, b, W ~ N(0, std^2), in that order, as one FP64 vector."""
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, std, size=n)
    b = rng.normal(0.0, std, size=m)
    w = rng.normal(0.0, std, size=(m, n))
    return np.concatenate([a, b, w.ravel()]).astype(np.float64)


def ffnn_params(n: int, widths, seed: int, bias_std: float = 0.0) -> np.ndarray:
    """He-initialised dense layers W_l ~ N(0, 2/fan_in); biases N(0, bias_std^2) (0 by default)."""
    rng = np.random.default_rng(seed)
    out = []
    prev = n
    for w in widths:
        W = rng.normal(0.0, np.sqrt(2.0 / prev), size=(w, prev))
        b = rng.normal(0.0, bias_std, size=w) if bias_std > 0 else np.zeros(w)
        out.append(W.ravel())
        out.append(b)
        prev = w
    return np.concatenate(out).astype(np.float64)


def crbm_params(n: int, m: int, std_re: float, std_im: float, seed: int) -> np.ndarray:
    """Complex RBM: real parts of a, b, W ~ N(0, std_re^2), then imaginary parts ~ N(0, std_im^2)."""
    rng = np.random.default_rng(seed)
    P = n + m + m * n
    return np.concatenate([rng.normal(0.0, std_re, size=P), rng.normal(0.0, std_im, size=P)]).astype(np.float64)


def rescnn_params(F: int, R: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Residual convolutional network (App. H), in its parameter order: conv weights
    N(0, scale^2 2/fan_in), biases N(0, 0.1^2), layer-norm scales 1 + N(0, 0.1^2) and
    shifts N(0, 0.1^2); the final layer norm's scale and shift N(0, (0.1/F)^2)."""
    rng = np.random.default_rng(seed)
    out = [rng.normal(0.0, scale * np.sqrt(2.0 / 9.0), size=9 * F), rng.normal(0.0, 0.1, size=F)]
    for _ in range(R):
        out += [1.0 + rng.normal(0.0, 0.1, size=F), rng.normal(0.0, 0.1, size=F),
                rng.normal(0.0, scale * np.sqrt(2.0 / (9 * F)), size=9 * F * F), rng.normal(0.0, 0.1, size=F),
                rng.normal(0.0, scale * np.sqrt(2.0 / (9 * F)), size=9 * F * F), rng.normal(0.0, 0.1, size=F)]
    out += [rng.normal(0.0, 0.1 / F, size=F), rng.normal(0.0, 0.1 / F, size=F)]
    return np.concatenate(out)


def params_for(wl: Workload) -> np.ndarray:
    m = wl.model
    if m.arch == "rbm":
        return rbm_params(m.n_visible, m.widths[0], wl.weight_std, wl.seed)
    return ffnn_params(m.n_visible, m.widths, wl.seed)


def product_state_params(n: int, m: int, a_std: float, seed: int) -> np.ndarray:
    """RBM with W = 0, b = 0 and random visible biases a: a product state."""
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, a_std, size=n)
    return np.concatenate([a, np.zeros(m), np.zeros(m * n)])


def random_spins(n_samples: int, n: int, seed: int, zero_mag: bool = False) -> np.ndarray:
    """Random +-1 configurations as int8 [n_samples][n]; optionally with zero magnetisation."""
    rng = np.random.default_rng(seed)
    if not zero_mag:
        return (2 * rng.integers(0, 2, size=(n_samples, n)) - 1).astype(np.int8)
    base = np.array([1] * (n // 2) + [-1] * (n - n // 2), dtype=np.int8)
    out = np.empty((n_samples, n), dtype=np.int8)
    for k in range(n_samples):
        out[k] = rng.permutation(base)
    return out


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the paper's settings (1D chain with ED
# check; 2D TFIM at the critical field used in Sec. IV.B; 2D Heisenberg with
# exchange moves, App. E), with seeded random weights.
# ---------------------------------------------------------------------------

def cfg1_tfim_chain16() -> Workload:
    return Workload("tfim1d_n16_rbm_a1", Hamiltonian("tfim", Lattice(1, 16), 1.0, 1.0),
                    Model("rbm", 16, (16,)), n_chains=64, n_sweeps=200, n_burnin=50,
                    move="flip", weight_std=0.01, seed=1)


def cfg2_tfim_10x10() -> Workload:
    return Workload("tfim2d_10x10_rbm_a2", Hamiltonian("tfim", Lattice(2, 10), 1.0, 3.04),
                    Model("rbm", 100, (200,)), n_chains=4096, n_sweeps=1000, n_burnin=100,
                    move="flip", weight_std=0.02, seed=2)


def cfg3_heis_10x10() -> Workload:
    return Workload("heis2d_10x10_ffnn_400_200", Hamiltonian("heisenberg", Lattice(2, 10), 1.0, 0.0, True),
                    Model("ffnn", 100, (400, 200)), n_chains=16384, n_sweeps=500, n_burnin=50,
                    move="exchange", seed=3)


def cfg5_heis_20x20() -> Workload:
    return Workload("heis2d_20x20_ffnn_1600_800_400", Hamiltonian("heisenberg", Lattice(2, 20), 1.0, 0.0, True),
                    Model("ffnn", 400, (1600, 800, 400)), n_chains=65536, n_sweeps=200, n_burnin=20,
                    move="exchange", seed=5)


def cfg4_instances(seed: int = 4, n_inst: int = 32, chains: int = 1024) -> List[Workload]:
    """32 uneven 2D TFIM instances: L in {6..16}, h ~ U[2,4], alpha in {1,2,4}."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        L = int(rng.choice([6, 8, 10, 12, 14, 16]))
        h = float(rng.uniform(2.0, 4.0))
        alpha = int(rng.choice([1, 2, 4]))
        n = L * L
        out.append(Workload(f"tfim2d_{L}x{L}_a{alpha}_inst{k}", Hamiltonian("tfim", Lattice(2, L), 1.0, h),
                            Model("rbm", n, (alpha * n,)), n_chains=chains, n_sweeps=200, n_burnin=20,
                            move="flip", weight_std=0.02, seed=1000 + k))
    return out


def scaled(wl: Workload, n_chains: Optional[int] = None, n_sweeps: Optional[int] = None,
           n_burnin: Optional[int] = None) -> Workload:
    """Same lattice/model/weights, fewer chains or sweeps (parity-test sizes)."""
    return dataclasses.replace(wl, n_chains=n_chains or wl.n_chains,
                               n_sweeps=wl.n_sweeps if n_sweeps is None else n_sweeps,
                               n_burnin=wl.n_burnin if n_burnin is None else n_burnin)
