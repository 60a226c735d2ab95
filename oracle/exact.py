"""Exact references for small systems and the paper's closed-form bounds.

TEST INFRASTRUCTURE ONLY (see the package docstring).

- Exact diagonalisation of the TFIM (Eq. eq:TFIM) and Heisenberg (App. E)
  Hamiltonians, assembled from Kronecker products of 2x2 Pauli matrices --
  a construction independent of the local-energy code.
- Full enumeration of pi = |psi|^2 / sum |psi|^2 (Sec. II) for N <= 16.
- TV distance (Eq. eq:tv), KL divergence, the Gaussian/Pinsker bound
  (Eq. eq:tv_gaussian), the acceptance-difference bound of Lemma 3.2
  (Eq. eq:step3) and the local-MH Gaussian bound of Thm 3.3 (Eq. eq:avg_bound).
- The free-fermion ground energy of the periodic 1D TFIM and product-state
  closed forms used as pins.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.integrate
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.special

# Basis convention: state index x has bit i set  <=>  spin i is up (s_i = +1).
# Site 0 is the least significant bit, i.e. the LAST Kronecker factor.
_SZ = sp.csr_matrix(np.diag([-1.0, 1.0]))                    # (bit 0, bit 1) = (down, up)
_SX = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
_SY = sp.csr_matrix(np.array([[0.0, 1.0j], [-1.0j, 0.0]]))   # sigma^y in (down, up) order
_ID = sp.identity(2, format="csr")


def _site_op(op, i: int, n: int):
    mats = [_ID] * n
    mats[n - 1 - i] = op
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(out, m, format="csr")
    return out


def _bond_list(dim: int, L: int, pbc: bool):
    """Nearest-neighbour bonds written independently of the oracle's lattice code."""
    out = set()
    if dim == 1:
        rng = range(L) if pbc else range(L - 1)
        for i in rng:
            out.add(tuple(sorted((i, (i + 1) % L))))
    else:
        for x in range(L):
            for y in range(L):
                for dx, dy in ((1, 0), (0, 1)):
                    if not pbc and (x + dx >= L or y + dy >= L):
                        continue
                    a, b = x * L + y, ((x + dx) % L) * L + (y + dy) % L
                    out.add(tuple(sorted((a, b))))
    return sorted(out)


def hamiltonian_matrix(kind: str, dim: int, L: int, J: float = 1.0, h: float = 0.0, pbc: bool = True):
    """Sparse H: TFIM  J sum sz sz + h sum sx ;  Heisenberg  J sum sigma_i . sigma_j (Pauli)."""
    n = L if dim == 1 else L * L
    bonds = _bond_list(dim, L, pbc)
    dimh = 2 ** n
    H = sp.csr_matrix((dimh, dimh), dtype=np.complex128)
    for (i, j) in bonds:
        H = H + J * (_site_op(_SZ, i, n) @ _site_op(_SZ, j, n))
        if kind == "heisenberg":
            H = H + J * (_site_op(_SX, i, n) @ _site_op(_SX, j, n))
            H = H + J * (_site_op(_SY, i, n) @ _site_op(_SY, j, n))
    if kind == "tfim" and h != 0.0:
        for i in range(n):
            H = H + h * _site_op(_SX, i, n)
    assert abs(H - H.conj().T).max() < 1e-12
    return sp.csr_matrix(H.real)


def ground_state(kind: str, dim: int, L: int, J: float = 1.0, h: float = 0.0, pbc: bool = True):
    """(E_0, psi_0) by Lanczos (dense eigh for tiny spaces)."""
    H = hamiltonian_matrix(kind, dim, L, J, h, pbc)
    if H.shape[0] <= 512:
        w, v = np.linalg.eigh(H.toarray())
        return float(w[0]), v[:, 0]
    w, v = spla.eigsh(H, k=1, which="SA", tol=1e-13, maxiter=100000)
    return float(w[0]), v[:, 0]


def free_fermion_tfim_e0(n: int, J: float, h: float) -> float:
    """Periodic 1D TFIM ground energy (Jordan-Wigner / Bogoliubov closed form):
    E_0 = -sum_{m=0}^{n-1} sqrt(J^2 + h^2 - 2 J h cos(pi (2m+1)/n))."""
    k = np.pi * (2 * np.arange(n) + 1) / n
    return float(-np.sum(np.sqrt(J * J + h * h - 2 * J * h * np.cos(k))))


@functools.lru_cache(maxsize=8)
def all_configs(n: int) -> np.ndarray:
    """All 2^n configurations as int8 +-1 rows; row x has s_i = +1 iff bit i of x is set."""
    x = np.arange(2 ** n, dtype=np.int64)[:, None]
    bits = (x >> np.arange(n)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)


def enumerate_pi(model) -> tuple:
    """(pi, log|psi|, sign) over all configurations: pi = |psi|^2 / sum |psi|^2."""
    cfgs = all_configs(model.n)
    f, sg = model.logamp(cfgs)
    lp = 2.0 * f
    lp = lp - lp.max()
    p = np.exp(lp) * (sg != 0)
    return p / p.sum(), f, sg


def psi_vector(model) -> np.ndarray:
    """Normalised amplitude vector psi(x) over the full basis."""
    _, f, sg = enumerate_pi(model)
    v = sg * np.exp(f - f.max())
    return v / np.linalg.norm(v)


def exact_energy(model, kind: str, dim: int, L: int, J: float, h: float, pbc: bool = True) -> float:
    """<psi|H|psi>/<psi|psi> from the full matrix (no local energies involved)."""
    H = hamiltonian_matrix(kind, dim, L, J, h, pbc)
    v = psi_vector(model)
    return float(v @ (H @ v))


def tv(p: np.ndarray, q: np.ndarray) -> float:
    """Total-variation distance (Eq. eq:tv)."""
    return 0.5 * float(np.sum(np.abs(p - q)))


def kl(p: np.ndarray, q: np.ndarray) -> float:
    m = p > 0
    return float(np.sum(p[m] * (np.log(p[m]) - np.log(q[m]))))


def perturbed_pi(pi: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """pi~ = pi e^delta / Z (Eq. eq: pi tilde def)."""
    w = pi * np.exp(delta - np.max(delta))
    return w / w.sum()


def pinsker_bound(sigma: float) -> float:
    """Gaussian delta => KL = sigma^2/2 => TV <= sigma/2 (Eq. eq:tv_gaussian)."""
    return 0.5 * sigma


def avg_bound(sigma: float, mu: float = 0.0, r: float = 0.0) -> float:
    """Thm 3.3 (Eq. eq:avg_bound): local single-flip MH with eps ~ N(mu, 2 sigma^2)."""
    if sigma <= 0.0:
        return 0.0
    a = sigma - mu / (2.0 * sigma)
    b = sigma + mu / (2.0 * sigma)
    bracket = np.exp(-mu) * scipy.special.erfc(a) + np.exp(mu) * scipy.special.erfc(b)
    return float((1.0 - 0.5 * np.exp(sigma ** 2) * bracket) / (1.0 - r))


def avg_bound_quadrature(sigma: float, mu: float = 0.0) -> float:
    """1 - E[exp(-|eps|)], eps ~ N(mu, 2 sigma^2), by numerical integration (the
    quantity Thm 3.3 evaluates in closed form, Lemma 3.2 specialised)."""
    s2 = 2.0 * sigma * sigma
    dens = lambda e: np.exp(-(e - mu) ** 2 / (2 * s2)) / np.sqrt(2 * np.pi * s2)
    lo, hi = mu - 40 * np.sqrt(s2), mu + 40 * np.sqrt(s2)
    pts = [0.0] if lo < 0.0 < hi else None
    val, _ = scipy.integrate.quad(lambda e: np.exp(-abs(e)) * dens(e), lo, hi, points=pts,
                                  epsabs=1e-14, epsrel=1e-13, limit=500)
    return 1.0 - val


def acceptance_difference(s: np.ndarray, eps: np.ndarray) -> np.ndarray:
    """|min(1, s e^eps) - min(1, s)| (Lemma 3.2, Eq. eq:step3 left-hand side)."""
    return np.abs(np.minimum(1.0, s * np.exp(eps)) - np.minimum(1.0, s))


def lemma32_bound(eps: np.ndarray) -> np.ndarray:
    """1 - e^{-|eps|} (Lemma 3.2, Eq. eq:step3 right-hand side)."""
    return 1.0 - np.exp(-np.abs(eps))


def mh_flip_matrix(pi: np.ndarray, n: int) -> np.ndarray:
    """Exact single-flip MH kernel P (Sec. III.A): q = 1/n, alpha = min(1, pi(y)/pi(x))."""
    dimh = pi.size
    P = np.zeros((dimh, dimh))
    for x in range(dimh):
        for i in range(n):
            y = x ^ (1 << i)
            P[x, y] += (1.0 / n) * min(1.0, pi[y] / pi[x])
        P[x, x] = 1.0 - P[x].sum()
    return P


def product_state_tfim(a: np.ndarray, bonds: np.ndarray, J: float, h: float):
    """RBM with W = 0: pi factorises.  Returns (<s_i>, <H_TFIM>, MH acceptance).

    p(s) ~ prod_i exp(2 a_i s_i):  <s_i> = tanh 2a_i,
    <H> = J sum_<ij> tanh 2a_i tanh 2a_j + h sum_i sech 2a_i,
    acceptance of a uniform single flip = (1/N) sum_i exp(-2|a_i|) / cosh 2a_i.
    """
    m = np.tanh(2 * a)
    e = J * np.sum(m[bonds[:, 0]] * m[bonds[:, 1]]) + h * np.sum(1.0 / np.cosh(2 * a))
    acc = np.mean(np.exp(-2 * np.abs(a)) / np.cosh(2 * a))
    return m, float(e), float(acc)


def unit_roundoff(fmt: str) -> float:
    """u = 2^-p for a format with p significand bits (incl. the implicit bit) (App. A)."""
    p = {"bf16": 8, "f16": 11, "f32": 24, "f64": 53}[fmt]
    return 2.0 ** (-p)


def marshall_sign(configs: np.ndarray, dim: int, L: int) -> np.ndarray:
    """(-1)^{number of up spins on sublattice A}, A = {(x+y) even} (2D) or {i even} (1D)."""
    n = configs.shape[1]
    idx = np.arange(n)
    on_a = (idx % 2 == 0) if dim == 1 else (((idx // L) + (idx % L)) % 2 == 0)
    ups = np.sum((configs > 0) & on_a[None, :], axis=1)
    return np.where(ups % 2 == 0, 1, -1).astype(np.int8)
