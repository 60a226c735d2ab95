"""CPU FP64 oracle for mixed-precision NQS sampling.

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU path is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product package never does.

`nqs_oracle.c` holds the method (sampling, local energies, log-derivatives,
averages) as plain FP64 loops; `exact.py` holds the exact references
(enumeration of |psi|^2, exact diagonalisation, TV distance, the paper's
closed-form bounds).  This module is the ctypes binding of the C part.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nqs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F64, F32, F16, BF16, E4M3 = 0, 1, 2, 3, 4
RBM, FFNN, TABLE = 0, 1, 2
FLIP, EXCHANGE = 0, 1
TFIM, HEIS = 0, 1
MAX_LAYERS = 8
DTYPES = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16, "e4m3": E4M3}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP over chains only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [("arch", ctypes.c_int32), ("n_visible", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("widths", ctypes.c_int32 * MAX_LAYERS), ("act_dtype", ctypes.c_int32),
                ("marshall", ctypes.c_int32), ("lat_dim", ctypes.c_int32), ("lat_L", ctypes.c_int32),
                ("act_scale", ctypes.c_double * MAX_LAYERS),
                ("params", ctypes.c_void_p), ("table_logamp", ctypes.c_void_p), ("table_sign", ctypes.c_void_p)]


class _Ham(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dim", ctypes.c_int32), ("L", ctypes.c_int32),
                ("pbc", ctypes.c_int32), ("J", ctypes.c_double), ("h", ctypes.c_double)]


class _Cfg(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int64), ("n_sweeps", ctypes.c_int32), ("n_burnin", ctypes.c_int32),
                ("sweep_size", ctypes.c_int32), ("move", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("step_offset", ctypes.c_uint64), ("instance_id", ctypes.c_uint32),
                ("init_chains", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        _lib.orc_philox4x32_10.argtypes = [P, P, P]
        _lib.orc_noise_zeta.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, P]
        _lib.orc_round.argtypes = [ctypes.c_double, ctypes.c_int32]
        _lib.orc_round.restype = ctypes.c_double
        _lib.orc_round_array.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P]
        _lib.orc_bonds.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P]
        _lib.orc_bonds.restype = ctypes.c_int32
        _lib.orc_logamp_batch.argtypes = [P, P, ctypes.c_int64, P, P]
        _lib.orc_init_chain.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_uint32, P]
        _lib.orc_sample.argtypes = [P, P, P, P, P, P]
        _lib.orc_sample.restype = ctypes.c_int32
        _lib.orc_replay.argtypes = [P, P, ctypes.c_int64, P, P, ctypes.c_int64, P, P, P, P, ctypes.c_double, P, P]
        _lib.orc_local_energy.argtypes = [P, P, P, ctypes.c_int64, P]
        _lib.orc_num_params.argtypes = [P]
        _lib.orc_num_params.restype = ctypes.c_int64
        _lib.orc_logpsi_grad.argtypes = [P, P, ctypes.c_int64, P, P]
        _lib.orc_stats.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P]
        _lib.orc_forces.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int64, P]
        _lib.orc_smatrix.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, P]
        _lib.orc_tmatrix.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P]
        _lib.orc_num_threads.restype = ctypes.c_int32
        _lib.orc_set_num_threads.argtypes = [ctypes.c_int32]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Reduced-precision formats (App. A, Table A)
# ---------------------------------------------------------------------------

def round_to(x, dtype: str) -> np.ndarray:
    """Round-to-nearest-even of FP64 values straight to `dtype` (one rounding)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.empty_like(x)
    lib().orc_round_array(_ptr(x), x.size, DTYPES[dtype], _ptr(out))
    return out


E4M3_MAX = 448.0


def e4m3_scale(x: np.ndarray) -> float:
    """Per-tensor FP8 scale amax/448 (a value is stored as q*scale), kept as an FP32 number."""
    amax = float(np.max(np.abs(x))) if x.size else 0.0
    if amax == 0.0:
        return 1.0
    return float(np.float32(amax / E4M3_MAX))


def layer_slices(arch: str, n: int, widths):
    """(name, slice) of each operand tensor in the flat parameter vector."""
    out = []
    if arch == "rbm":
        (m,) = widths
        out.append(("a", slice(0, n)))
        out.append(("b", slice(n, n + m)))
        out.append(("W", slice(n + m, n + m + m * n)))
        return out
    off, prev = 0, n
    for l, w in enumerate(widths):
        out.append((f"W{l + 1}", slice(off, off + w * prev)))
        off += w * prev
        out.append((f"b{l + 1}", slice(off, off + w)))
        off += w
        prev = w
    return out


def downcast(params: np.ndarray, arch: str, n: int, widths, dtype: str):
    """The downcast of the FP64 master to the sampling copy (Sec. IV.B, two-copy scheme).

    Returns (rounded parameter values as FP64, per-tensor scales).  For E4M3
    every tensor gets the scale amax/448 and is stored as round(x/scale)*scale;
    other formats round each value directly.
    """
    params = np.asarray(params, dtype=np.float64)
    if dtype != "e4m3":
        return round_to(params, dtype), {}
    out = np.empty_like(params)
    scales = {}
    for name, sl in layer_slices(arch, n, widths):
        sc = e4m3_scale(params[sl])
        scales[name] = sc
        out[sl] = round_to(params[sl] / sc, "e4m3") * sc
    return out, scales


def e4m3_act_scales(rounded: np.ndarray, n: int, widths) -> dict:
    """E4M3 scales of the hidden-layer outputs of a dense network (the inputs of
    layers 2..L), {l + 1: scale of the output of layer l} for l < L - 1.

    The paper fixes no FP8 recipe (App. A lists FP16/BF16/FP32/FP64).  Reading:
    a per-layer power of two 2^ceil(log2(B_l / 448)), where B_l bounds |h_l|
    over every spin configuration, computed on the rounded weights:
    B_0 = 1 (spins), B_l = max_k (sum_i |W_l[k, i]| B_{l-1} + |b_l[k]|) (ReLU
    never increases a magnitude).  No value can exceed 448 after scaling, and
    multiplying by a power of two is exact, so a layer input is stored as
    q * scale with q = RNE_e4m3(h / scale) and no saturation."""
    out = {}
    B, off, prev = 1.0, 0, n
    rounded = np.asarray(rounded, dtype=np.float64)
    for l, w in enumerate(widths[:-1]):
        W = rounded[off:off + w * prev].reshape(w, prev)
        off += w * prev
        b = rounded[off:off + w]
        off += w
        B = float(np.max(np.abs(W).sum(axis=1) * B + np.abs(b)))
        out[l + 1] = float(2.0 ** np.ceil(np.log2(B / E4M3_MAX))) if B > 0 else 1.0
        prev = w
    return out


# ---------------------------------------------------------------------------
# Models and Hamiltonians
# ---------------------------------------------------------------------------

class OracleModel:
    """A log-amplitude the oracle can evaluate (RBM, dense network, or lookup table)."""

    def __init__(self, arch: str, n: int, widths=(), params=None, act_dtype: str = "f64",
                 marshall: bool = False, lattice=None, table_logamp=None, table_sign=None,
                 act_scales=None):
        self.arch = arch
        self.n = n
        self.widths = tuple(widths)
        self.params = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        self.table_logamp = None if table_logamp is None else np.ascontiguousarray(table_logamp, np.float64)
        self.table_sign = None if table_sign is None else np.ascontiguousarray(table_sign, np.int8)
        self.act_dtype = act_dtype
        self.act_scales = dict(act_scales) if act_scales else None
        s = _Model()
        s.arch = {"rbm": RBM, "ffnn": FFNN, "table": TABLE}[arch]
        s.n_visible = n
        s.n_layers = len(self.widths) if arch != "table" else 0
        for k, w in enumerate(self.widths):
            s.widths[k] = w
        s.act_dtype = DTYPES[act_dtype]
        for k in range(MAX_LAYERS):
            s.act_scale[k] = 1.0
        if act_scales:
            for k, v in act_scales.items():
                s.act_scale[k] = v
        s.marshall = 1 if marshall else 0
        if lattice is not None:
            s.lat_dim, s.lat_L = lattice.dim, lattice.L
        s.params = _ptr(self.params) if self.params is not None else None
        s.table_logamp = _ptr(self.table_logamp) if self.table_logamp is not None else None
        s.table_sign = _ptr(self.table_sign) if self.table_sign is not None else None
        self._s = s

    @property
    def ref(self):
        return ctypes.byref(self._s)

    @property
    def n_params(self) -> int:
        return int(lib().orc_num_params(self.ref))

    def logamp(self, samples: np.ndarray):
        """log|psi| and sign(psi) of each row of `samples` (int8 +-1)."""
        samples = np.ascontiguousarray(samples, dtype=np.int8).reshape(-1, self.n)
        out = np.empty(samples.shape[0])
        sg = np.empty(samples.shape[0], dtype=np.int32)
        lib().orc_logamp_batch(self.ref, _ptr(samples), samples.shape[0], _ptr(out), _ptr(sg))
        return out, sg


def model_from_workload(wl, params=None, dtype: str = "f64") -> OracleModel:
    """The oracle's model for a workload, optionally emulating a reduced format."""
    import workloads
    m = wl.model
    p = workloads.params_for(wl) if params is None else params
    rounded, _ = downcast(p, m.arch, m.n_visible, m.widths, dtype)
    act, scales = dtype, None
    if dtype == "e4m3":
        # RBM: the only layer input is the spins (exact); dense: layer inputs with per-layer power-of-two scales
        act, scales = ("e4m3", e4m3_act_scales(rounded, m.n_visible, m.widths)) if m.arch == "ffnn" else ("f64", None)
    return OracleModel(m.arch, m.n_visible, m.widths, rounded, act_dtype=act, marshall=wl.ham.marshall,
                       lattice=wl.ham.lattice, act_scales=scales)


def ham_struct(ham) -> _Ham:
    h = _Ham()
    h.kind = TFIM if ham.kind == "tfim" else HEIS
    h.dim, h.L, h.pbc = ham.lattice.dim, ham.lattice.L, 1 if ham.lattice.pbc else 0
    h.J, h.h = ham.J, ham.h
    return h


def bonds(dim: int, L: int, pbc: bool = True) -> np.ndarray:
    nb = lib().orc_bonds(dim, L, 1 if pbc else 0, None)
    out = np.empty((max(nb, 1), 2), dtype=np.int32)
    lib().orc_bonds(dim, L, 1 if pbc else 0, _ptr(out))
    return out[:nb]


# ---------------------------------------------------------------------------
# Philox, chain initialisation, sampling, replay
# ---------------------------------------------------------------------------

def philox(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def init_chain(n: int, move: str, seed: int, chain: int, instance: int = 0) -> np.ndarray:
    s = np.empty(n, dtype=np.int8)
    lib().orc_init_chain(n, FLIP if move == "flip" else EXCHANGE, seed, chain, instance, _ptr(s))
    return s


def make_cfg(n_chains, n_sweeps, n_burnin, move="flip", seed=0, step_offset=0, instance_id=0,
             init_chains=True, sweep_size=0) -> _Cfg:
    c = _Cfg()
    c.n_chains, c.n_sweeps, c.n_burnin, c.sweep_size = n_chains, n_sweeps, n_burnin, sweep_size
    c.move = FLIP if move == "flip" else EXCHANGE
    c.seed, c.step_offset, c.instance_id = seed, step_offset, instance_id
    c.init_chains = 1 if init_chains else 0
    return c


def sample(model: OracleModel, cfg: _Cfg, chain_state=None):
    """Plain MH; returns (chain_state, samples [sweeps][chains][N], logpsi, n_accepted)."""
    N, C = model.n, cfg.n_chains
    st = np.zeros((C, N), dtype=np.int8) if chain_state is None else np.ascontiguousarray(chain_state, np.int8).copy()
    smp = np.empty((cfg.n_sweeps, C, N), dtype=np.int8)
    lp = np.empty((cfg.n_sweeps, C))
    acc = np.empty(C, dtype=np.uint64)
    rc = lib().orc_sample(model.ref, ctypes.byref(cfg), _ptr(st), _ptr(smp), _ptr(lp), _ptr(acc))
    if rc != 0:
        raise ValueError("oracle sample rejected its arguments")
    return st, smp, lp, acc


def replay(model: OracleModel, cfg: _Cfg, chain_ids, start_states, tr_site, tr_ubits, tr_delta, tr_acc,
           tau_rel: float = 1e-5):
    """Check a device decision trace step by step (see orc_replay)."""
    chain_ids = np.ascontiguousarray(chain_ids, dtype=np.int32)
    start_states = np.ascontiguousarray(start_states, dtype=np.int8)
    tr_site = np.ascontiguousarray(tr_site, dtype=np.int32)
    tr_ubits = np.ascontiguousarray(tr_ubits, dtype=np.uint32)
    tr_delta = np.ascontiguousarray(tr_delta, dtype=np.float32)
    tr_acc = np.ascontiguousarray(tr_acc, dtype=np.uint8)
    T, K = tr_site.shape
    end = np.empty((T, model.n), dtype=np.int8)
    st = np.zeros(5)
    lib().orc_replay(model.ref, ctypes.byref(cfg), T, _ptr(chain_ids), _ptr(start_states), K, _ptr(tr_site),
                     _ptr(tr_ubits), _ptr(tr_delta), _ptr(tr_acc), tau_rel, _ptr(end), _ptr(st))
    return {"site_u_mismatch": int(st[0]), "decision_mismatch": int(st[1]), "near_ties": int(st[2]),
            "decisions_equal": int(st[3]), "max_delta_err": float(st[4]), "end_states": end}


# ---------------------------------------------------------------------------
# Local energies, log-derivatives, averages
# ---------------------------------------------------------------------------

def local_energy(model: OracleModel, ham, samples: np.ndarray) -> np.ndarray:
    samples = np.ascontiguousarray(samples, dtype=np.int8).reshape(-1, model.n)
    out = np.empty(samples.shape[0])
    h = ham_struct(ham)
    lib().orc_local_energy(model.ref, ctypes.byref(h), _ptr(samples), samples.shape[0], _ptr(out))
    return out


def logpsi_grad(model: OracleModel, samples: np.ndarray, want_O: bool = True):
    samples = np.ascontiguousarray(samples, dtype=np.int8).reshape(-1, model.n)
    n = samples.shape[0]
    lp = np.empty(n)
    O = np.empty((n, model.n_params)) if want_O else None
    lib().orc_logpsi_grad(model.ref, _ptr(samples), n, _ptr(lp), _ptr(O))
    return lp, O


def stats(eloc: np.ndarray, n_chains: int) -> np.ndarray:
    e = np.ascontiguousarray(eloc, dtype=np.float64)
    out = np.empty(4)
    lib().orc_stats(_ptr(e), e.size, n_chains, _ptr(out))
    return out


def forces(O: np.ndarray, eloc: np.ndarray, weights=None) -> np.ndarray:
    O = np.ascontiguousarray(O, dtype=np.float64)
    e = np.ascontiguousarray(eloc, dtype=np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    F = np.empty(O.shape[1])
    lib().orc_forces(_ptr(O), _ptr(e), _ptr(w), O.shape[0], O.shape[1], _ptr(F))
    return F


def smatrix(O: np.ndarray, weights=None) -> np.ndarray:
    O = np.ascontiguousarray(O, dtype=np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    S = np.empty((O.shape[1], O.shape[1]))
    lib().orc_smatrix(_ptr(O), _ptr(w), O.shape[0], O.shape[1], _ptr(S))
    return S


def noise_zeta(configs: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """zeta(x) of the noisy target log pi~ = log pi + zeta (Sec. IV.A): sigma times a
    standard normal fixed per configuration (Philox keyed by the configuration
    bits, Box-Muller), FP64, one value per row of `configs` (N <= 128)."""
    c = np.ascontiguousarray(configs, dtype=np.int8)
    n, N = c.shape
    out = np.empty(n)
    lib().orc_noise_zeta(_ptr(c), n, N, float(sigma), int(seed), _ptr(out))
    return out


def sr_direction(O: np.ndarray, eloc: np.ndarray, shift: float, weights=None) -> np.ndarray:
    """Stochastic-reconfiguration direction in parameter space (App. I.2,
    Eq. eq:smat with the forces of Eq. eq:forces): delta solving
    (S + shift I) delta = F, S and F as defined above, FP64, dense solve."""
    S = smatrix(O, weights)
    F = forces(O, eloc, weights)
    return np.linalg.solve(S + shift * np.eye(S.shape[0]), F)


def tmatrix(O: np.ndarray) -> np.ndarray:
    O = np.ascontiguousarray(O, dtype=np.float64)
    T = np.empty((O.shape[0], O.shape[0]))
    lib().orc_tmatrix(_ptr(O), O.shape[0], O.shape[1], _ptr(T))
    return T


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(n)
