"""Python binding of libnqs: mixed-precision Metropolis-Hastings sampling of
neural quantum states on MI355X (gfx950).

Every function here marshals arguments for the C entry point of the same name
(include/nqs.h) and calls it on the current HIP stream; all computation runs
in the library's kernels.  PyTorch supplies device memory and streams only.
There is no CPU fallback: importing the package works without a GPU, but any
call needs the built libnqs.so and a device.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import DTYPE_CODES, NqsError, check, load

LANES_TUNED = -2   # SampleConfig.lanes_per_chain: the measured launch plan (include/nqs.h NQS_LANES_TUNED)

__all__ = [
    "Model", "SampleConfig", "Hamiltonian", "nqs_sample", "nqs_sample_checked", "nqs_sample_batched", "nqs_sample_plan", "nqs_local_energy", "nqs_energy_stats", "nqs_energy_stats_noalloc", "nqs_logpsi_grad",
    "nqs_logpsi_grad_cols", "nqs_forces", "nqs_gram", "nqs_sample_gram", "nqs_sample_gram_factored",
    "nqs_sr_solve", "nqs_sr_solve_mixed", "nqs_sr_solve_complex", "nqs_sr_update", "nqs_sample_noisy", "nqs_probe_rate", "nqs_local_energy_complex", "nqs_downcast", "LogPsi", "NqsError", "load",
    "LANES_TUNED",
]


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libnqs takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libnqs takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype(d) -> int:
    return DTYPE_CODES[d] if isinstance(d, str) else int(d)


class Model:
    """Handle to a library-owned model (FP64 master + reduced-precision copies)."""

    def __init__(self, arch: str, n_visible: int, widths: Sequence[int], params, marshall: bool = False,
                 lat_dim: int = 0, lat_L: int = 0, n_layers: Optional[int] = None):
        lib = load()
        d = _abi.ModelDesc()
        d.arch = {"rbm": _abi.RBM, "ffnn": _abi.FFNN, "rescnn": _abi.RESCNN, "crbm": _abi.CRBM}[arch]
        d.n_visible = n_visible
        d.n_layers = len(widths) if n_layers is None else n_layers
        for k, w in enumerate(widths):
            d.widths[k] = int(w)
        d.marshall = 1 if marshall else 0
        d.lat_dim, d.lat_L = lat_dim, lat_L
        self.desc = d
        self.arch, self.n_visible, self.widths = arch, n_visible, tuple(widths)
        p = np.ascontiguousarray(params, dtype=np.float64)
        h = ctypes.c_void_p()
        check(lib.nqs_model_create(ctypes.byref(d), p.ctypes.data_as(ctypes.c_void_p), p.size, ctypes.byref(h)))
        self._h = h

    @classmethod
    def rescnn(cls, L: int, F: int, R: int, params):
        """Residual convolutional network with F filters and R blocks on the periodic L x L lattice."""
        return cls("rescnn", L * L, (F,), params, lat_dim=2, lat_L=L, n_layers=R)

    @classmethod
    def from_workload(cls, wl, params=None):
        import workloads as _w   # seeded synthetic inputs (no method arithmetic)
        m = wl.model
        p = _w.params_for(wl) if params is None else params
        lat = wl.ham.lattice
        return cls(m.arch, m.n_visible, m.widths, p, marshall=wl.ham.marshall, lat_dim=lat.dim, lat_L=lat.L)

    @property
    def handle(self):
        return self._h

    @property
    def n_params(self) -> int:
        return int(load().nqs_model_num_params(self._h))

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float64)
        check(load().nqs_model_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size))

    def set_params_device(self, params: torch.Tensor, stream=None) -> None:
        check(load().nqs_model_set_params_device(self._h, _ptr(params), params.numel(), _stream(stream)))

    def prepare(self, dtype, stream=None) -> None:
        """Build the `dtype` sampling copy from the FP64 master now (the downcast step)."""
        check(load().nqs_model_prepare(self._h, _dtype(dtype), _stream(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load().nqs_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SampleConfig:
    n_chains: int
    n_sweeps: int
    n_burnin: int = 0
    move: str = "flip"
    dtype: str = "f32"
    seed: int = 0
    step_offset: int = 0
    instance_id: int = 0
    init_chains: bool = True
    sweep_size: int = 0
    chain_id_offset: int = 0
    lanes_per_chain: int = 0
    refresh_sweeps: int = 0

    def to_c(self) -> _abi.SampleCfg:
        c = _abi.SampleCfg()
        c.n_chains, c.n_sweeps, c.n_burnin, c.sweep_size = self.n_chains, self.n_sweeps, self.n_burnin, self.sweep_size
        c.move = _abi.MOVE_FLIP if self.move == "flip" else _abi.MOVE_EXCHANGE
        c.dtype = _dtype(self.dtype)
        c.init_chains = 1 if self.init_chains else 0
        c.seed, c.step_offset, c.instance_id = self.seed, self.step_offset, self.instance_id
        c.chain_id_offset = self.chain_id_offset
        c.lanes_per_chain = self.lanes_per_chain
        c.refresh_sweeps = self.refresh_sweeps
        return c


@dataclass
class Hamiltonian:
    kind: str          # "tfim" | "heisenberg"
    dim: int
    L: int
    J: float = 1.0
    h: float = 0.0
    pbc: bool = True

    @classmethod
    def from_workload(cls, ham):
        return cls(ham.kind, ham.lattice.dim, ham.lattice.L, ham.J, ham.h, ham.lattice.pbc)

    def to_c(self) -> _abi.HamDesc:
        h = _abi.HamDesc()
        h.kind = _abi.TFIM if self.kind == "tfim" else _abi.HEISENBERG
        h.dim, h.L, h.pbc = self.dim, self.L, 1 if self.pbc else 0
        h.J, h.h = self.J, self.h
        return h


def nqs_downcast(src: torch.Tensor, dtype, dst: torch.Tensor, scale_out: Optional[torch.Tensor] = None,
                 stream=None) -> None:
    assert src.dtype == torch.float64 and dst.dtype == torch.float32 and dst.numel() == src.numel()
    check(load().nqs_downcast(_ptr(src), src.numel(), _dtype(dtype), _ptr(dst), _ptr(scale_out), _stream(stream)))


def _trace_struct(trace: Optional[dict], cfg: "SampleConfig", N: int):
    if trace is None:
        return None
    tr = _abi.Trace()
    tr.n_chains_traced = trace["n"]
    total = (cfg.n_sweeps + cfg.n_burnin) * (cfg.sweep_size or N)
    for key, dt in (("site", torch.int32), ("ubits", torch.int32), ("delta", torch.float32), ("accepted", torch.uint8)):
        t = trace[key]
        assert t.dtype == dt and t.numel() == trace["n"] * total, key
        setattr(tr, key, t.data_ptr())
    return tr


def nqs_sample_plan(model: Model, cfg: SampleConfig, stream=None) -> dict:
    """Launch plan of the RBM sampler for this model and cfg (measured when cfg.lanes_per_chain is LANES_TUNED)."""
    plan = _abi.LaunchPlan()
    c = cfg.to_c()
    check(load().nqs_sample_plan(model.handle, ctypes.byref(c), ctypes.byref(plan), _stream(stream)))
    return {"lanes_per_chain": plan.lanes_per_chain, "units_per_lane": plan.units_per_lane,
            "chains_per_block": plan.chains_per_block, "table_in_lds": bool(plan.table_in_lds),
            "tuned": bool(plan.tuned), "tuned_ms": plan.tuned_ms}


def nqs_sample(model: Model, cfg: SampleConfig, chain_state: torch.Tensor, samples: Optional[torch.Tensor] = None,
               logpsi: Optional[torch.Tensor] = None, n_accepted: Optional[torch.Tensor] = None,
               trace: Optional[dict] = None, stream=None) -> None:
    N = model.n_visible
    assert chain_state.dtype == torch.int8 and chain_state.numel() == cfg.n_chains * N
    if samples is not None:
        assert samples.dtype == torch.int8 and samples.numel() == cfg.n_sweeps * cfg.n_chains * N
    if logpsi is not None:
        assert logpsi.dtype == torch.float32 and logpsi.numel() == cfg.n_sweeps * cfg.n_chains
    if n_accepted is not None:
        assert n_accepted.dtype in (torch.int64, torch.uint64) and n_accepted.numel() == cfg.n_chains
    tr = _trace_struct(trace, cfg, N)
    c = cfg.to_c()
    check(load().nqs_sample(model.handle, ctypes.byref(c), _ptr(chain_state), _ptr(samples), _ptr(logpsi),
                            _ptr(n_accepted), ctypes.byref(tr) if tr is not None else None, _stream(stream)))


def nqs_sample_checked(model: Model, cfg: SampleConfig, chain_state: torch.Tensor,
                       samples: Optional[torch.Tensor] = None, logpsi: Optional[torch.Tensor] = None,
                       n_accepted: Optional[torch.Tensor] = None, trace: Optional[dict] = None, stuck_after: int = 0,
                       nonfinite: Optional[torch.Tensor] = None, longest_stuck: Optional[torch.Tensor] = None,
                       drift: Optional[torch.Tensor] = None, stream=None) -> dict:
    """nqs_sample with the run-time detectors (include/nqs.h nqs_sample_checked).  Returns the host summary;
    a non-finite log-ratio is reported as status NQS_ENUMERIC in it rather than raised."""
    N = model.n_visible
    assert chain_state.dtype == torch.int8 and chain_state.numel() == cfg.n_chains * N
    if samples is not None:
        assert samples.dtype == torch.int8 and samples.numel() == cfg.n_sweeps * cfg.n_chains * N
    if logpsi is not None:
        assert logpsi.dtype == torch.float32 and logpsi.numel() == cfg.n_sweeps * cfg.n_chains
    if n_accepted is not None:
        assert n_accepted.dtype in (torch.int64, torch.uint64) and n_accepted.numel() == cfg.n_chains
    for t, dt in ((nonfinite, (torch.int64, torch.uint64)), (longest_stuck, (torch.int32,)), (drift, (torch.float32,))):
        if t is not None:
            assert t.dtype in dt and t.numel() == cfg.n_chains
    tr = _trace_struct(trace, cfg, N)
    d = _abi.SampleDiag()
    d.stuck_after = int(stuck_after)
    d.nonfinite, d.longest_stuck, d.drift = _ptr(nonfinite), _ptr(longest_stuck), _ptr(drift)
    c = cfg.to_c()
    st = load().nqs_sample_checked(model.handle, ctypes.byref(c), _ptr(chain_state), _ptr(samples), _ptr(logpsi),
                                   _ptr(n_accepted), ctypes.byref(tr) if tr is not None else None, ctypes.byref(d),
                                   _stream(stream))
    if st != _abi.NQS_ENUMERIC:
        check(st)
    return {"status": int(st), "total_nonfinite": int(d.total_nonfinite), "chains_stuck": int(d.chains_stuck),
            "max_drift": float(d.max_drift)}


def nqs_sample_noisy(model: Model, cfg: SampleConfig, noise_sigma: float, noise_seed: int, chain_state: torch.Tensor,
                     samples: Optional[torch.Tensor] = None, logpsi: Optional[torch.Tensor] = None,
                     n_accepted: Optional[torch.Tensor] = None, stream=None) -> None:
    N = model.n_visible
    assert chain_state.dtype == torch.int8 and chain_state.numel() == cfg.n_chains * N
    if samples is not None:
        assert samples.dtype == torch.int8 and samples.numel() == cfg.n_sweeps * cfg.n_chains * N
    if logpsi is not None:
        assert logpsi.dtype == torch.float32 and logpsi.numel() == cfg.n_sweeps * cfg.n_chains
    if n_accepted is not None:
        assert n_accepted.dtype in (torch.int64, torch.uint64) and n_accepted.numel() == cfg.n_chains
    c = cfg.to_c()
    check(load().nqs_sample_noisy(model.handle, ctypes.byref(c), float(noise_sigma), int(noise_seed),
                                  _ptr(chain_state), _ptr(samples), _ptr(logpsi), _ptr(n_accepted), _stream(stream)))


def nqs_sample_batched(jobs, mode: int = 0, stream=None) -> None:
    """Sample many RBM instances; `jobs` is a list of dicts with keys model, cfg, chain_state and
    optionally samples, logpsi, n_accepted, trace (same meaning as for nqs_sample)."""
    arr = (_abi.SampleJob * len(jobs))()
    keep = []
    for k, j in enumerate(jobs):
        model, cfg = j["model"], j["cfg"]
        N = model.n_visible
        assert j["chain_state"].dtype == torch.int8 and j["chain_state"].numel() == cfg.n_chains * N
        if j.get("samples") is not None:
            assert j["samples"].numel() == cfg.n_sweeps * cfg.n_chains * N
        arr[k].model = model.handle.value
        arr[k].cfg = cfg.to_c()
        arr[k].chain_state = j["chain_state"].data_ptr()
        arr[k].samples = j["samples"].data_ptr() if j.get("samples") is not None else None
        arr[k].logpsi = j["logpsi"].data_ptr() if j.get("logpsi") is not None else None
        arr[k].n_accepted = j["n_accepted"].data_ptr() if j.get("n_accepted") is not None else None
        tr = _trace_struct(j.get("trace"), cfg, N)
        keep.append(tr)
        arr[k].trace = ctypes.addressof(tr) if tr is not None else None
    check(load().nqs_sample_batched(arr, len(jobs), mode, _stream(stream)))


def nqs_local_energy(model: Model, ham: Hamiltonian, samples: torch.Tensor, eloc: torch.Tensor,
                     eval_dtype="f32", stream=None) -> None:
    n = samples.numel() // model.n_visible
    assert samples.dtype == torch.int8 and eloc.dtype == torch.float64 and eloc.numel() == n
    h = ham.to_c()
    check(load().nqs_local_energy(model.handle, ctypes.byref(h), _ptr(samples), n, _dtype(eval_dtype), _ptr(eloc),
                                  _stream(stream)))


def nqs_local_energy_complex(model: Model, ham: Hamiltonian, samples: torch.Tensor, eloc_re: torch.Tensor,
                             eloc_im: torch.Tensor, eval_dtype="f32", stream=None) -> None:
    n = samples.numel() // model.n_visible
    assert samples.dtype == torch.int8 and eloc_re.dtype == torch.float64 and eloc_re.numel() == n
    assert eloc_im.dtype == torch.float64 and eloc_im.numel() == n
    h = ham.to_c()
    check(load().nqs_local_energy_complex(model.handle, ctypes.byref(h), _ptr(samples), n, _dtype(eval_dtype),
                                          _ptr(eloc_re), _ptr(eloc_im), _stream(stream)))


def nqs_energy_stats(eloc: torch.Tensor, n_chains: int, stats: torch.Tensor, stream=None) -> None:
    assert eloc.dtype == torch.float64 and stats.dtype == torch.float64 and stats.numel() >= 4
    check(load().nqs_energy_stats(_ptr(eloc), eloc.numel(), n_chains, _ptr(stats), _stream(stream)))


def nqs_energy_stats_noalloc(eloc: torch.Tensor, n_chains: int, stats: torch.Tensor, stream=None) -> None:
    assert eloc.dtype == torch.float64 and stats.dtype == torch.float64 and stats.numel() >= 4
    check(load().nqs_energy_stats_noalloc(_ptr(eloc), eloc.numel(), n_chains, _ptr(stats), _stream(stream)))


def nqs_logpsi_grad(model: Model, samples: torch.Tensor, logpsi: Optional[torch.Tensor] = None,
                    O: Optional[torch.Tensor] = None, vjp_in: Optional[torch.Tensor] = None,
                    vjp_out: Optional[torch.Tensor] = None, stream=None) -> None:
    n = samples.numel() // model.n_visible
    P = model.n_params
    if O is not None:
        assert O.dtype == torch.float32 and O.numel() == n * P
    if logpsi is not None:
        assert logpsi.dtype == torch.float32 and logpsi.numel() == n
    if vjp_in is not None:
        assert vjp_in.dtype == torch.float32 and vjp_in.numel() == n
        assert vjp_out is not None and vjp_out.dtype == torch.float32 and vjp_out.numel() == P
    check(load().nqs_logpsi_grad(model.handle, _ptr(samples), n, _ptr(logpsi), _ptr(O), _ptr(vjp_in), _ptr(vjp_out),
                                 _stream(stream)))


def nqs_logpsi_grad_cols(model: Model, samples: torch.Tensor, p0: int, p1: int, O: torch.Tensor,
                         stream=None) -> None:
    n = samples.numel() // model.n_visible
    assert O.dtype == torch.float32 and O.numel() == n * (p1 - p0)
    check(load().nqs_logpsi_grad_cols(model.handle, _ptr(samples), n, p0, p1, _ptr(O), _stream(stream)))


def nqs_sample_gram(model: Model, samples: torch.Tensor, T: torch.Tensor, chunk_params: int = 0,
                    stream=None) -> None:
    n = samples.numel() // model.n_visible
    assert T.dtype == torch.float32 and T.numel() == n * n
    check(load().nqs_sample_gram(model.handle, _ptr(samples), n, chunk_params, _ptr(T), _stream(stream)))


def nqs_sample_gram_factored(model: Model, samples: torch.Tensor, T: torch.Tensor, stream=None) -> None:
    n = samples.numel() // model.n_visible
    assert T.dtype == torch.float32 and T.numel() == n * n
    check(load().nqs_sample_gram_factored(model.handle, _ptr(samples), n, _ptr(T), _stream(stream)))


def nqs_sr_solve(T: torch.Tensor, eloc: torch.Tensor, shift: float, y: torch.Tensor, tol: float = 1e-10,
                 max_iter: int = 1000, stream=None):
    """(T + shift) y = eloc - mean(eloc); returns (iterations, relative residual)."""
    n = eloc.numel()
    assert T.dtype == torch.float32 and T.numel() == n * n
    assert eloc.dtype == torch.float64 and y.dtype == torch.float64 and y.numel() == n
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    check(load().nqs_sr_solve(_ptr(T), _ptr(eloc), n, float(shift), float(tol), int(max_iter), _ptr(y),
                              ctypes.byref(it), ctypes.byref(rr), _stream(stream)))
    return it.value, rr.value


def nqs_sr_solve_mixed(T: torch.Tensor, eloc: torch.Tensor, shift: float, y: torch.Tensor, factor_dtype="bf16",
                       tol: float = 1e-10, max_iter: int = 1000, stream=None):
    """The same solve, preconditioned by a Cholesky factor computed in `factor_dtype`;
    returns (iterations, relative residual, replaced pivots, format used: a dtype
    name, or "jacobi")."""
    n = eloc.numel()
    assert T.dtype == torch.float32 and T.numel() == n * n
    assert eloc.dtype == torch.float64 and y.dtype == torch.float64 and y.numel() == n
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    nf = ctypes.c_int64(0)
    fu = ctypes.c_int32(0)
    check(load().nqs_sr_solve_mixed(_ptr(T), _ptr(eloc), n, float(shift), _dtype(factor_dtype), float(tol),
                                    int(max_iter), _ptr(y), ctypes.byref(it), ctypes.byref(rr), ctypes.byref(nf),
                                    ctypes.byref(fu), _stream(stream)))
    names = {v: k for k, v in DTYPE_CODES.items()}
    return it.value, rr.value, nf.value, names.get(fu.value, "jacobi")


def nqs_sr_solve_complex(T2: torch.Tensor, eloc_re: torch.Tensor, eloc_im: torch.Tensor, shift: float, y2: torch.Tensor,
                         tol: float = 1e-10, max_iter: int = 1000, stream=None):
    """(T + shift) z = eps - mean(eps) for a complex network, T given as its real 2n x 2n embedding T2
    (nqs_gram mode 3), y2 = (Re z, Im z); returns (iterations, relative residual)."""
    n = eloc_re.numel()
    assert T2.dtype == torch.float32 and T2.numel() == 4 * n * n
    assert eloc_re.dtype == torch.float64 and eloc_im.dtype == torch.float64 and eloc_im.numel() == n
    assert y2.dtype == torch.float64 and y2.numel() == 2 * n
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    check(load().nqs_sr_solve_complex(_ptr(T2), _ptr(eloc_re), _ptr(eloc_im), n, float(shift), float(tol),
                                      int(max_iter), _ptr(y2), ctypes.byref(it), ctypes.byref(rr), _stream(stream)))
    return it.value, rr.value


def nqs_sr_update(model: Model, samples: torch.Tensor, y: torch.Tensor, lr: float, master: torch.Tensor,
                  stream=None) -> None:
    n = samples.numel() // model.n_visible
    assert y.dtype == torch.float64 and y.numel() == (2 * n if model.arch == "crbm" else n)
    assert master.dtype == torch.float64 and master.numel() == model.n_params
    check(load().nqs_sr_update(model.handle, _ptr(samples), n, _ptr(y), float(lr), _ptr(master), _stream(stream)))


def nqs_forces(O: torch.Tensor, eloc: torch.Tensor, F: torch.Tensor, Omean: Optional[torch.Tensor] = None,
               stream=None) -> None:
    n, P = O.shape
    assert O.dtype == torch.float32 and eloc.dtype == torch.float64 and F.dtype == torch.float64 and F.numel() == P
    check(load().nqs_forces(_ptr(O), _ptr(eloc), n, P, _ptr(F), _ptr(Omean), _stream(stream)))


def nqs_gram(O: torch.Tensor, mode: int, out: torch.Tensor, stream=None) -> None:
    n, P = O.shape
    side = P if mode == 0 else (2 * n if mode == 3 else n)
    assert O.dtype == torch.float32 and out.dtype == torch.float32 and out.numel() == side * side
    check(load().nqs_gram(_ptr(O), n, P, mode, _ptr(out), _stream(stream)))


class LogPsi(torch.autograd.Function):
    """log psi(samples) as a function of the model parameters.

    forward: nqs_logpsi_grad without O; backward: the vector-Jacobian product
    of the hand-written backward kernel (grad_theta = sum_k g_k O_k).
    The `params` tensor only carries the autograd edge: the values used are
    the model's current parameters.
    """

    @staticmethod
    def forward(ctx, params: torch.Tensor, model: Model, samples: torch.Tensor):
        n = samples.numel() // model.n_visible
        out = torch.empty(n, dtype=torch.float32, device=samples.device)
        nqs_logpsi_grad(model, samples, logpsi=out)
        ctx.model = model
        ctx.save_for_backward(samples)
        ctx.pdtype = params.dtype
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (samples,) = ctx.saved_tensors
        g = grad_out.contiguous().to(torch.float32)
        vjp = torch.empty(ctx.model.n_params, dtype=torch.float32, device=samples.device)
        nqs_logpsi_grad(ctx.model, samples, vjp_in=g, vjp_out=vjp)
        return vjp.to(ctx.pdtype), None, None


def nqs_probe_rate(kind: str, size: int, src: Optional[torch.Tensor], dst: torch.Tensor, stream=None) -> float:
    """One launch of a rate microbenchmark (include/nqs_probe.h); returns its work (flops or bytes)."""
    w = ctypes.c_double(0.0)
    check(load().nqs_probe_rate(_abi.PROBE_KINDS[kind], int(size), _ptr(src) if src is not None else None, _ptr(dst),
                                ctypes.byref(w), _stream(stream)))
    return w.value
