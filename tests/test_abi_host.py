"""Host-side checks of the C interface (no GPU needed): the library loads, it
exports every function the headers under include/ declare, and argument validation rejects
bad calls before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    inc = os.path.join(ROOT, "include")
    text = "\n".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s\*]+(nqs_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2601_20782_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libnqs.so is not built (run __graft_entry__.build())")
    return _abi.load()


def test_exports_every_declared_symbol(lib):
    from paper_2601_20782_amd import _abi
    declared = _declared_functions()
    assert len(declared) >= 14
    assert sorted(_abi.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_version_and_error_strings(lib):
    assert b"gfx950" in lib.nqs_version()
    assert isinstance(lib.nqs_last_error(), bytes)


def test_model_create_rejects_bad_descriptions(lib):
    from paper_2601_20782_amd import _abi
    out = ctypes.c_void_p()
    p = np.zeros(10)
    d = _abi.ModelDesc()
    d.arch, d.n_visible, d.n_layers = _abi.RBM, 16, 1
    d.widths[0] = 16
    # wrong parameter count: rejected before any device work
    assert lib.nqs_model_create(ctypes.byref(d), p.ctypes.data_as(ctypes.c_void_p), 10, ctypes.byref(out)) == _abi.NQS_EINVAL
    assert b"n_params" in lib.nqs_last_error()
    # NaN parameters
    P = 16 + 16 + 256
    bad = np.zeros(P)
    bad[7] = np.nan
    assert lib.nqs_model_create(ctypes.byref(d), bad.ctypes.data_as(ctypes.c_void_p), P, ctypes.byref(out)) == _abi.NQS_ENUMERIC
    # unknown architecture / bad widths
    d.arch = 7
    assert lib.nqs_model_create(ctypes.byref(d), bad.ctypes.data_as(ctypes.c_void_p), P, ctypes.byref(out)) == _abi.NQS_EINVAL
    d.arch, d.n_layers = _abi.FFNN, 0
    assert lib.nqs_model_create(ctypes.byref(d), bad.ctypes.data_as(ctypes.c_void_p), P, ctypes.byref(out)) == _abi.NQS_EINVAL
    # Marshall lattice must match N
    d.arch, d.n_layers, d.marshall, d.lat_dim, d.lat_L = _abi.RBM, 1, 1, 2, 5
    assert lib.nqs_model_create(ctypes.byref(d), bad.ctypes.data_as(ctypes.c_void_p), P, ctypes.byref(out)) == _abi.NQS_EINVAL


def test_calls_without_model_are_rejected(lib):
    from paper_2601_20782_amd import _abi
    cfg = _abi.SampleCfg()
    cfg.n_chains = 4
    assert lib.nqs_sample(None, ctypes.byref(cfg), None, None, None, None, None, None) == _abi.NQS_EINVAL
    assert lib.nqs_local_energy(None, None, None, 1, 1, None, None) == _abi.NQS_EINVAL
    assert lib.nqs_energy_stats(None, 0, 1, None, None) == _abi.NQS_EINVAL
    assert lib.nqs_energy_stats_noalloc(None, 0, 1, None, None) == _abi.NQS_EINVAL
    assert lib.nqs_forces(None, None, 0, 5, None, None, None) == _abi.NQS_EINVAL
    assert lib.nqs_gram(None, 4, 4, 3, None, None) == _abi.NQS_EINVAL
    assert lib.nqs_downcast(None, 5, 1, None, None, None) == _abi.NQS_EINVAL
    assert lib.nqs_downcast(None, 0, 1, None, None, None) == _abi.NQS_OK   # empty input is a no-op


def test_new_entry_points_reject_bad_arguments(lib):
    """The SR solves, the complex local energies and the rate probes validate
    their arguments before any device work."""
    from paper_2601_20782_amd import _abi
    it, rr = ctypes.c_int32(0), ctypes.c_double(0.0)
    nf, fu = ctypes.c_int64(0), ctypes.c_int32(0)
    fake = ctypes.c_void_p(16)
    # n = 0, a NULL T, a negative shift, an unsupported factor format
    assert lib.nqs_sr_solve_mixed(fake, fake, 0, 1e-2, _abi.BF16, 1e-8, 10, fake, ctypes.byref(it), ctypes.byref(rr),
                                  ctypes.byref(nf), ctypes.byref(fu), None) == _abi.NQS_EINVAL
    assert lib.nqs_sr_solve_mixed(None, fake, 8, 1e-2, _abi.BF16, 1e-8, 10, fake, ctypes.byref(it), ctypes.byref(rr),
                                  ctypes.byref(nf), ctypes.byref(fu), None) == _abi.NQS_EINVAL
    assert lib.nqs_sr_solve_mixed(fake, fake, 8, -1.0, _abi.BF16, 1e-8, 10, fake, ctypes.byref(it), ctypes.byref(rr),
                                  ctypes.byref(nf), ctypes.byref(fu), None) == _abi.NQS_EINVAL
    for fmt in (_abi.F64, _abi.FP8_E4M3, 9):
        assert lib.nqs_sr_solve_mixed(fake, fake, 8, 1e-2, fmt, 1e-8, 10, fake, ctypes.byref(it), ctypes.byref(rr),
                                      ctypes.byref(nf), ctypes.byref(fu), None) == _abi.NQS_EINVAL
    assert b"factor dtype" in lib.nqs_last_error()
    assert lib.nqs_sr_solve_mixed(fake, fake, 70000, 1e-2, _abi.F32, 1e-8, 10, fake, ctypes.byref(it),
                                  ctypes.byref(rr), ctypes.byref(nf), ctypes.byref(fu), None) == _abi.NQS_EINVAL
    # the complex SR solve: n = 0, NULL buffers, a negative shift; the complex T needs an even column count
    assert lib.nqs_sr_solve_complex(fake, fake, fake, 0, 1e-2, 1e-8, 10, fake, ctypes.byref(it), ctypes.byref(rr),
                                    None) == _abi.NQS_EINVAL
    assert lib.nqs_sr_solve_complex(fake, None, fake, 8, 1e-2, 1e-8, 10, fake, ctypes.byref(it), ctypes.byref(rr),
                                    None) == _abi.NQS_EINVAL
    assert lib.nqs_sr_solve_complex(fake, fake, fake, 8, -1.0, 1e-8, 10, fake, ctypes.byref(it), ctypes.byref(rr),
                                    None) == _abi.NQS_EINVAL
    assert lib.nqs_gram(fake, 4, 5, 3, fake, None) == _abi.NQS_EINVAL
    assert b"[n][2P']" in lib.nqs_last_error()
    assert lib.nqs_gram(fake, 4, 6, 4, fake, None) == _abi.NQS_EINVAL
    # complex local energies without a model
    h = _abi.HamDesc()
    assert lib.nqs_local_energy_complex(None, ctypes.byref(h), fake, 4, _abi.F32, fake, fake, None) == _abi.NQS_EINVAL
    # probes: unknown kind, bad sizes, unaligned or missing buffers, NULL work
    w = ctypes.c_double(0.0)
    assert lib.nqs_probe_rate(99, 10, None, fake, ctypes.byref(w), None) == _abi.NQS_EINVAL
    assert lib.nqs_probe_rate(_abi.PROBE_KINDS["fma_f32"], 0, None, fake, ctypes.byref(w), None) == _abi.NQS_EINVAL
    assert lib.nqs_probe_rate(_abi.PROBE_KINDS["fma_f32"], 10, None, None, ctypes.byref(w), None) == _abi.NQS_EINVAL
    assert lib.nqs_probe_rate(_abi.PROBE_KINDS["hbm_read"], 24, fake, fake, ctypes.byref(w), None) == _abi.NQS_EINVAL
    assert lib.nqs_probe_rate(_abi.PROBE_KINDS["hbm_copy"], 32, ctypes.c_void_p(20), fake, ctypes.byref(w),
                              None) == _abi.NQS_EINVAL
    assert lib.nqs_probe_rate(_abi.PROBE_KINDS["fma_f32"], 10, None, fake, None, None) == _abi.NQS_EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2601_20782_amd import _abi
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _abi.load()


def test_noalloc_stats_reject_more_chains_than_the_static_scratch(lib):
    """The no-allocation statistics hold at most 131072 - 512 chain means; a larger request is refused
    before any device call (so it is refused here, without a GPU)."""
    from paper_2601_20782_amd import _abi
    fake = ctypes.c_void_p(16)
    n_chains = 131072 - 512 + 1
    assert lib.nqs_energy_stats_noalloc(fake, 2 * n_chains, n_chains, fake, None) == _abi.NQS_EINVAL
    assert b"static scratch" in lib.nqs_last_error()


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the interface structs have the C layout: sizes and field offsets
    printed by a program compiled against include/nqs.h."""
    import shutil
    import subprocess
    from paper_2601_20782_amd import _abi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"nqs_model_desc": _abi.ModelDesc, "nqs_ham_desc": _abi.HamDesc, "nqs_sample_cfg": _abi.SampleCfg,
               "nqs_sample_job": _abi.SampleJob, "nqs_trace": _abi.Trace, "nqs_launch_plan": _abi.LaunchPlan,
               "nqs_sample_diag": _abi.SampleDiag}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "nqs.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
