"""The no-allocation energy statistics against the allocating entry point, through the C ABI.

nqs_energy_stats_noalloc runs the kernels of nqs_energy_stats with their scratch
in a fixed device array instead of the library workspace, so the two must give
bit-identical statistics (same kernels, same fixed reduction order).  Two calls
in a row, the second on a smaller input (the array keeps the first call's
contents, which must not leak into the second), plus the case without an error
bar and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20782_amd as m
    m.load()
    from paper_2601_20782_amd import _abi
    return _abi.load()


def _both(lib, eloc, n_chains):
    from paper_2601_20782_amd import _abi
    s_ref = torch.full((4,), -1.0, dtype=torch.float64, device=DEV)
    s_new = torch.full((4,), -2.0, dtype=torch.float64, device=DEV)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p(eloc.data_ptr())
    assert lib.nqs_energy_stats(p, eloc.numel(), n_chains, ctypes.c_void_p(s_ref.data_ptr()), stream) == _abi.NQS_OK
    assert lib.nqs_energy_stats_noalloc(p, eloc.numel(), n_chains, ctypes.c_void_p(s_new.data_ptr()),
                                        stream) == _abi.NQS_OK
    torch.cuda.synchronize()
    return s_ref.cpu().numpy(), s_new.cpu().numpy()


def test_noalloc_stats_equal_the_allocating_entry_point(lib):
    g = torch.Generator(device="cpu").manual_seed(7)
    # first call: 64 sweeps x 4096 chains; second: a smaller ragged input, 10 chains
    for n, C in ((64 * 4096, 4096), (1000, 10)):
        eloc = (300.0 + 15.0 * torch.randn(n, generator=g, dtype=torch.float64)).to(DEV)
        ref, new = _both(lib, eloc, C)
        print(f"n={n} chains={C}: {new}", flush=True)
        assert np.array_equal(ref, new)
        assert new[3] == n and np.isfinite(new[2])
    # no error bar (n not a multiple of the chain count): stats[2] is NaN in both
    eloc = torch.linspace(-1.0, 1.0, 999, dtype=torch.float64, device=DEV)
    ref, new = _both(lib, eloc, 10)
    assert np.array_equal(ref, new, equal_nan=True) and np.isnan(new[2])


def test_noalloc_stats_refuse_too_many_chains(lib):
    from paper_2601_20782_amd import _abi
    C = 131072 - 512 + 1
    eloc = torch.zeros(2 * C, dtype=torch.float64, device=DEV)
    stats = torch.zeros(4, dtype=torch.float64, device=DEV)
    assert lib.nqs_energy_stats_noalloc(ctypes.c_void_p(eloc.data_ptr()), eloc.numel(), C,
                                        ctypes.c_void_p(stats.data_ptr()), None) == _abi.NQS_EINVAL
    # the largest count the scratch holds still works
    C = 131072 - 512
    eloc = torch.ones(2 * C, dtype=torch.float64, device=DEV)
    ref, new = _both(lib, eloc, C)
    assert np.array_equal(ref, new) and new[0] == 1.0 and new[2] == 0.0
