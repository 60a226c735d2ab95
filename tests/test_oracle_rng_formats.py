"""Pins for the oracle's generator and reduced-precision formats (CPU only)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import exact

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# Philox4x32-10: known answers from rocRAND's independent implementation
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND known-answer program")
    d = tmp_path_factory.mktemp("kat")
    exe = str(d / "kat")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_kat.cpp")], check=True,
                   capture_output=True)

    def run(queries):
        text = "".join(f"{s} {c[0]} {c[1]} {c[2]} {c[3]}\n" for s, c in queries)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)

    return run


def test_philox_matches_rocrand(orc, rocrand_kat):
    rng = np.random.default_rng(7)
    queries = [(0, (0, 0, 0, 0)), (1, (0, 0, 0, 0)), (2**64 - 1, (1, 0, 0, 0)),
               (0x0123456789ABCDEF, (10, 0, 5, 0)), (42, (2**32 - 1, 7, 3, 0x101))]
    for _ in range(200):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        c = tuple(int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64))
        c = (c[0], c[1] % (2**29), c[2], c[3])   # keep 4*offset inside 64 bits
        queries.append((seed, c))
    ref = rocrand_kat(queries)
    for (seed, c), r in zip(queries, ref):
        got = oracle.philox(c, [seed & 0xFFFFFFFF, seed >> 32])
        assert list(got) == list(r.astype(np.uint32)), (seed, c)


def test_philox_uniform_and_index_statistics(orc):
    # chi^2 on site indices floor(r*N/2^32) and a KS test on u = (r>>8)*2^-24
    import scipy.stats
    n_sites, K = 100, 40000
    words = np.array([oracle.philox([k, 0, 3, 0], [11, 0]) for k in range(K // 4)]).ravel()
    sites = ((words.astype(np.uint64) * n_sites) >> 32).astype(np.int64)
    counts = np.bincount(sites, minlength=n_sites)
    chi2 = np.sum((counts - K / n_sites) ** 2 / (K / n_sites))
    assert scipy.stats.chi2.sf(chi2, n_sites - 1) > 1e-4
    u = (words >> 8).astype(np.float64) * 2.0**-24
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-4


def test_init_chain_flip_and_exchange(orc):
    s = np.array([oracle.init_chain(37, "flip", 5, c) for c in range(400)])
    assert set(np.unique(s)) == {-1, 1}
    assert abs(s.mean()) < 0.03
    e = np.array([oracle.init_chain(36, "exchange", 5, c) for c in range(400)])
    assert np.all(e.sum(axis=1) == 0)
    # every site is up half the time (the shuffle is unbiased)
    assert np.all(np.abs((e > 0).mean(axis=0) - 0.5) < 0.12)
    # different chains, different states
    assert len({row.tobytes() for row in e}) == 400


# ---------------------------------------------------------------------------
# Reduced-precision formats (App. A, Table A)
# ---------------------------------------------------------------------------

def _edge_values(rng):
    x = np.concatenate([
        rng.normal(0, 1, 20000), rng.normal(0, 0.02, 20000), rng.normal(0, 1e3, 5000),
        np.exp(rng.uniform(-40, 40, 20000)) * rng.choice([-1, 1], 20000),
        rng.uniform(-1e-5, 1e-5, 5000), [0.0, -0.0, 1.0, -1.0, 65504.0, 65519.9, 65520.0, 448.0, 464.0]])
    # values exactly on and next to half-ulp ties of bf16/f16
    base = rng.normal(0, 1, 2000).astype(np.float32).astype(np.float64)
    ties = []
    for b in base:
        for frac_bits in (8, 11):
            m, e = np.frexp(b)
            q = 2.0 ** (e - frac_bits)
            t = (np.floor(b / q) + 0.5) * q
            ties += [t, np.nextafter(t, np.inf), np.nextafter(t, -np.inf)]
    return np.concatenate([x, np.array(ties)])


def test_f16_rounding_matches_numpy(orc):
    x = _edge_values(np.random.default_rng(1))
    x = x[np.abs(x) < 1e6]
    ref = x.astype(np.float16).astype(np.float64)
    got = oracle.round_to(x, "f16")
    both_inf = np.isinf(ref) & np.isinf(got) & (np.sign(ref) == np.sign(got))
    assert np.all((got == ref) | both_inf)


def _nearest_even_bruteforce(x, fmt_dtype):
    """Nearest representable value by searching the neighbours of a candidate (ties to even code)."""
    import torch
    c = torch.tensor(x, dtype=torch.float64).to(fmt_dtype)
    bits = c.view(torch.int16).item()
    cands = []
    for d in (-1, 0, 1):
        v = torch.tensor([bits + d], dtype=torch.int16).view(fmt_dtype).to(torch.float64).item()
        cands.append((abs(v - x), (bits + d) & 1, v))
    cands.sort()
    best = [c for c in cands if c[0] == cands[0][0]]
    if len(best) > 1:
        best = [c for c in best if c[1] == 0]
    return best[0][2]


def test_bf16_and_f32_rounding_match_torch(orc):
    torch = pytest.importorskip("torch")
    x = _edge_values(np.random.default_rng(2))
    # On FP32-exact inputs torch's cast is a single RNE rounding.
    xf = x.astype(np.float32).astype(np.float64)
    ref_bf = torch.from_numpy(xf).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_to(xf, "bf16"), ref_bf)
    assert np.array_equal(oracle.round_to(x, "f32"), x.astype(np.float32).astype(np.float64))
    # On general FP64 inputs (torch's f64 cast goes through f32, a double rounding)
    # compare with a brute-force nearest-value search, ties to the even code.
    sel = x[np.isfinite(x) & (np.abs(x) < 1e30) & (np.abs(x) > 1e-30)]
    sel = np.concatenate([sel[-6000:], sel[:3000]])
    got = oracle.round_to(sel, "bf16")
    ref = np.array([_nearest_even_bruteforce(v, torch.bfloat16) for v in sel])
    assert np.array_equal(got, ref)


def test_e4m3_rounding_matches_torch(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-448, 448, 20000), rng.normal(0, 1, 20000), rng.normal(0, 0.01, 5000),
                        [0.0, 448.0, -448.0, 2.0**-9, 2.0**-10, 3 * 2.0**-11, 2.0**-6]])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_to(x, "e4m3"), ref)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "f32"])
def test_unit_roundoff_matches_table_a(orc, fmt):
    """Max relative rounding error of each format equals its unit round-off (Table A)."""
    printed = {}
    with open(os.path.join(HERE, "golden", "table_a_unit_roundoff.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, _, sig, err = line.split()
                printed[name] = (int(sig), float(err))
    sig, err = printed[fmt]
    u = exact.unit_roundoff(fmt)
    assert u == 2.0 ** -(sig + 1)
    if fmt != "f16":
        assert abs(u - err) / u < 2e-3          # printed to 3 significant digits
    else:
        assert abs(u - 4.88e-4) / u < 2e-3     # the printed 4.88e-5 is a misprint
        assert abs(err - 4.88e-5) < 1e-12
    x = np.random.default_rng(4).uniform(1.0, 2.0, 200000) * 2.0 ** np.random.default_rng(5).integers(-10, 10, 200000)
    rel = np.abs(oracle.round_to(x, fmt) - x) / np.abs(x)
    assert rel.max() <= u * (1 + 1e-12)
    assert rel.max() > 0.9 * u


def test_e4m3_downcast_scale(orc):
    rng = np.random.default_rng(6)
    p = rng.normal(0, 0.05, 5000)
    out, scales = oracle.downcast(p, "rbm", 50, (49,), "e4m3")
    sl = dict(oracle.layer_slices("rbm", 50, (49,)))
    for name, s in sl.items():
        sc = scales[name]
        q = out[s] / sc
        assert np.max(np.abs(q)) <= 448.0
        assert np.isclose(np.max(np.abs(q)), 448.0, rtol=1e-6)   # amax maps onto the largest code
        assert np.array_equal(oracle.round_to(q, "e4m3"), q)      # every value is an E4M3 code
