"""GPU parity of the mixed-precision SR solve: (T + shift) y = eps - mean eps
by FP64 conjugate gradients preconditioned with a Cholesky factor computed in
FP32, BF16 or FP16 (Sec. V's mixed-precision solvers for the preconditioning
step of App. I.2), against the FP64 dense solve.  T is the oracle's sample-space
Gram matrix of seeded log-derivatives, rounded to FP32 as the solver receives
it.  Every call goes through the C interface."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def nqs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_20782_amd as m
    m.load()
    return m


def _say(msg):
    print(msg, flush=True)


def _system(n, P, seed):
    rng = np.random.default_rng(seed)
    O = (rng.normal(size=(n, P)) + rng.normal(size=P)).astype(np.float32)
    T32 = oracle.tmatrix(O).astype(np.float32)
    eps = rng.normal(-3.0, 1.5, size=n)
    return T32, eps


# n = 64 (one tile), 65 and 129 (a last tile of one row), 300 (five tiles, the last one partly
# padding), 1000 (16 tiles)
@pytest.mark.parametrize("fmt", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("n,P,shift", [(64, 80, 1e-3), (65, 90, 1e-2), (129, 200, 1e-2), (300, 500, 1e-2),
                                       (1000, 1500, 1e-3)])
def test_mixed_solve_matches_dense_solve(nqs, fmt, n, P, shift):
    T32, eps = _system(n, P, n + P)
    T = torch.from_numpy(T32).to(DEV)
    e = torch.from_numpy(eps).to(DEV)
    y = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
    its, rr, fixed, used = nqs.nqs_sr_solve_mixed(T, e, shift, y, fmt, tol=1e-12, max_iter=500)
    yj = torch.empty_like(y)
    its_j, _ = nqs.nqs_sr_solve(T, e, shift, yj, tol=1e-12, max_iter=5000)
    b = eps - eps.mean()
    ref = np.linalg.solve(T32.astype(np.float64) + shift * np.eye(n), b)
    got = y.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.abs(ref).max()
    _say(f"  {fmt} n={n} shift={shift}: {its} iterations (Jacobi {its_j}), residual {rr:.1e}, "
         f"max |dy| / max |y| = {err:.1e}, {fixed} pivots replaced")
    assert rr <= 1e-12 and err <= 1e-8
    assert fixed == 0 and used == fmt
    assert its <= {"f32": 4, "f16": 12, "bf16": 40}[fmt] and its < its_j
    y2 = torch.empty_like(y)
    assert nqs.nqs_sr_solve_mixed(T, e, shift, y2, fmt, tol=1e-12, max_iter=500)[:2] == (its, rr)
    assert torch.equal(y, y2)


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_rank_deficient_with_tiny_shift(nqs, fmt):
    """P < n: T has rank P - 1 and T + 1e-6 a condition number near 1e7.  In
    BF16 the trailing pivots fall below the format's resolution: more than n / 8
    of them are replaced, so the solve moves to an FP32 factor (whose replaced
    pivots it reports), and the FP64 iteration reaches the FP64 residual."""
    n, P, shift = 200, 60, 1e-6
    T32, eps = _system(n, P, 5)
    T = torch.from_numpy(T32).to(DEV)
    y = torch.empty(n, dtype=torch.float64, device=DEV)
    its, rr, fixed, used = nqs.nqs_sr_solve_mixed(T, torch.from_numpy(eps).to(DEV), shift, y, fmt, tol=1e-11,
                                                  max_iter=2000)
    A = T32.astype(np.float64) + shift * np.eye(n)
    b = eps - eps.mean()
    res = np.linalg.norm(A @ y.cpu().numpy() - b) / np.linalg.norm(b)
    _say(f"  {fmt}: factor used {used}, {its} iterations, reported residual {rr:.1e}, FP64 residual {res:.1e}, "
         f"{fixed} pivots replaced")
    assert rr <= 1e-11 and res <= 1e-9
    assert used == "f32"


def test_edge_cases_and_rejections(nqs):
    # n = 1: the centred right-hand side is zero
    T = torch.ones(1, 1, dtype=torch.float32, device=DEV)
    y = torch.full((1,), 5.0, dtype=torch.float64, device=DEV)
    its, rr, fixed, used = nqs.nqs_sr_solve_mixed(T, torch.tensor([2.5], dtype=torch.float64, device=DEV), 0.1, y,
                                                  "bf16")
    assert its == 0 and rr == 0.0 and y.item() == 0.0 and fixed == 0 and used == "bf16"
    T32, eps = _system(40, 50, 2)
    T = torch.from_numpy(T32).to(DEV)
    e = torch.from_numpy(eps).to(DEV)
    y = torch.empty(40, dtype=torch.float64, device=DEV)
    its, rr, _, _ = nqs.nqs_sr_solve_mixed(T, e, 1e-2, y, "f16", tol=1e-30, max_iter=2)
    assert its == 2 and rr > 0.0
    for bad in ("e4m3", "f64"):
        with pytest.raises(nqs.NqsError):
            nqs.nqs_sr_solve_mixed(T, e, 1e-2, y, bad)
    with pytest.raises(nqs.NqsError):
        nqs.nqs_sr_solve_mixed(T, e, -1.0, y, "f32")
