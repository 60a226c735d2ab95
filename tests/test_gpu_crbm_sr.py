"""GPU parity of the complex-parameter RBM's log-derivatives and SR step
against the numpy oracle (App. G with complex a, b, W; Eqs. eq:forces,
eq:smat, eq:sr_step): O element by element, the real embedding of the
sample-space T, the direction the sample-space solve and the update produce
against the oracle's parameter-space solve (S + shift) delta = F, and SR
training to the exact ground energy.  Every call goes through the C
interface."""
import numpy as np
import pytest
import torch

import workloads
from oracle import crbm
from oracle import exact

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


def _grad(nqs, model, x, P):
    n = x.shape[0]
    O = torch.empty(n, P, dtype=torch.float32, device=DEV)
    lp = torch.empty(n, dtype=torch.float32, device=DEV)
    nqs.nqs_logpsi_grad(model, x, lp, O)
    torch.cuda.synchronize()
    return lp.cpu().numpy(), O.cpu().numpy()


@pytest.mark.parametrize("N,M,n", [(100, 200, 96), (16, 16, 300), (33, 7, 50)])
def test_log_derivatives_match_the_oracle(nqs, N, M, n):
    """O of the FP32 copy against the oracle's O of the FP32-rounded parameters, element by element
    (10x10 lattice at alpha = 2, a 16-site chain, two spin words with few hidden units).  tanh has poles at
    theta = i pi (k + 1/2), so a unit's error is bounded by the FP32 error of its theta, at most
    N u (|b_j| + sum_i |W_ji|) for N-term recursive summation (u = 2^-24), times |d tanh / d theta| =
    |1 - tanh^2|, plus a few units of rounding in tanh itself (relative to |tanh|^2 near a pole, where the
    denominator cosh 2x + cos 2y cancels); the test holds every element to that bound."""
    p = workloads.crbm_params(N, M, 0.2, 0.4, N + M)
    model = nqs.Model("crbm", N, (M,), p)
    Pc = N + M + M * N
    x = workloads.random_spins(n, N, 7)
    lp, O = _grad(nqs, model, torch.from_numpy(x).to(DEV), 2 * Pc)
    net = crbm.ComplexRBM(N, M, p, "f32")
    ref = net.logpsi_grad(x)
    got = O[:, :Pc] + 1j * O[:, Pc:]
    u = 2.0 ** -24
    t = ref[:, N:N + M]
    e_theta = N * u * (np.abs(net.b) + np.abs(net.W).sum(axis=1))              # [M]
    e_t = np.abs(1.0 - t * t) * e_theta[None, :] + 16 * u * (1.0 + np.abs(t) ** 2)   # [n][M]
    bound = np.concatenate([np.full((n, N), 1e-7), e_t, np.repeat(e_t, N, axis=1)], axis=1)
    err = np.abs(got - ref)
    _say(f"  N={N} M={M}: max |dO| {err.max():.2e}, max |dO| / bound {np.max(err / bound):.2f}, "
         f"max |tanh theta| {np.abs(t).max():.1f}")
    assert np.all(err <= bound)
    lref = net.logpsi(x).real
    assert np.max(np.abs(lp - lref) / np.maximum(1.0, np.abs(lref))) <= 1e-5
    model.close()


def test_complex_t_matches_the_embedding(nqs):
    """nqs_gram mode 3 against [[Re T, -Im T], [Im T, Re T]], T = Obar Obar^H / n in FP64 from the same O."""
    N, M, n = 16, 24, 384
    p = workloads.crbm_params(N, M, 0.3, 0.5, 3)
    model = nqs.Model("crbm", N, (M,), p)
    Pc = N + M + M * N
    x = workloads.random_spins(n, N, 8)
    _, O = _grad(nqs, model, torch.from_numpy(x).to(DEV), 2 * Pc)
    T2 = torch.empty(2 * n, 2 * n, dtype=torch.float32, device=DEV)
    nqs.nqs_gram(torch.from_numpy(O).to(DEV), 3, T2)
    torch.cuda.synchronize()
    Oc = O[:, :Pc].astype(np.float64) + 1j * O[:, Pc:].astype(np.float64)
    ref = crbm.tmatrix_embedded(Oc)
    got = T2.cpu().numpy()
    scale = np.max(np.abs(np.diag(ref)))
    _say(f"  max |dT2| {np.max(np.abs(got - ref)):.2e} (diagonal scale {scale:.2e})")
    assert np.max(np.abs(got - ref)) <= 2e-5 * scale
    assert np.allclose(got, got.T, atol=2e-5 * scale)
    model.close()


def test_sr_step_is_the_parameter_space_direction(nqs):
    """Sampled configurations of a complex RBM on the 16-site TFIM chain: the device's sample-space step
    (nqs_gram mode 3, nqs_sr_solve_complex, nqs_sr_update with lr = 1) moves the parameters by -delta, delta the
    oracle's solution of (S + shift) delta = F with S and F from their definitions, on the same O and energies."""
    N, M, C, S = 16, 16, 128, 4
    n, shift = C * S, 1e-2
    p = workloads.crbm_params(N, M, 0.2, 0.3, 9)
    model = nqs.Model("crbm", N, (M,), p)
    ham = nqs.Hamiltonian.from_workload(workloads.Hamiltonian("tfim", workloads.Lattice(1, N), 1.0, -1.0))
    state = torch.empty(C, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    nqs.nqs_sample(model, nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=10, seed=4, dtype="f32"), state, samples)
    flat = samples.reshape(n, N)
    er = torch.empty(n, dtype=torch.float64, device=DEV)
    ei = torch.empty(n, dtype=torch.float64, device=DEV)
    nqs.nqs_local_energy_complex(model, ham, flat, er, ei)
    Pc = N + M + M * N
    O = torch.empty(n, 2 * Pc, dtype=torch.float32, device=DEV)
    nqs.nqs_logpsi_grad(model, flat, None, O)
    T2 = torch.empty(2 * n, 2 * n, dtype=torch.float32, device=DEV)
    nqs.nqs_gram(O, 3, T2)
    y2 = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    it, rr = nqs.nqs_sr_solve_complex(T2, er, ei, shift, y2, tol=1e-12, max_iter=4000)
    master = torch.from_numpy(p.copy()).to(DEV)
    nqs.nqs_sr_update(model, flat, y2, 1.0, master)
    torch.cuda.synchronize()
    step = p - master.cpu().numpy()
    got = step[:Pc] + 1j * step[Pc:]
    On = O.cpu().numpy().astype(np.float64)
    ref = crbm.sr_direction(On[:, :Pc] + 1j * On[:, Pc:], er.cpu().numpy() + 1j * ei.cpu().numpy(), shift)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say(f"  CG {it} iterations, residual {rr:.1e}; |delta_dev - delta_oracle| / |delta_oracle| = {rel:.2e}")
    assert rr <= 1e-10
    assert rel <= 1e-3
    model.close()


def test_complex_vmc_training_reaches_ground_state(nqs):
    """SR steps of a complex RBM (alpha = 2, imaginary parts drawn like the real ones) on the 12-site TFIM chain
    at the critical field (J = 1, h = -1, periodic): the energy reaches the exact ground energy to 1e-3."""
    N, M = 12, 24
    e0, _ = exact.ground_state("tfim", 1, N, 1.0, -1.0)
    p = workloads.crbm_params(N, M, 0.01, 0.01, 3)
    model = nqs.Model("crbm", N, (M,), p)
    ham = nqs.Hamiltonian.from_workload(workloads.Hamiltonian("tfim", workloads.Lattice(1, N), 1.0, -1.0))
    master = torch.from_numpy(p.copy()).to(DEV)
    C, S = 512, 4
    n = C * S
    Pc = N + M + M * N
    state = torch.empty(C, N, dtype=torch.int8, device=DEV)
    samples = torch.empty(S, C, N, dtype=torch.int8, device=DEV)
    er = torch.empty(n, dtype=torch.float64, device=DEV)
    ei = torch.empty(n, dtype=torch.float64, device=DEV)
    stats = torch.empty(4, dtype=torch.float64, device=DEV)
    O = torch.empty(n, 2 * Pc, dtype=torch.float32, device=DEV)
    T2 = torch.empty(2 * n, 2 * n, dtype=torch.float32, device=DEV)
    y2 = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    energies, offset = [], 0
    for it in range(120):
        model.set_params_device(master)
        burn = 20 if it == 0 else 2
        cfg = nqs.SampleConfig(n_chains=C, n_sweeps=S, n_burnin=burn, seed=11, dtype="f32", step_offset=offset,
                               init_chains=it == 0)
        nqs.nqs_sample(model, cfg, state, samples)
        offset += (burn + S) * N
        flat = samples.reshape(n, N)
        nqs.nqs_local_energy_complex(model, ham, flat, er, ei)
        nqs.nqs_energy_stats(er, C, stats)
        nqs.nqs_logpsi_grad(model, flat, None, O)
        nqs.nqs_gram(O, 3, T2)
        nqs.nqs_sr_solve_complex(T2, er, ei, 1e-2, y2, tol=1e-6, max_iter=300)
        nqs.nqs_sr_update(model, flat, y2, 0.05, master)
        energies.append(float(stats[0].item()))
        if it % 20 == 0:
            _say(f"  iteration {it}: E = {energies[-1]:.5f} (exact {e0:.5f})")
    e_end = float(np.mean(energies[-10:]))
    _say(f"  mean of the last 10 energies {e_end:.5f}, exact {e0:.5f}, rel {abs(e_end - e0) / abs(e0):.2e}")
    assert abs(e_end - e0) <= 1e-3 * abs(e0)
    model.close()
