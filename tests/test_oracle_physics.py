"""Pins for the oracle's Hamiltonians, local energies and exact references (CPU only)."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import exact


# ---------------------------------------------------------------------------
# Exact diagonalisation pinned to closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,J,h", [(8, 1.0, 1.0), (12, 1.0, 0.5), (12, 1.0, 2.0), (10, 1.0, 3.04), (12, -1.0, 0.7),
                                   (10, 1.0, -1.3)])
def test_ed_tfim_chain_matches_free_fermions(n, J, h):
    """Periodic TFIM chain: ED equals the Jordan-Wigner closed form (spectrum independent of the signs of J, h)."""
    e0, _ = exact.ground_state("tfim", 1, n, J, h)
    assert abs(e0 - exact.free_fermion_tfim_e0(n, abs(J), abs(h))) < 1e-9


def test_free_fermion_n16_closed_form():
    # J = h = 1: every term is 2 sin(k/2), and the sum telescopes to 1/sin(pi/2N)
    assert abs(exact.free_fermion_tfim_e0(16, 1.0, 1.0) + 2.0 / np.sin(np.pi / 32)) < 1e-12


def test_ed_classical_and_field_limits():
    # h = 0 on an even periodic square lattice: Neel state satisfies all 2N bonds -> E0 = -2N J
    e0, _ = exact.ground_state("tfim", 2, 4, 1.0, 0.0)
    assert abs(e0 + 2 * 16) < 1e-9
    # J = 0: independent spins in a field -> E0 = -|h| N
    e0, _ = exact.ground_state("tfim", 2, 3, 0.0, 2.5)
    assert abs(e0 + 2.5 * 9) < 1e-9


def test_ed_heisenberg_four_site_ring():
    # J sum S_i.S_j on a 4-ring = (J/2)(S_tot^2 - S_13^2 - S_24^2) -> -2J; Pauli matrices are 4x that
    e0, _ = exact.ground_state("heisenberg", 1, 4, 1.0)
    assert abs(e0 + 8.0) < 1e-10


def test_ed_heisenberg_two_site_singlet_on_open_pair():
    # a single bond: singlet energy of sigma.sigma is -3
    e0, _ = exact.ground_state("heisenberg", 1, 2, 1.0, pbc=False)
    assert abs(e0 + 3.0) < 1e-12


@pytest.mark.parametrize("dim,L", [(1, 10), (2, 4)])
def test_marshall_sign_of_heisenberg_ground_state(dim, L):
    """Bipartite Heisenberg AFM: psi_0(x) * Marshall(x) has one sign (Perron-Frobenius after the rotation)."""
    e0, v = exact.ground_state("heisenberg", dim, L, 1.0)
    n = L if dim == 1 else L * L
    cfg = exact.all_configs(n)
    m = exact.marshall_sign(cfg, dim, L)
    w = v * m
    big = np.abs(v) > 1e-10 * np.abs(v).max()
    assert np.all(np.sign(w[big]) == np.sign(w[big][0]))


# ---------------------------------------------------------------------------
# Local energies: zero variance on exact eigenstates (pins E_loc exactly)
# ---------------------------------------------------------------------------

def _table_model(n, v, marshall=False, lattice=None, sign_override=None):
    sg = np.sign(v).astype(np.int8) if sign_override is None else sign_override
    la = np.log(np.maximum(np.abs(v), 1e-300))
    return oracle.OracleModel("table", n, table_logamp=la, table_sign=sg, marshall=marshall, lattice=lattice)


@pytest.mark.parametrize("kind,dim,L,J,h", [("tfim", 1, 10, 1.0, 1.0), ("tfim", 1, 12, 1.0, 0.5),
                                            ("tfim", 2, 3, 1.0, 3.04), ("tfim", 2, 4, 1.0, 3.04),
                                            ("heisenberg", 1, 10, 1.0, 0.0), ("heisenberg", 2, 4, 1.0, 0.0)])
def test_local_energy_is_constant_on_ground_state(orc, kind, dim, L, J, h):
    e0, v = exact.ground_state(kind, dim, L, J, h)
    n = L if dim == 1 else L * L
    model = _table_model(n, v)
    ham = workloads.Hamiltonian(kind, workloads.Lattice(dim, L), J, h)
    cfg = exact.all_configs(n)
    keep = np.abs(v) > 1e-8 * np.abs(v).max()
    el = oracle.local_energy(model, ham, cfg[keep])
    assert np.max(np.abs(el - e0)) < 1e-6 * max(1.0, abs(e0))


def test_local_energy_marshall_sign_path(orc):
    """Heisenberg ground state stored as |psi| * (sign/Marshall) with the Marshall flag on: same zero variance."""
    L = 4
    e0, v = exact.ground_state("heisenberg", 2, L, 1.0)
    cfg = exact.all_configs(16)
    m = exact.marshall_sign(cfg, 2, L)
    sg = (np.sign(v) * m).astype(np.int8)   # the sign left after removing Marshall's
    model = _table_model(16, v, marshall=True, lattice=workloads.Lattice(2, L), sign_override=sg)
    ham = workloads.Hamiltonian("heisenberg", workloads.Lattice(2, L), 1.0)
    keep = np.abs(v) > 1e-8 * np.abs(v).max()
    el = oracle.local_energy(model, ham, cfg[keep])
    assert np.max(np.abs(el - e0)) < 1e-6 * abs(e0)
    # after removing the Marshall sign the remaining sign is constant (Marshall's theorem)
    assert len(np.unique(sg[keep])) == 1


@pytest.mark.parametrize("kind,dim,L,h,arch", [("tfim", 1, 10, 1.0, "rbm"), ("tfim", 2, 3, 3.04, "rbm"),
                                               ("heisenberg", 1, 10, 0.0, "ffnn"), ("tfim", 1, 8, 0.7, "ffnn")])
def test_exact_energy_local_vs_matrix(orc, kind, dim, L, h, arch):
    """sum_x pi(x) eps(x) equals <psi|H|psi>/<psi|psi> from the assembled matrix (Eq. eq:loss)."""
    n = L if dim == 1 else L * L
    if arch == "rbm":
        p = workloads.rbm_params(n, 2 * n, 0.3, 11)
        model = oracle.OracleModel("rbm", n, (2 * n,), p)
    else:
        p = workloads.ffnn_params(n, (2 * n, n), 12, bias_std=0.1)
        model = oracle.OracleModel("ffnn", n, (2 * n, n), p, marshall=(kind == "heisenberg"),
                                   lattice=workloads.Lattice(dim, L))
    ham = workloads.Hamiltonian(kind, workloads.Lattice(dim, L), 1.0, h)
    pi, _, _ = exact.enumerate_pi(model)
    el = oracle.local_energy(model, ham, exact.all_configs(n))
    e_local = float(np.sum(pi * el))
    e_matrix = exact.exact_energy(model, kind, dim, L, 1.0, h)
    assert abs(e_local - e_matrix) < 1e-9 * max(1.0, abs(e_matrix))
    # variational principle
    e0, _ = exact.ground_state(kind, dim, L, 1.0, h)
    assert e_matrix >= e0 - 1e-9


def test_uniform_state_energy_and_local_energy(orc):
    """W = a = b = 0: every ratio is 1, so eps(x) = J sum s_i s_j + h N exactly and <H> = h N."""
    n = 16
    model = oracle.OracleModel("rbm", n, (16,), np.zeros(n + 16 + 256))
    ham = workloads.Hamiltonian("tfim", workloads.Lattice(1, n), 1.0, 1.0)
    cfg = exact.all_configs(n)
    el = oracle.local_energy(model, ham, cfg)
    zz = np.sum(cfg * np.roll(cfg, -1, axis=1), axis=1)
    assert np.array_equal(el, zz + 16.0)
    assert abs(el.mean() - 16.0) < 1e-12


def test_bonds_counts_and_uniqueness(orc):
    for dim, L in [(1, 16), (2, 3), (2, 10), (2, 20)]:
        b = oracle.bonds(dim, L, True)
        n = L if dim == 1 else L * L
        assert b.shape[0] == (n if dim == 1 else 2 * n)
        assert len({tuple(sorted(p)) for p in b}) == b.shape[0]
        assert sorted(map(tuple, np.sort(b, axis=1))) == exact._bond_list(dim, L, True)
        deg = np.bincount(b.ravel(), minlength=n)
        assert np.all(deg == (2 if dim == 1 else 4))
