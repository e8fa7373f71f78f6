"""Pins of the oracle's Trotterized evolution and QK matrices (Sec. 3.7).

References not computed by the code under test: scipy's matrix exponential
of dense Kronecker matrices (exact evolution, and the Trotter product term
by term), the first-order Trotter error bound, closed-form Hartree-Fock
energies and exact diagonalization."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import qf_inputs as qi
from oracle import ansatz as an, core, dense, hamiltonian as ham, krylov, statevec as sv


def test_commuting_strings_evolve_exactly():
    n = 6
    rng = np.random.default_rng(3)
    zs = np.array([int(v) for v in rng.integers(0, 1 << n, 12)], dtype=np.uint64)
    xs = np.zeros(12, dtype=np.uint64)
    cs = rng.standard_normal(12)
    hm = dense.pauli_sum_matrix(xs, zs, cs, n)
    psi0 = qi.random_state(n, 4)
    for t, r in ((0.7, 1), (-1.3, 3)):
        assert np.allclose(krylov.trotter(psi0, n, xs, zs, cs, t, r), expm(-1j * t * hm) @ psi0, atol=1e-12)


def test_trotter_product_term_by_term_and_core():
    n = 5
    xs, zs, cs = qi.random_paulis(n, 9, 5, max_weight=3)
    psi0 = qi.random_state(n, 6)
    t, r = 0.9, 2
    U = np.eye(1 << n, dtype=np.complex128)
    for _ in range(r):
        for x, z, c in zip(xs, zs, cs):  # the first string acts first
            U = expm(-1j * t * c / r * dense.pauli_matrix(int(x), int(z), n)) @ U
    want = U @ psi0
    assert np.allclose(krylov.trotter(psi0, n, xs, zs, cs, t, r), want, atol=1e-13)
    assert np.allclose(krylov.trotter_core(psi0.copy(), n, xs, zs, cs, t, r), want, atol=1e-13)


def test_trotter_error_within_first_order_bound_and_shrinks_with_r():
    w, h, g = qi.workload("8q")
    n, occ = 8, 15
    hx, hz, hc, _ = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    hm = dense.pauli_sum_matrix(hx, hz, hc, n)
    phi = sv.prepare(n, occ)
    t = 0.05
    exact = expm(-1j * t * hm) @ phi
    # ||prod - exp|| <= t^2 / (2 r) sum_{l<m} ||[h_l P_l, h_m P_m]||, the
    # commutator of two strings is 0 or 2 h_l h_m P
    bound = 0.0
    for a in range(len(hx)):
        for b in range(a + 1, len(hx)):
            anti = bin(int(hx[a]) & int(hz[b])).count("1") + bin(int(hz[a]) & int(hx[b])).count("1")
            if anti % 2:
                bound += 2.0 * abs(hc[a] * hc[b])
    errs = []
    for r in (1, 2, 4):
        err = np.linalg.norm(krylov.trotter(phi, n, hx, hz, hc, t, r) - exact)
        assert err <= t * t / (2 * r) * bound
        errs.append(err)
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.15) and errs[1] / errs[2] == pytest.approx(2.0, rel=0.15)


def test_qk_matrices_structure_and_bounds():
    w, h, g = qi.workload("8q")
    n, occ = 8, 15
    hx, hz, hc, _ = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    S, Hm = krylov.qk_matrices(n, occ, hx, hz, hc, 0.5, 3, 1)
    S2, H2 = krylov.qk_matrices(n, occ, hx, hz, hc, 0.5, 3, 1, use_core=True)
    assert np.allclose(S, S2, atol=1e-12) and np.allclose(Hm, H2, atol=1e-12)
    assert np.allclose(S, S.conj().T, atol=1e-12) and np.allclose(Hm, Hm.conj().T, atol=1e-12)
    assert np.allclose(np.diag(S), 1.0, atol=1e-12)
    e_hf = 2 * sum(h[i, i] for i in range(2)) + sum(2 * g[i, i, j, j] - g[i, j, j, i] for i in range(2)
                                                    for j in range(2))
    assert Hm[0, 0].real == pytest.approx(e_hf, abs=1e-12)
    hd = dense.fermion_matrix(list(ham.fermion_hamiltonian_terms(h, g)), n)
    e0 = dense.ground_energy_in_sector(hd, n, 4, 0)
    e_qk = krylov.qk_energy(S, Hm)
    assert e0 - 1e-9 <= e_qk <= e_hf + 1e-12
    assert e_qk < e_hf - 1e-3  # the Krylov space improves on the reference
