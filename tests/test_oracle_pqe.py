"""Pins of the oracle's PQE residuals and update (Sec. 3.3).

References not computed by the code under test: the paper's three-energy
form of the residual, dense matrices built from second quantization on bit
strings (U as a product of matrix exponentials of the kappa matrices, no
Pauli algebra), Slater-Condon elements at t = 0 and Koopmans-type
differences of determinant energies for the Fock diagonal.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import qf_inputs as qi
from oracle import ansatz as an, dense, hamiltonian as ham, pqe, statevec as sv


@pytest.fixture(scope="module")
def sys8():
    w, h, g = qi.workload("8q")
    n, ne = 8, w["n_elec"]
    occ = an.reference_mask(ne)
    hx, hz, hc, _ = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    excs, ax, az, ac, aoff, _ = an.build(w["n_orb"], ne)
    hm = dense.fermion_matrix(list(ham.fermion_hamiltonian_terms(h, g)), n)
    return dict(n=n, ne=ne, occ=occ, h=h, g=g, hx=hx, hz=hz, hc=hc, excs=excs, ax=ax, az=az, ac=ac, aoff=aoff,
                hm=hm)


def _theta(d, t):
    return an.angles(d["ac"], d["aoff"], t)


def test_excitation_sign_matches_bitstring_second_quantization(sys8):
    for cre, ann in sys8["excs"]:
        assert pqe.excitation_sign(sys8["occ"], cre, ann) == dense.apply_string(sys8["occ"], cre, ann)


def test_residuals_direct_equal_three_energy_form(sys8):
    d = sys8
    t = qi.amplitudes(len(d["excs"]), 1008, 0.3)
    args = (d["n"], d["occ"], d["ax"], d["az"], _theta(d, t), d["hx"], d["hz"], d["hc"], d["excs"])
    e, r = pqe.residuals(*args)
    r3 = pqe.residuals_three_energies(*args)
    assert np.max(np.abs(r - r3)) < 1e-12
    assert np.max(np.abs(r)) > 1e-2


def test_residuals_equal_dense_unitary_matrix_element(sys8):
    d = sys8
    n, occ = d["n"], d["occ"]
    t = qi.amplitudes(len(d["excs"]), 77, 0.4)
    e, r = pqe.residuals(n, occ, d["ax"], d["az"], _theta(d, t), d["hx"], d["hz"], d["hc"], d["excs"])
    U = np.eye(1 << n, dtype=np.complex128)
    for (cre, ann), tm in zip(d["excs"], t):  # first factor acts first
        K = dense.fermion_matrix([(1.0, cre, ann), (-1.0, tuple(reversed(ann)), tuple(reversed(cre)))], n)
        U = expm(tm * K) @ U
    M = U.conj().T @ d["hm"] @ U
    assert e == pytest.approx(M[occ, occ].real, abs=1e-12)
    for mu, (cre, ann) in enumerate(d["excs"]):
        s, det = dense.apply_string(occ, cre, ann)
        assert r[mu] == pytest.approx(s * M[det, occ].real, abs=1e-12)
        assert abs(M[det, occ].imag) < 1e-12


def test_residuals_at_zero_are_hamiltonian_elements(sys8):
    d = sys8
    n, occ = d["n"], d["occ"]
    K = len(d["ax"])
    e, r = pqe.residuals(n, occ, d["ax"], d["az"], np.zeros(K), d["hx"], d["hz"], d["hc"], d["excs"])
    for mu, (cre, ann) in enumerate(d["excs"]):
        s, det = dense.apply_string(occ, cre, ann)
        assert r[mu] == pytest.approx(s * d["hm"][det, occ].real, abs=1e-12)


def test_fock_diagonal_is_a_koopmans_difference(sys8):
    # eps_i = E(Phi_0) - E(Phi_0 without i); eps_a = E(Phi_0 with a) - E(Phi_0),
    # determinant energies from the dense second-quantized H
    d = sys8
    eps = pqe.fock_diagonal(d["h"], d["g"], d["ne"])
    hm, occ = d["hm"], d["occ"]
    for p in range(d["n"]):
        other = occ ^ (1 << p)
        want = hm[occ, occ] - hm[other, other] if (occ >> p) & 1 else hm[other, other] - hm[occ, occ]
        assert eps[p] == pytest.approx(want.real, abs=1e-12)
    delta = pqe.mp_denominators(eps, d["excs"])
    assert np.all(delta < 0)  # HF-lowering diagonal shift: occupied below virtual here


def weak_system():
    """The 8-qubit recipe with the off-diagonal one-body integrals scaled by
    0.2: a reference close to a Hartree-Fock determinant, for which the
    diagonal quasi-Newton update of Sec. 3.3 converges.  (With the recipe's
    N(0, 1) off-diagonal h the singles residuals are O(1) and the update
    oscillates: the reference is far from self-consistent.)"""
    h, g = qi.integrals(4, 4, 1008)
    h = np.where(np.eye(4, dtype=bool), h, 0.2 * h)
    return h, g


def test_fixed_point_iteration_drives_residuals_to_zero():
    h, g = weak_system()
    n, ne, occ = 8, 4, 15
    hx, hz, hc, _ = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    excs, ax, az, ac, aoff, _ = an.build(4, 4)
    eps = pqe.fock_diagonal(h, g, ne)
    delta = pqe.mp_denominators(eps, excs)
    t = np.zeros(len(excs))
    for it in range(60):
        e, r = pqe.residuals(n, occ, ax, az, an.angles(ac, aoff, t), hx, hz, hc, excs)
        if np.max(np.abs(r)) < 1e-10:
            break
        t = pqe.update(t, r, delta)
    assert np.max(np.abs(r)) < 1e-10, (it, np.max(np.abs(r)))
    # a dUCCSD state: between the exact ground state and the reference energy
    hm = dense.fermion_matrix(list(ham.fermion_hamiltonian_terms(h, g)), n)
    e0 = dense.ground_energy_in_sector(hm, n, ne, 0)
    assert e0 - 1e-9 <= e < hm[occ, occ].real
