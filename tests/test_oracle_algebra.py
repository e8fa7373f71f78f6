"""Pins of the oracle's Pauli algebra, JW map and gate-level examples.

Each test checks the oracle against something it does not compute itself:
dense Kronecker matrices, fermionic operators acting on occupation bit
strings, the paper's worked examples, or algebraic identities.
"""
import json
import math
import os

import numpy as np
import pytest

import qf_inputs as qi
from oracle import dense, pauli, statevec as sv

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def op_matrix(op, n):
    m = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for (x, z), c in op.items():
        m += c * dense.pauli_matrix(x, z, n)
    return m


def test_pauli_mul_matches_dense_products():
    rng = np.random.default_rng(7)
    n = 4
    for _ in range(200):
        x1, z1, x2, z2 = (int(v) for v in rng.integers(0, 1 << n, 4))
        x3, z3, k = pauli.pauli_mul(x1, z1, x2, z2)
        lhs = dense.pauli_matrix(x1, z1, n) @ dense.pauli_matrix(x2, z2, n)
        rhs = pauli.PHASE[k] * dense.pauli_matrix(x3, z3, n)
        assert np.array_equal(lhs, rhs)


def test_pauli_strings_hermitian_involutions():
    n = 3
    for x in range(1 << n):
        for z in range(1 << n):
            m = dense.pauli_matrix(x, z, n)
            assert np.allclose(m, m.conj().T)
            assert np.allclose(m @ m, np.eye(1 << n))


def test_apply_pauli_matches_dense():
    n = 5
    psi = qi.random_state(n, 11)
    for x, z in [(0, 0), (1, 0), (0b10110, 0b01101), (31, 31), (0b1000, 0b0111)]:
        assert np.allclose(sv.apply_pauli(psi, n, x, z), dense.pauli_matrix(x, z, n) @ psi, atol=1e-15)


def test_jw_ladder_equals_bitstring_second_quantization():
    # Eqs. (13)-(14) vs. a_p acting on occupation strings with the
    # (-1)^(occupied below p) sign.
    n = 5
    for p in range(n):
        for dag in (False, True):
            assert np.allclose(op_matrix(pauli.ladder(p, dag), n), dense.ladder_matrix(p, dag, n))


def test_jw_canonical_anticommutation():
    n = 5
    a = [op_matrix(pauli.ladder(p, False), n) for p in range(n)]
    ad = [op_matrix(pauli.ladder(p, True), n) for p in range(n)]
    eye = np.eye(1 << n)
    for p in range(n):
        for q in range(n):
            assert np.allclose(a[p] @ ad[q] + ad[q] @ a[p], eye if p == q else 0 * eye)
            assert np.allclose(a[p] @ a[q] + a[q] @ a[p], 0 * eye)


def test_creation_sets_bit_with_jw_sign():
    n = 4
    m = op_matrix(pauli.ladder(2, True), n)
    # |b=0b0011> (qubits 0,1 occupied) -> +|0b0111> (two occupied below: +1)
    assert m[0b0111, 0b0011] == pytest.approx(1.0)
    # |0b0001> -> -|0b0101>? one occupied below p=2 -> sign -1
    assert m[0b0101, 0b0001] == pytest.approx(-1.0)


def test_sqoperator_example_matches_fermion_matrix():
    gold = GOLD["sqop_example"]
    n = 5
    op = {}
    terms = []
    for re, im, cre, ann in gold["terms"]:
        c = complex(re, im)
        pauli.op_add(op, pauli.sq_term(c, cre, ann))
        terms.append((c, tuple(cre), tuple(ann)))
    assert np.allclose(op_matrix(pauli.clean(op), n), dense.fermion_matrix(terms, n))


def test_bell_state_and_expectation():
    gold = GOLD["bell_state"]
    n = 2
    psi = np.zeros(4, dtype=np.complex128)
    psi[0] = 1
    psi = dense.gate("CNOT", 1, 0, n=n) @ (dense.gate("H", 0, n=n) @ psi)
    for idx, amp in gold["amplitudes"].items():
        assert psi[int(idx)] == pytest.approx(amp, abs=1e-15)
    assert abs(psi[1]) < 1e-15 and abs(psi[2]) < 1e-15
    # <X0 + X1> on the Bell state is 0
    e = sv.energy(psi, n, np.array([1, 2], np.uint64), np.array([0, 0], np.uint64), np.array([1.0, 1.0]))
    assert abs(e) < 1e-15


def test_exp_pauli_equals_paper_circuit():
    g = GOLD["exp_pt_example"]
    n = 3
    th, phi = g["theta"], g["rz_angle"]
    assert phi == 2 * th
    # Fig. exp_pt, left to right: H2, CNOT(0->1), CNOT(1->2), Rz(2 theta) on
    # q2, CNOT(1->2), CNOT(0->1), H2.  gate('CNOT', target, control).
    spec = [("H", 2), ("CNOT", 1, 0), ("CNOT", 2, 1), ("Rz", 2),
            ("CNOT", 2, 1), ("CNOT", 1, 0), ("H", 2)]
    gates = [dense.gate("Rz", 2, angle=phi, n=n) if s[0] == "Rz"
             else dense.gate(s[0], s[1], s[2] if len(s) > 2 else None, n=n) for s in spec]
    u_circ = dense.circuit(gates, n)
    assert sum(1 for s in spec if s[0] == "CNOT") == g["n_cnot"]
    P = dense.pauli_matrix(g["x"], g["z"], n)
    assert pauli.to_string(g["x"], g["z"], n) == "X2 Z1 Z0"
    u_def = math.cos(th) * np.eye(8) - 1j * math.sin(th) * P
    assert np.allclose(u_circ, u_def, atol=1e-14)
    for b in range(8):
        e = np.zeros(8, dtype=np.complex128)
        e[b] = 1
        assert np.allclose(sv.apply_exp(e, n, g["x"], g["z"], th), u_def @ e, atol=1e-15)


def test_exp_closed_form_random_strings():
    n = 6
    psi = qi.random_state(n, 3)
    xs, zs, cs = qi.random_paulis(n, 30, 5)
    th = qi.random_angles(30, 6)
    for x, z, t in zip(xs, zs, th):
        P = dense.pauli_matrix(int(x), int(z), n)
        want = (math.cos(t) * np.eye(1 << n) - 1j * math.sin(t) * P) @ psi
        assert np.allclose(sv.apply_exp(psi, n, int(x), int(z), float(t)), want, atol=1e-14)


def test_product_order_and_inverse():
    n = 5
    psi = qi.random_state(n, 8)
    xs, zs, _ = qi.random_paulis(n, 12, 9)
    th = qi.random_angles(12, 10)
    u = np.eye(1 << n, dtype=np.complex128)
    for x, z, t in zip(xs, zs, th):  # k = 0 acts first
        u = (math.cos(t) * np.eye(1 << n) - 1j * math.sin(t) * dense.pauli_matrix(int(x), int(z), n)) @ u
    out = sv.apply_product(psi, n, xs, zs, th)
    assert np.allclose(out, u @ psi, atol=1e-14)
    back = sv.apply_product(out, n, xs, zs, th, inverse=True)
    assert np.allclose(back, psi, atol=1e-14)


def test_theta_zero_is_identity_bit_exact():
    n = 6
    psi = qi.random_state(n, 12)
    xs, zs, _ = qi.random_paulis(n, 20, 13)
    out = sv.apply_product(psi.copy(), n, xs, zs, np.zeros(20))
    assert np.array_equal(out, psi)
