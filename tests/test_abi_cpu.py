"""CPU tests of the C-ABI library: exports, host builder parity, validation.

The host builder (C++, ordered-form JW) is compared with the oracle's
Pauli-dict builder: masks and phases bit-exact, coefficients within 1e-13
relative (the builders sum contributions in different orders).
Device entry points are only called on argument errors that the library
rejects before touching the GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import qf_inputs as qi
from oracle import ansatz as an, hamiltonian as ham

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def qf():
    import paper_2108_04413_amd as qf
    return qf


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "qforte_mi355x.h")).read()
    return sorted(set(re.findall(r"\b(qf_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_header_symbol(qf):
    syms = header_symbols()
    assert "qf_build_paulis" in syms and "qf_energy_grad" in syms
    for s in syms:
        assert hasattr(qf.lib, s), s
    from paper_2108_04413_amd import _lib
    assert set(_lib.EXPORTS) == set(syms)


def test_term_layout(qf):
    assert qf.TERM_DTYPE.itemsize == 24


def _oracle_h(name):
    w, h, g = qi.workload(name)
    x, z, c, off = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    return w, h, g, x, z, c, off


def _compare(terms, off, x, z, c, off_o):
    assert len(terms) == len(x)
    assert np.array_equal(terms["x"], x)
    assert np.array_equal(terms["z"], z)
    assert np.array_equal(off, off_o)
    # the two builders sum up to ~10^3 contributions per string in different
    # orders: coefficients agree to 1e-13 relative to max(1, |c|)
    assert np.max(np.abs(terms["c"] - c) / np.maximum(1.0, np.abs(c))) <= 1e-13
    assert np.array_equal(np.sign(terms["c"]), np.sign(c))


@pytest.mark.parametrize("name", ["8q", "20q"])
def test_hamiltonian_builder_matches_oracle(qf, name):
    w, h, g, x, z, c, off = _oracle_h(name)
    terms, goff, _ = qf.build_paulis("hamiltonian", w["n_orb"], w["n_elec"], h, g)
    _compare(terms, goff, x, z, c, off)


@pytest.mark.slow
def test_hamiltonian_builder_matches_oracle_28q(qf):
    w, h, g, x, z, c, off = _oracle_h("28q")
    terms, goff, _ = qf.build_paulis("hamiltonian", w["n_orb"], w["n_elec"], h, g)
    _compare(terms, goff, x, z, c, off)


def test_builder_e_core_and_odd_shell(qf):
    h, g = qi.integrals(3, 3, 41)
    terms, goff, _ = qf.build_paulis("hamiltonian", 3, 3, h, g, e_core=1.25)
    x, z, c, off = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g, e_core=1.25))
    _compare(terms, goff, x, z, c, off)


@pytest.mark.parametrize("n_orb,n_e", [(4, 4), (5, 4), (7, 7), (10, 10)])
def test_uccsd_builder_matches_oracle(qf, n_orb, n_e):
    excs, x, z, c, off, kept = an.build(n_orb, n_e)
    terms, eoff, k2 = qf.build_paulis("uccsd", n_orb, n_e)
    _compare(terms, eoff, x, z, c, off)
    assert np.array_equal(k2, np.arange(len(excs)))


def test_uccd_top_builder_matches_oracle(qf):
    w = qi.WORKLOADS["28q"]
    terms_all, off_all, _ = qf.build_paulis("uccd", w["n_orb"], w["n_elec"])
    n_d = len(off_all) - 1
    assert n_d == len(an.excitations(28, 14, singles=False)) == 3283
    t_all = qi.amplitudes(n_d, w["seed"], w["t_scale"])
    excs, x, z, c, off, kept = an.build(w["n_orb"], w["n_elec"], "uccd_top", t_all, w["top_k"])
    terms, eoff, k2 = qf.build_paulis("uccd_top", w["n_orb"], w["n_elec"], t_rank=t_all, top_k=w["top_k"])
    _compare(terms, eoff, x, z, c, off)
    assert np.array_equal(k2, kept) and len(k2) == 512 and len(terms) == 4096


def test_top_k_ties_in_library(qf):
    t = np.array([0.1, -0.3, 0.3, 0.05, -0.1] + [0.0] * 13)  # 18 doubles for (4,4)
    terms, off, kept = qf.build_paulis("uccd_top", 4, 4, t_rank=t, top_k=4)
    assert kept.tolist() == an.top_k(t, 4).tolist() == [0, 1, 2, 4]


def test_puccd_builder_matches_oracle(qf):
    excs, x, z, c, off, _ = an.build(4, 4, "pduccd")
    terms, eoff, _ = qf.build_paulis("puccd", 4, 4)
    _compare(terms, eoff, x, z, c, off)


@pytest.mark.parametrize("n_orb", [2, 4, 7])
def test_gsd_pool_builder_matches_oracle(qf, n_orb):
    from oracle import adapt
    ops, x, z, c, off = adapt.pool_terms(2 * n_orb)
    terms, poff, kept = qf.build_paulis("gsd_pool", n_orb, 0)
    _compare(terms, poff, x, z, c, off)
    assert np.array_equal(kept, np.arange(len(ops)))


@pytest.mark.parametrize("kind,n_orb,n_e", [("uccsd", 4, 4), ("uccsd", 7, 7), ("uccsd", 5, 3), ("puccd", 4, 4)])
def test_excited_determinants_and_denominators_match_oracle(qf, kind, n_orb, n_e):
    from oracle import pqe
    det, sign = qf.excited_determinants(kind, n_orb, n_e)
    excs = an.build(n_orb, n_e, "pduccd" if kind == "puccd" else "uccsd")[0]
    want = [pqe.excitation_sign((1 << n_e) - 1, c, a) for c, a in excs]
    assert [(int(s), int(d)) for s, d in zip(sign, det)] == want
    h, g = qi.integrals(n_orb, n_e, 31)
    delta = qf.mp_denominators(kind, n_orb, n_e, h, g)
    assert np.max(np.abs(delta - pqe.mp_denominators(pqe.fock_diagonal(h, g, n_e), excs))) < 1e-13


def test_excited_determinants_of_truncated_doubles(qf):
    from oracle import pqe
    w = qi.WORKLOADS["28q"]
    n_d = len(an.excitations(28, 14, singles=False))
    t_all = qi.amplitudes(n_d, w["seed"], w["t_scale"])
    det, sign = qf.excited_determinants("uccd_top", 14, 14, t_rank=t_all, top_k=512)
    excs = an.build(14, 14, "uccd_top", t_all, 512)[0]
    assert [(int(s), int(d)) for s, d in zip(sign, det)] == [pqe.excitation_sign((1 << 14) - 1, c, a)
                                                               for c, a in excs]


def test_angles_and_chain_rule_match_oracle(qf):
    excs, x, z, c, off, _ = an.build(5, 4)
    terms, eoff, _ = qf.build_paulis("uccsd", 5, 4)
    t = qi.amplitudes(len(excs), 5, 0.3)
    th = qf.ansatz_angles(terms, eoff, t)
    assert np.array_equal(th, an.angles(c, off, t))
    dth = qi.random_angles(len(th), 17)
    assert np.allclose(qf.grad_t(terms, eoff, dth), an.grad_t(c, off, dth), atol=1e-15)


def test_build_size_protocol(qf):
    from paper_2108_04413_amd import _lib
    lib = qf.lib
    n_out, n_off = ctypes.c_int64(), ctypes.c_int64()
    assert lib.qf_build_paulis(1, 4, 4, None, None, 0.0, None, 0, None, 0, ctypes.byref(n_out), None, 0,
                               ctypes.byref(n_off), None) == 0
    assert (n_out.value, n_off.value) == (160, 27)
    small = np.zeros(10, dtype=qf.TERM_DTYPE)
    off = np.zeros(27, dtype=np.int64)
    st = lib.qf_build_paulis(1, 4, 4, None, None, 0.0, None, 0, small.ctypes.data, 10, ctypes.byref(n_out),
                             off.ctypes.data, 27, ctypes.byref(n_off), None)
    assert st == -5 and n_out.value == 160
    assert "need 160" in lib.qf_last_error().decode()
    assert _lib.STATUS[st] == "QF_E_SIZE"


@pytest.mark.parametrize("args,status", [
    ((9, 4, 4), -1),      # unknown kind
    ((0, 0, 0), -2),      # n_orb out of range
    ((1, 4, 9), -2),      # n_elec > spin orbitals
    ((0, 4, 4), -1),      # Hamiltonian without integrals
    ((3, 4, 4), -1),      # top-k without t_rank
])
def test_build_argument_errors(qf, args, status):
    n_out, n_off = ctypes.c_int64(), ctypes.c_int64()
    st = qf.lib.qf_build_paulis(*args, None, None, 0.0, None, 0, None, 0, ctypes.byref(n_out), None, 0,
                                ctypes.byref(n_off), None)
    assert st == status
    assert qf.lib.qf_last_error()


def test_nonhermitian_rejected_on_host(qf):
    # an asymmetric h gives imaginary strings: rejected before any device work
    h, g = qi.integrals(2, 2, 3)
    h[0, 1] += 0.5
    n_out, n_off = ctypes.c_int64(), ctypes.c_int64()
    st = qf.lib.qf_build_paulis(0, 2, 2, h.ctypes.data, g.ctypes.data, 0.0, None, 0, None, 0,
                                ctypes.byref(n_out), None, 0, ctypes.byref(n_off), None)
    assert st == -6


def test_device_calls_reject_bad_arguments_before_gpu(qf):
    lib = qf.lib
    dummy = ctypes.c_void_p(0x1000)
    bad = np.zeros(1, dtype=qf.TERM_DTYPE)
    bad["x"] = 1 << 9  # bit 9 with n = 8
    th = np.zeros(1)
    E = ctypes.c_double()
    assert lib.qf_prepare_state(None, 8, 3, None) == -1
    assert lib.qf_prepare_state(dummy, 0, 0, None) == -2
    assert lib.qf_prepare_state(dummy, 33, 0, None) == -2
    assert lib.qf_prepare_state(dummy, 31, 0, None) == -2  # above the tested 30 qubits
    assert lib.qf_prepare_state(dummy, 8, 1 << 8, None) == -2
    assert lib.qf_apply_pauli_exp(dummy, 8, bad.ctypes.data, th.ctypes.data, 1, 0, None) == -2
    assert lib.qf_apply_pauli_exp(dummy, 8, bad.ctypes.data, th.ctypes.data, -1, 0, None) == -1
    assert lib.qf_apply_pauli_exp(dummy, 8, None, th.ctypes.data, 1, 0, None) == -1
    off = np.array([0, 1], dtype=np.int64)
    assert lib.qf_energy(dummy, 8, bad.ctypes.data, off.ctypes.data, 1, ctypes.byref(E), None) == -2
    assert lib.qf_energy(None, 8, bad.ctypes.data, off.ctypes.data, 1, ctypes.byref(E), None) == -1
    mixed = np.zeros(2, dtype=qf.TERM_DTYPE)
    mixed["x"] = [1, 2]
    off2 = np.array([0, 2], dtype=np.int64)
    assert lib.qf_energy(dummy, 8, mixed.ctypes.data, off2.ctypes.data, 1, ctypes.byref(E), None) == -1
    assert "mixes flip masks" in lib.qf_last_error().decode()
    assert lib.qf_energy_grad(8, 3, None, None, 0, bad.ctypes.data, off.ctypes.data, 0, dummy,
                              ctypes.byref(E), None, None) == -1


def test_batch_create_rejects_bad_arguments_before_gpu(qf):
    lib = qf.lib
    h = ctypes.c_void_p()
    n = (ctypes.c_int * 1)(40)
    occ = (ctypes.c_uint64 * 1)(3)
    K = (ctypes.c_int64 * 1)(0)
    G = (ctypes.c_int64 * 1)(1)
    nulls = (ctypes.c_void_p * 1)(None)
    assert lib.qf_batch_create(1, n, occ, nulls, K, nulls, nulls, G, None, ctypes.byref(h)) == -2
    assert lib.qf_batch_create(0, n, occ, nulls, K, nulls, nulls, G, None, ctypes.byref(h)) == -1
    n[0] = 8
    occ[0] = 1 << 9
    assert lib.qf_batch_create(1, n, occ, nulls, K, nulls, nulls, G, None, ctypes.byref(h)) == -2
    occ[0] = 3
    assert lib.qf_batch_create(1, n, occ, nulls, K, nulls, nulls, G, None, ctypes.byref(h)) == -1
    assert lib.qf_batch_run(None, None, None, None, 0, None) == -1
