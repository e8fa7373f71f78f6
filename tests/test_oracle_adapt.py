"""Pins of the oracle's ADAPT-VQE pool and pool gradients (Sec. 3.2).

References not computed by the code under test: counting formulas, second
quantization on occupation bit strings (dense fermion matrices, no Pauli
algebra), the dense commutator <Psi|[H, kappa]|Psi>, and the exact shift
rule of the strings of kappa appended to the ansatz.
"""
import math
from math import comb

import numpy as np
import pytest

import qf_inputs as qi
from oracle import adapt, ansatz as an, core, dense, hamiltonian as ham, pauli, statevec as sv


def pool_size(n_orb):
    """singles 2 C(n,2); doubles: pairs of distinct pairs within one S_z class
    (alpha-alpha, beta-beta: C(n,2) pairs each; alpha-beta: n^2 pairs)."""
    return 2 * comb(n_orb, 2), 2 * comb(comb(n_orb, 2), 2) + comb(n_orb * n_orb, 2)


@pytest.mark.parametrize("n_orb", [2, 3, 4, 10])
def test_pool_counts_and_string_structure(n_orb):
    N = 2 * n_orb
    ops = adapt.gsd_pool(N)
    ns, nd = pool_size(n_orb)
    assert sum(1 for c, a in ops if len(c) == 1) == ns
    assert sum(1 for c, a in ops if len(c) == 2) == nd
    assert len(set(ops)) == len(ops)
    if n_orb > 4:
        return
    for cre, ann in ops:
        st = an.kappa_strings(cre, ann)
        idx = list(cre) + list(ann)
        shared = len(idx) - len(set(idx))
        assert len(st) == (2 if len(cre) == 1 else 8 if shared == 0 else 4)
        x = 0
        for p in idx:
            x ^= 1 << p
        assert {k[0] for k in st} == {x}
        for a in st:  # commuting strings with an odd number of Y
            assert bin(a[0] & a[1]).count("1") % 2 == 1
            for b in st:
                assert pauli.pauli_mul(*a, *b) == pauli.pauli_mul(*b, *a)


def test_pool_kappa_equals_fermion_matrices():
    n = 6
    ops, x, z, c, off = adapt.pool_terms(n)
    for nu, (cre, ann) in enumerate(ops):
        m = sum(1j * c[k] * dense.pauli_matrix(int(x[k]), int(z[k]), n) for k in range(off[nu], off[nu + 1]))
        want = dense.fermion_matrix([(1.0, cre, ann), (-1.0, tuple(reversed(ann)), tuple(reversed(cre)))], n)
        assert np.allclose(m, want, atol=1e-14), (cre, ann)


@pytest.fixture(scope="module")
def adapt8():
    w, h, g = qi.workload("8q")
    n, occ = 8, an.reference_mask(w["n_elec"])
    hx, hz, hc, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    excs, ax, az, ac, aoff, _ = an.build(w["n_orb"], w["n_elec"])
    t = qi.amplitudes(len(excs), w["seed"], w["t_scale"])
    psi = sv.apply_product(sv.prepare(n, occ), n, ax, az, an.angles(ac, aoff, t))
    hm = dense.fermion_matrix(list(ham.fermion_hamiltonian_terms(h, g)), n)
    ops, px, pz, pc, poff = adapt.pool_terms(n)
    return dict(n=n, occ=occ, psi=psi, hm=hm, hx=hx, hz=hz, hc=hc, ops=ops, px=px, pz=pz, pc=pc, poff=poff)


def test_pool_gradient_equals_dense_commutator(adapt8):
    d = adapt8
    n, psi, hm = d["n"], d["psi"], d["hm"]
    g = adapt.pool_gradients(psi, n, d["px"], d["pz"], d["pc"], d["poff"], d["hx"], d["hz"], d["hc"])
    lam = core.sigma(psi.copy(), n, d["hx"], d["hz"], d["hc"])
    gc = core.pool_grad(psi.copy(), lam, n, d["px"], d["pz"], d["pc"], d["poff"])
    assert np.max(np.abs(g - gc)) < 1e-12
    for nu, (cre, ann) in enumerate(d["ops"]):
        K = dense.fermion_matrix([(1.0, cre, ann), (-1.0, tuple(reversed(ann)), tuple(reversed(cre)))], n)
        want = np.vdot(psi, (hm @ K - K @ hm) @ psi)
        assert abs(want.imag) < 1e-12
        assert g[nu] == pytest.approx(want.real, abs=1e-12), (cre, ann)
    assert np.max(np.abs(g)) > 1e-2  # not a vacuous comparison


def test_pool_gradient_equals_shift_rule_of_appended_strings(adapt8):
    # appending exp(t kappa_nu) = prod_k exp(-i theta_k P_k), theta_k = -c_k t:
    # dE/dt at 0 = -sum_k c_k (E(theta_k = pi/4) - E(theta_k = -pi/4)), each
    # E computed with dense matrices
    d = adapt8
    n, psi = d["n"], d["psi"]
    hp = dense.pauli_sum_matrix(d["hx"], d["hz"], d["hc"], n)
    g = adapt.pool_gradients(psi, n, d["px"], d["pz"], d["pc"], d["poff"], d["hx"], d["hz"], d["hc"])
    rng = np.random.default_rng(5)
    for nu in sorted(set(rng.integers(0, len(d["ops"]), 12).tolist()) | {0, len(d["ops"]) - 1}):
        tot = 0.0
        for k in range(d["poff"][nu], d["poff"][nu + 1]):
            P = dense.pauli_matrix(int(d["px"][k]), int(d["pz"][k]), n)
            e = []
            for th in (math.pi / 4, -math.pi / 4):
                v = math.cos(th) * psi - 1j * math.sin(th) * (P @ psi)
                e.append(np.vdot(v, hp @ v).real)
            tot += -d["pc"][k] * (e[0] - e[1])
        assert g[nu] == pytest.approx(tot, abs=1e-12)


def test_pool_gradient_at_reference_is_matrix_element(adapt8):
    # at Psi = Phi_0 only members connecting Phi_0 to another determinant
    # contribute: g = 2 s <Phi_0|H|Phi_mu> for tau Phi_0 = s Phi_mu
    d = adapt8
    n, occ = d["n"], d["occ"]
    psi0 = sv.prepare(n, occ)
    g = adapt.pool_gradients(psi0, n, d["px"], d["pz"], d["pc"], d["poff"], d["hx"], d["hz"], d["hc"])
    for nu, (cre, ann) in enumerate(d["ops"]):
        s, det = dense.apply_string(occ, cre, ann)
        s2, det2 = dense.apply_string(occ, tuple(reversed(ann)), tuple(reversed(cre)))
        want = 0.0
        if s:
            want += 2 * s * d["hm"][occ, det].real
        if s2:  # tau^dagger Phi_0 = s2 Phi_det2: kappa Phi_0 gains -s2 Phi_det2
            want -= 2 * s2 * d["hm"][occ, det2].real
        assert g[nu] == pytest.approx(want, abs=1e-12)
