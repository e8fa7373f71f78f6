"""Pins of the oracle's Hamiltonian, ansatz, energy and gradient.

References used here, none computed by the code under test:
* second quantization on occupation bit strings (oracle.dense.fermion_matrix),
* closed-form Hartree-Fock energies, exact diagonalization lower bounds,
* the paper's printed integers (Table 1) and Eq. (24),
* closed-form string/group counts of a JW Hamiltonian,
* parameter-shift and finite-difference derivatives.
"""
import json
import math
import os
from math import comb

import numpy as np
import pytest

import qf_inputs as qi
from oracle import ansatz as an
from oracle import core, dense, hamiltonian as ham, pauli, statevec as sv

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def expected_counts(n):
    """(strings, groups) of the JW Hamiltonian of n spatial orbitals with
    generic real 8-fold-symmetric integrals: diagonal group 1 + N + C(N,2);
    same-spin pairs 2(N-1) strings; same-spin quadruples 6; opposite-spin
    pairs of pairs 4."""
    N = 2 * n
    strings = 1 + N + N * (N - 1) // 2 + 2 * comb(n, 2) * 2 * (N - 1) + 2 * comb(n, 4) * 6 \
        + comb(n, 2) ** 2 * 4
    groups = 1 + 2 * comb(n, 2) + 2 * comb(n, 4) + comb(n, 2) ** 2
    return strings, groups


def hf_closed_shell(h, g, ndocc):
    e = 2.0 * sum(h[i, i] for i in range(ndocc))
    for i in range(ndocc):
        for j in range(ndocc):
            e += 2.0 * g[i, i, j, j] - g[i, j, j, i]
    return e


def fermion_terms(h, g):
    return list(ham.fermion_hamiltonian_terms(h, g))


def sz_number_s2(n_qubits):
    """Dense N, S_z, S^2 from bit-string second quantization."""
    nso = n_qubits
    num = [(1.0, (p,), (p,)) for p in range(nso)]
    sz = [(0.5 if p % 2 == 0 else -0.5, (p,), (p,)) for p in range(nso)]
    splus = [(1.0, (2 * p,), (2 * p + 1,)) for p in range(nso // 2)]
    sminus = [(1.0, (2 * p + 1,), (2 * p,)) for p in range(nso // 2)]
    N = dense.fermion_matrix(num, nso)
    Sz = dense.fermion_matrix(sz, nso)
    Sp = dense.fermion_matrix(splus, nso)
    Sm = dense.fermion_matrix(sminus, nso)
    S2 = Sm @ Sp + Sz @ Sz + Sz
    return N, Sz, S2


@pytest.fixture(scope="module")
def sys8():
    w, h, g = qi.workload("8q")
    H = ham.qubit_hamiltonian(h, g)
    hx, hz, hc, goff = ham.group_by_flip_mask(H)
    excs, ax, az, ac, off, _ = an.build(w["n_orb"], w["n_elec"])
    t = qi.amplitudes(len(excs), w["seed"], w["t_scale"])
    return dict(w=w, h=h, g=g, hx=hx, hz=hz, hc=hc, goff=goff, excs=excs, ax=ax, az=az, ac=ac,
                off=off, t=t, th=an.angles(ac, off, t), n=8, occ=an.reference_mask(w["n_elec"]))


@pytest.fixture(scope="module")
def dense8(sys8):
    hm = dense.fermion_matrix(fermion_terms(sys8["h"], sys8["g"]), sys8["n"])
    return hm


# ---------------------------------------------------------------- Hamiltonian

@pytest.mark.parametrize("n_orb,seed", [(2, 5), (3, 6)])
def test_qubit_hamiltonian_equals_fermion_matrix_small(n_orb, seed):
    h, g = qi.integrals(n_orb, n_orb, seed)
    x, z, c, _ = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    n = 2 * n_orb
    assert np.allclose(dense.pauli_sum_matrix(x, z, c, n),
                       dense.fermion_matrix(fermion_terms(h, g), n), atol=1e-12)


def test_qubit_hamiltonian_equals_fermion_matrix_8q(sys8, dense8):
    assert np.allclose(dense.pauli_sum_matrix(sys8["hx"], sys8["hz"], sys8["hc"], 8), dense8, atol=1e-12)


def test_hamiltonian_symmetries_8q(dense8):
    # real spatial integrals: H is real symmetric and commutes with N, S_z, S^2
    assert np.allclose(dense8, dense8.conj().T)
    assert np.allclose(dense8.imag, 0)
    N, Sz, S2 = sz_number_s2(8)
    for op in (N, Sz, S2):
        assert np.allclose(dense8 @ op, op @ dense8, atol=1e-10)


def test_spin_orbital_integral_symmetry():
    h, g = qi.integrals(3, 4, 9)
    h_so, v = ham.spin_orbital_integrals(h, g)
    assert np.allclose(v, -v.transpose(1, 0, 2, 3))
    assert np.allclose(v, -v.transpose(0, 1, 3, 2))
    assert np.allclose(v, v.transpose(2, 3, 0, 1))
    assert np.allclose(h_so, h_so.T)


@pytest.mark.parametrize("name", ["8q", "20q"])
def test_structural_counts(name):
    w, h, g = qi.workload(name)
    x, z, c, off = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    assert (len(x), len(off) - 1) == expected_counts(w["n_orb"])
    # every string of a real Hamiltonian has an even number of Y factors
    assert all(bin(int(a) & int(b)).count("1") % 2 == 0 for a, b in zip(x, z))
    # groups sorted by flip mask, strings by (x, z)
    keys = list(zip(x.tolist(), z.tolist()))
    assert keys == sorted(keys) and len(set(keys)) == len(keys)


@pytest.mark.slow
def test_structural_counts_28q():
    w, h, g = qi.workload("28q")
    x, z, c, off = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    assert (len(x), len(off) - 1) == expected_counts(14) == (55371, 10466)


# -------------------------------------------------- Table 1 structural pins

def _d2h_filter(n_orb):
    # linear H4 / STO-3G: MOs alternate a_g, b_1u; a product is totally
    # symmetric iff it holds an even number of b_1u orbitals.
    return lambda *so: sum((p // 2) % 2 for p in so) % 2 == 0


def _cnots(x, z):
    return sum(2 * (bin(int(a) | int(b)).count("1") - 1) for a, b in zip(x, z)
               if (int(a) | int(b)) != 0)


def test_table1_pduccd_counts():
    gold = GOLD["table1_h4_sto3g"]["p-dUCCD-VQE"]
    excs = an.paired_doubles(8, 4)
    x, z, c, off = an.ansatz_terms(excs)
    assert len(excs) == gold["N_par"]
    assert _cnots(x, z) == gold["N_CNOT"]


def test_table1_duccsd_counts():
    gold = GOLD["table1_h4_sto3g"]["dUCCSD-VQE"]
    assert gold == GOLD["table1_h4_sto3g"]["dUCCSD-PQE"]
    ok = _d2h_filter(4)
    excs = [e for e in an.excitations(8, 4) if ok(*e[0], *e[1])]
    x, z, c, off = an.ansatz_terms(excs)
    assert len(excs) == gold["N_par"]
    assert _cnots(x, z) == gold["N_CNOT"]


def test_table1_qk_trotter_cnots():
    # One Trotter step (r = 1) of exp(-i dt H) for the D2h-symmetric H4
    # Hamiltonian; the Krylov matrix elements use U_m^dagger U_n, two steps.
    gold = GOLD["table1_h4_sto3g"]["QK"]
    h, g = qi.integrals(4, 4, 77)
    par = [p % 2 for p in range(4)]
    for p in range(4):
        for q in range(4):
            if par[p] != par[q]:
                h[p, q] = 0.0
            for r in range(4):
                for s in range(4):
                    if (par[p] + par[q] + par[r] + par[s]) % 2:
                        g[p, q, r, s] = 0.0
    x, z, c, _ = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    assert len(x) == 185
    assert 2 * _cnots(x, z) == gold["N_CNOT"]


# ------------------------------------------------------------------ ansatz

def test_excitation_counts_and_order():
    for n_orb, n_e, ns, nd in [(4, 4, 8, 18), (10, 10, 50, 825), (6, 6, 18, 99), (7, 7, 24, 180)]:
        excs = an.excitations(2 * n_orb, n_e)
        assert sum(1 for e in excs if len(e[0]) == 1) == ns
        assert sum(1 for e in excs if len(e[0]) == 2) == nd
        ref = an.reference_mask(n_e)
        dets = []
        for cre, ann in excs:
            s, b = dense.apply_string(ref, cre, ann)
            assert s != 0
            assert bin(b).count("1") == n_e
            dets.append(b)
        assert dets == sorted(dets)


def test_kappa_strings_commute_share_mask():
    excs = an.excitations(10, 4)
    for cre, ann in excs:
        st = an.kappa_strings(cre, ann)
        assert len(st) == (2 if len(cre) == 1 else 8)
        keys = list(st)
        xs = {k[0] for k in keys}
        assert len(xs) == 1 and xs.pop() == sum(1 << p for p in cre + ann)
        for a in keys:
            for b in keys:
                x1, z1, k1 = pauli.pauli_mul(a[0], a[1], b[0], b[1])
                x2, z2, k2 = pauli.pauli_mul(b[0], b[1], a[0], a[1])
                assert (x1, z1, k1) == (x2, z2, k2)
        # kappa = i sum c P is anti-Hermitian: odd number of Y in every string
        assert all(bin(k[0] & k[1]).count("1") % 2 == 1 for k in keys)


def test_kappa_matches_fermion_matrix():
    n = 6
    for cre, ann in an.excitations(n, 2)[:6]:
        st = an.kappa_strings(cre, ann)
        m = sum(1j * c * dense.pauli_matrix(x, z, n) for (x, z), c in st.items())
        want = dense.fermion_matrix([(1.0, cre, ann), (-1.0, tuple(reversed(ann)),
                                                        tuple(reversed(cre)))], n)
        assert np.allclose(m, want)


def test_top_k_ties_and_order():
    t = np.array([0.1, -0.3, 0.3, 0.05, -0.1])
    assert an.top_k(t, 3).tolist() == [0, 1, 2]
    assert an.top_k(t, 2).tolist() == [1, 2]
    assert an.top_k(t, 4).tolist() == [0, 1, 2, 4]


def test_single_factor_closed_form_and_omega(sys8):
    # exp(t kappa) Phi_0 = cos t Phi_0 + s sin t Phi_mu; at t = pi/4 this is
    # Omega_mu of Eq. (24) (up to the fermionic sign s of tau Phi_0).
    n, occ = sys8["n"], sys8["occ"]
    t_om = GOLD["omega_mu"]["t"]
    for cre, ann in sys8["excs"]:
        s, det = dense.apply_string(occ, cre, ann)
        x, z, c, off = an.ansatz_terms([(cre, ann)])
        for t in (0.37, -1.1, t_om):
            psi = sv.apply_product(sv.prepare(n, occ), n, x, z, an.angles(c, off, np.array([t])))
            want = np.zeros(1 << n, dtype=np.complex128)
            want[occ] = math.cos(t)
            want[det] = s * math.sin(t)
            assert np.allclose(psi, want, atol=1e-14)
        assert abs(psi[occ]) == pytest.approx(1 / math.sqrt(2), abs=1e-15)


# ------------------------------------------------------------- energies

def test_theta_zero_energy_is_hf(sys8, dense8):
    n, occ = sys8["n"], sys8["occ"]
    psi = sv.prepare(n, occ)
    e = sv.energy(psi, n, sys8["hx"], sys8["hz"], sys8["hc"])
    assert e == pytest.approx(hf_closed_shell(sys8["h"], sys8["g"], 2), abs=1e-12)
    assert e == pytest.approx(dense8[occ, occ].real, abs=1e-12)


def test_energy_equals_dense_expectation(sys8, dense8):
    n, occ = sys8["n"], sys8["occ"]
    psi = sv.apply_product(sv.prepare(n, occ), n, sys8["ax"], sys8["az"], sys8["th"])
    e = sv.energy(psi, n, sys8["hx"], sys8["hz"], sys8["hc"])
    assert e == pytest.approx(np.vdot(psi, dense8 @ psi).real, abs=1e-12)
    lam = sv.sigma(psi, n, sys8["hx"], sys8["hz"], sys8["hc"])
    assert np.allclose(lam, dense8 @ psi, atol=1e-12)


def test_variational_bound(sys8, dense8):
    n, occ = sys8["n"], sys8["occ"]
    e0 = dense.ground_energy_in_sector(dense8, n, 4, 0)
    for seed in range(5):
        t = qi.amplitudes(len(sys8["excs"]), 500 + seed, 1.0)
        th = an.angles(sys8["ac"], sys8["off"], t)
        e = sv.energy_of(n, occ, sys8["ax"], sys8["az"], th, sys8["hx"], sys8["hz"], sys8["hc"])
        assert e >= e0 - 1e-12


def test_invariants_at_excitation_boundaries(sys8):
    n, occ = sys8["n"], sys8["occ"]
    psi = sv.prepare(n, occ)
    off = sys8["off"]
    N, Sz, _ = sz_number_s2(n)
    sector = np.array([bin(b).count("1") == 4 for b in range(1 << n)])
    for mu in range(len(off) - 1):
        sl = slice(off[mu], off[mu + 1])
        psi = sv.apply_product(psi, n, sys8["ax"][sl], sys8["az"][sl], sys8["th"][sl])
        assert np.vdot(psi, psi).real == pytest.approx(1.0, abs=1e-12)
        assert np.vdot(psi, N @ psi).real == pytest.approx(4.0, abs=1e-12)
        assert np.vdot(psi, Sz @ psi).real == pytest.approx(0.0, abs=1e-12)
        assert np.max(np.abs(psi[~sector])) <= 1e-12


# ------------------------------------------------------------- gradients

def test_gradient_at_zero_is_matrix_element(sys8, dense8):
    n, occ = sys8["n"], sys8["occ"]
    K = len(sys8["ax"])
    e, gth = sv.adjoint_gradient(n, occ, sys8["ax"], sys8["az"], np.zeros(K),
                                 sys8["hx"], sys8["hz"], sys8["hc"])
    gt = an.grad_t(sys8["ac"], sys8["off"], gth)
    for mu, (cre, ann) in enumerate(sys8["excs"]):
        s, det = dense.apply_string(occ, cre, ann)
        assert gt[mu] == pytest.approx(2 * s * dense8[occ, det].real, abs=1e-12)


def test_adjoint_equals_parameter_shift_and_fd(sys8):
    n, occ = sys8["n"], sys8["occ"]
    args = (sys8["hx"], sys8["hz"], sys8["hc"])
    e, g_adj = sv.adjoint_gradient(n, occ, sys8["ax"], sys8["az"], sys8["th"], *args)
    g_ps = sv.parameter_shift_gradient(n, occ, sys8["ax"], sys8["az"], sys8["th"], *args)
    assert np.max(np.abs(g_adj - g_ps)) < 1e-12
    # central finite differences in t_mu on a few amplitudes
    t = sys8["t"]
    gt = an.grad_t(sys8["ac"], sys8["off"], g_adj)
    hstep = 1e-5
    for mu in (0, 5, len(t) - 1):
        tp, tm = t.copy(), t.copy()
        tp[mu] += hstep
        tm[mu] -= hstep
        ep = sv.energy_of(n, occ, sys8["ax"], sys8["az"], an.angles(sys8["ac"], sys8["off"], tp), *args)
        em = sv.energy_of(n, occ, sys8["ax"], sys8["az"], an.angles(sys8["ac"], sys8["off"], tm), *args)
        assert (ep - em) / (2 * hstep) == pytest.approx(gt[mu], abs=1e-8)


# ------------------------------------------------------------- C core

def test_c_core_matches_numpy_random_terms():
    n = 9
    psi0 = qi.random_state(n, 21)
    xs, zs, cs = qi.random_paulis(n, 40, 22)
    th = qi.random_angles(40, 23)
    a = sv.apply_product(psi0, n, xs, zs, th)
    b = core.apply_product(psi0.copy(), n, xs, zs, th)
    assert np.allclose(a, b, atol=1e-13)
    back = core.apply_product(b.copy(), n, xs, zs, th, inverse=True)
    assert np.allclose(back, psi0, atol=1e-13)
    # energy over a grouped random Hermitian sum vs dense
    order = np.lexsort((zs, xs))
    xs, zs, cs = xs[order], zs[order], cs[order]
    goff = [0] + [i for i in range(1, len(xs)) if xs[i] != xs[i - 1]] + [len(xs)]
    hm = dense.pauli_sum_matrix(xs, zs, cs, n)
    assert core.energy(a, n, xs, zs, cs, goff) == pytest.approx(np.vdot(a, hm @ a).real, abs=1e-12)
    assert np.allclose(core.sigma(a, n, xs, zs, cs), hm @ a, atol=1e-12)


def test_c_core_energy_grad_matches_numpy(sys8):
    n, occ = sys8["n"], sys8["occ"]
    args = (sys8["hx"], sys8["hz"], sys8["hc"])
    e1, g1 = sv.adjoint_gradient(n, occ, sys8["ax"], sys8["az"], sys8["th"], *args)
    e2, g2 = core.energy_grad(n, occ, sys8["ax"], sys8["az"], sys8["th"], *args)
    psi = core.apply_product(core.prepare(n, occ), n, sys8["ax"], sys8["az"], sys8["th"])
    e3 = core.energy(psi, n, *args, sys8["goff"])
    assert e1 == pytest.approx(e2, abs=1e-12) and e1 == pytest.approx(e3, abs=1e-12)
    assert np.max(np.abs(g1 - g2)) < 1e-12


def test_c_core_hf_energy_20q():
    w, h, g = qi.workload("20q")
    x, z, c, off = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    psi = core.prepare(20, an.reference_mask(10))
    assert core.energy(psi, 20, x, z, c, off) == pytest.approx(hf_closed_shell(h, g, 5), abs=1e-11)


# ---------------------------------------------- diagonal strings, <N>

def _diag_mix(n, count, seed):
    """Random strings with every third one diagonal (x = 0, Z-only, with the
    identity among them): the x = 0 branch of the C core's exponential."""
    xs, zs, cs = qi.random_paulis(n, count, seed)
    rng = np.random.default_rng([seed, 5])
    for k in range(0, count, 3):
        xs[k] = 0
        zs[k] = 0 if k == 0 else int(rng.integers(1, 1 << n))
    return xs, zs, cs


def test_c_core_exp_matches_matrix_exponential():
    # exp(-i theta P) by scipy's matrix exponential of the dense Kronecker
    # matrix: neither the cos/sin identity nor the pair loop is involved.
    from scipy.linalg import expm
    n = 6
    psi0 = qi.random_state(n, 31)
    xs, zs, _ = _diag_mix(n, 18, 32)
    th = qi.random_angles(18, 33)
    assert sum(1 for x in xs if int(x) == 0) >= 5
    for x, z, t in zip(xs, zs, th):
        want = expm(-1j * float(t) * dense.pauli_matrix(int(x), int(z), n)) @ psi0
        got = core.apply_product(psi0.copy(), n, [x], [z], [t])
        assert np.allclose(got, want, atol=1e-13), (int(x), int(z))


def test_c_core_diagonal_runs_energy_sigma_dense():
    n = 8
    psi0 = qi.random_state(n, 41)
    xs, zs, cs = _diag_mix(n, 45, 42)
    th = qi.random_angles(45, 43)
    a = core.apply_product(psi0.copy(), n, xs, zs, th)
    u = np.eye(1 << n, dtype=np.complex128)
    for x, z, t in zip(xs, zs, th):
        u = (math.cos(t) * np.eye(1 << n) - 1j * math.sin(t) * dense.pauli_matrix(int(x), int(z), n)) @ u
    assert np.allclose(a, u @ psi0, atol=1e-13)
    order = np.lexsort((zs, xs))
    hx, hz, hc = xs[order], zs[order], cs[order]
    goff = [0] + [i for i in range(1, len(hx)) if hx[i] != hx[i - 1]] + [len(hx)]
    assert hx[0] == 0 and goff[1] >= 5  # a diagonal group of several strings
    hm = dense.pauli_sum_matrix(hx, hz, hc, n)
    assert core.energy(a, n, hx, hz, hc, goff) == pytest.approx(np.vdot(a, hm @ a).real, abs=1e-12)
    assert np.allclose(core.sigma(a, n, hx, hz, hc), hm @ a, atol=1e-12)


def test_c_core_gradient_with_diagonal_runs_vs_dense_shift():
    # E(theta) through dense matrices; the exact shift rule of P^2 = I
    # gives dE/dtheta_k = E(theta_k + pi/4) - E(theta_k - pi/4).
    n = 8
    occ = 0b00110101
    xs, zs, _ = _diag_mix(n, 24, 51)
    th = qi.random_angles(24, 52)
    hx, hz, hc = qi.random_paulis(n, 30, 53, max_weight=4)
    order = np.lexsort((hz, hx))
    hx, hz, hc = hx[order], hz[order], hc[order]
    hm = dense.pauli_sum_matrix(hx, hz, hc, n)  # Hermitian: real coefficients of Hermitian strings
    pm = [dense.pauli_matrix(int(x), int(z), n) for x, z in zip(xs, zs)]

    def e_dense(theta):
        v = np.zeros(1 << n, dtype=np.complex128)
        v[occ] = 1
        for P, t in zip(pm, theta):
            v = math.cos(t) * v - 1j * math.sin(t) * (P @ v)
        return float(np.vdot(v, hm @ v).real)

    e, g = core.energy_grad(n, occ, xs, zs, th, hx, hz, hc)
    assert e == pytest.approx(e_dense(th), abs=1e-12)
    for k in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[k] += math.pi / 4
        tm[k] -= math.pi / 4
        assert g[k] == pytest.approx(e_dense(tp) - e_dense(tm), abs=1e-11), k


def test_number_expectation_matches_dense_operators(sys8):
    n = sys8["n"]
    N, _, _ = sz_number_s2(n)
    n_alpha = dense.fermion_matrix([(1.0, (p,), (p,)) for p in range(0, n, 2)], n)
    for seed in (61, 62):
        psi = qi.random_state(n, seed)
        assert sv.number_expectation(psi, n) == pytest.approx(np.vdot(psi, N @ psi).real, abs=1e-12)
        alpha = sum(1 << p for p in range(0, n, 2))
        assert sv.number_expectation(psi, n, alpha) == pytest.approx(np.vdot(psi, n_alpha @ psi).real, abs=1e-12)
    psi = sv.apply_product(sv.prepare(n, sys8["occ"]), n, sys8["ax"], sys8["az"], sys8["th"])
    assert sv.number_expectation(psi, n) == pytest.approx(4.0, abs=1e-12)
