"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances: energies 1e-10 Hartree, gradients 1e-9, amplitudes 1e-12 (the
state is unit-norm; FP64 rounding of a few thousand rotations stays near
1e-14).  Small cases run the oracle live; the 20- and 28-qubit workloads
compare with values written by tests/golden/make_golden.py (oracle only).
"""
import json
import math
import os

import numpy as np
import pytest

import qf_inputs as qi
from oracle import ansatz as an, core, hamiltonian as ham, statevec as sv

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")
E_TOL, G_TOL, A_TOL = 1e-10, 1e-9, 1e-12


@pytest.fixture(scope="module")
def qf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2108_04413_amd as qf
    return qf


def dev(psi):
    return torch.from_numpy(np.ascontiguousarray(psi)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def grouped(xs, zs, cs):
    order = np.lexsort((zs, xs))
    xs, zs, cs = xs[order], zs[order], cs[order]
    off = [0] + [i for i in range(1, len(xs)) if xs[i] != xs[i - 1]] + [len(xs)]
    return xs, zs, cs, np.array(off, dtype=np.int64)


def runs_of_terms(n, seed, count=60):
    """Random strings arranged in same-mask runs: commuting and
    anticommuting neighbours, diagonal (x = 0) runs, odd and even Y."""
    rng = np.random.default_rng([seed, 77])
    xs, zs = [], []
    while len(xs) < count:
        x = 0 if rng.random() < 0.2 else int(rng.integers(1, 1 << n))
        for _ in range(int(rng.integers(1, 11))):
            xs.append(x)
            zs.append(int(rng.integers(0, 1 << n)))
    return (np.array(xs[:count], dtype=np.uint64), np.array(zs[:count], dtype=np.uint64))


def system(name):
    w, h, g = qi.workload(name)
    n = 2 * w["n_orb"]
    x, z, c, off = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    excs, ax, az, ac, aoff, _ = an.build(w["n_orb"], w["n_elec"])
    t = qi.amplitudes(len(excs), w["seed"], w["t_scale"])
    return w, n, an.reference_mask(w["n_elec"]), (x, z, c, off), (ax, az, ac, aoff, an.angles(ac, aoff, t))


# ----------------------------------------------------------------- prepare

@pytest.mark.parametrize("n,occ", [(1, 1), (5, 0b10110), (13, 0b1111111), (20, (1 << 10) - 1)])
def test_prepare_bit_exact(qf, n, occ):
    psi = torch.full((1 << n,), 7.0 + 3.0j, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, n, occ)
    assert np.array_equal(host(psi), sv.prepare(n, occ))


# ------------------------------------------------------------------- apply

@pytest.mark.parametrize("n,seed", [(1, 1), (3, 2), (9, 3), (13, 4)])
@pytest.mark.parametrize("inverse", [False, True])
def test_apply_random_runs(qf, n, seed, inverse):
    xs, zs = runs_of_terms(n, seed)
    th = qi.random_angles(len(xs), seed + 100)
    psi0 = qi.random_state(n, seed)
    A = qf.terms_array(xs, zs, np.ones(len(xs)))
    psi = dev(psi0)
    qf.apply_pauli_exp(psi, n, A, th, inverse=inverse)
    want = sv.apply_product(psi0, n, xs, zs, th, inverse=inverse)
    assert np.max(np.abs(host(psi) - want)) < A_TOL


def test_apply_then_inverse_restores(qf):
    n = 12
    xs, zs = runs_of_terms(n, 9, 200)
    th = qi.random_angles(len(xs), 10)
    psi0 = qi.random_state(n, 11)
    A = qf.terms_array(xs, zs, np.ones(len(xs)))
    psi = dev(psi0)
    qf.apply_pauli_exp(psi, n, A, th)
    qf.apply_pauli_exp(psi, n, A, th, inverse=True)
    assert np.max(np.abs(host(psi) - psi0)) < A_TOL


def test_apply_theta_zero_bit_exact(qf):
    n = 10
    xs, zs = runs_of_terms(n, 12, 80)
    psi0 = qi.random_state(n, 13)
    psi = dev(psi0)
    qf.apply_pauli_exp(psi, n, qf.terms_array(xs, zs, np.ones(len(xs))), np.zeros(len(xs)))
    assert np.array_equal(host(psi), psi0)


@pytest.mark.parametrize("name", ["8q"])
def test_apply_ansatz_matches_oracle(qf, name):
    w, n, occ, _, (ax, az, ac, aoff, th) = system(name)
    A = qf.terms_array(ax, az, ac)
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, n, occ)
    qf.apply_pauli_exp(psi, n, A, th)
    want = sv.apply_product(sv.prepare(n, occ), n, ax, az, th)
    assert np.max(np.abs(host(psi) - want)) < A_TOL


# ------------------------------------------------------------------ energy

@pytest.mark.parametrize("n,seed", [(1, 5), (4, 6), (10, 7), (14, 8)])
def test_energy_random_hermitian_sum(qf, n, seed):
    xs, zs, cs = qi.random_paulis(n, 300, seed)
    xs[:20] = 0  # a diagonal group
    xs, zs, cs, off = grouped(xs, zs, cs)
    H = qf.terms_array(xs, zs, cs)
    psi0 = qi.random_state(n, seed + 1)
    e = qf.energy(dev(psi0), n, H, off)
    assert e == pytest.approx(core.energy(psi0, n, xs, zs, cs, off), abs=E_TOL)


def test_energy_hf_closed_form_8q(qf):
    w, h, g = qi.workload("8q")
    terms, off, _ = qf.build_paulis("hamiltonian", 4, 4, h, g)
    psi = torch.empty(256, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, 8, 0b1111)
    e_cf = 2 * sum(h[i, i] for i in range(2)) + sum(2 * g[i, i, j, j] - g[i, j, j, i]
                                                    for i in range(2) for j in range(2))
    assert qf.energy(psi, 8, terms, off) == pytest.approx(e_cf, abs=E_TOL)


def test_energy_and_grad_8q(qf):
    w, n, occ, (x, z, c, off), (ax, az, ac, aoff, th) = system("8q")
    H = qf.terms_array(x, z, c)
    A = qf.terms_array(ax, az, ac)
    e, g = qf.energy_grad(n, occ, A, th, H, off)
    e_o, g_o = sv.adjoint_gradient(n, occ, ax, az, th, x, z, c)
    g_ps = sv.parameter_shift_gradient(n, occ, ax, az, th, x, z, c)
    assert e == pytest.approx(e_o, abs=E_TOL)
    assert np.max(np.abs(g - g_o)) < G_TOL
    assert np.max(np.abs(g - g_ps)) < G_TOL


@pytest.mark.parametrize("n,seed", [(5, 20), (11, 21)])
def test_energy_grad_random_terms(qf, n, seed):
    """General runs (diagonal, mixed commuting sets) through the adjoint."""
    ax, az = runs_of_terms(n, seed, 70)
    th = qi.random_angles(len(ax), seed + 3, 1.0)
    hx, hz, hc = qi.random_paulis(n, 120, seed + 4)
    hx, hz, hc, off = grouped(hx, hz, hc)
    occ = (1 << (n // 2)) - 1
    e, g = qf.energy_grad(n, occ, qf.terms_array(ax, az, np.ones(len(ax))), th,
                          qf.terms_array(hx, hz, hc), off)
    e_o, g_o = core.energy_grad(n, occ, ax, az, th, hx, hz, hc)
    assert e == pytest.approx(e_o, abs=E_TOL)
    assert np.max(np.abs(g - g_o)) < G_TOL


def test_uccsd_12q_energy_grad(qf):
    h, g = qi.integrals(6, 6, 2005)
    x, z, c, off = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    excs, ax, az, ac, aoff, _ = an.build(6, 6)
    t = qi.amplitudes(len(excs), 2005, 0.2)
    th = an.angles(ac, aoff, t)
    occ = an.reference_mask(6)
    e, gth = qf.energy_grad(12, occ, qf.terms_array(ax, az, ac), th, qf.terms_array(x, z, c), off)
    e_o, g_o = core.energy_grad(12, occ, ax, az, th, x, z, c)
    assert e == pytest.approx(e_o, abs=E_TOL)
    assert np.max(np.abs(gth - g_o)) < G_TOL


def test_sigma_matches_oracle(qf):
    n = 10
    xs, zs, cs = qi.random_paulis(n, 200, 31)
    xs, zs, cs, off = grouped(xs, zs, cs)
    psi0 = qi.random_state(n, 32)
    plan = qf.Plan(n, None, qf.terms_array(xs, zs, cs), off)
    lam = torch.empty_like(dev(psi0))
    e = plan.sigma(dev(psi0), lam)
    want = core.sigma(psi0, n, xs, zs, cs)
    assert np.max(np.abs(host(lam) - want)) < 1e-11
    assert e == pytest.approx(core.energy(psi0, n, xs, zs, cs, off), abs=E_TOL)


@pytest.mark.parametrize("real_only", [False, True])
def test_sigma_17q_matches_oracle(qf, real_only):
    """lambda = H psi at 17 qubits, with and without imaginary-phase strings
    (odd number of Y): many groups, high flip bits and the diagonal group."""
    n = 17
    xs, zs, cs = qi.random_paulis(n, 900, 33)
    rng = np.random.default_rng(34)
    # strings with low flip masks only, so classes hold several groups
    lx = rng.integers(0, 1 << 11, 300).astype(np.uint64)
    lz = rng.integers(0, 1 << n, 300).astype(np.uint64)
    xs, zs = np.concatenate([xs, lx, np.zeros(20, np.uint64)]), np.concatenate([zs, lz, lz[:20]])
    cs = np.concatenate([cs, rng.normal(size=320)])
    if real_only:
        keep = np.array([bin(int(x) & int(z)).count("1") % 2 == 0 for x, z in zip(xs, zs)])
        xs, zs, cs = xs[keep], zs[keep], cs[keep]
    xs, zs, cs, off = grouped(xs, zs, cs)
    psi0 = qi.random_state(n, 35)
    plan = qf.Plan(n, None, qf.terms_array(xs, zs, cs), off)
    assert plan.info()["tile_bits"] == -11
    lam = torch.empty_like(dev(psi0))
    e = plan.sigma(dev(psi0), lam)
    want = core.sigma(psi0, n, xs, zs, cs)
    assert np.max(np.abs(host(lam) - want)) < 1e-11
    assert e == pytest.approx(core.energy(psi0, n, xs, zs, cs, off), abs=E_TOL)


@pytest.mark.parametrize("n", [12, 13])
def test_sigma_tiled_edge_cases_match_oracle(qf, n):
    """The class-tiled sigma at its smallest sizes (2 and 4 tiles of 2^11),
    with groups given out of flip-mask order (strings of a class are then
    not contiguous) and a diagonal group of 150 strings (longer than the
    64 strings a wave holds at a time)."""
    rng = np.random.default_rng([n, 41])
    xs, zs, cs = qi.random_paulis(n, 400, 40 + n)
    dz = rng.integers(0, 1 << n, 150).astype(np.uint64)
    xs = np.concatenate([xs, np.zeros(150, np.uint64)])
    zs = np.concatenate([zs, dz])
    cs = np.concatenate([cs, rng.normal(size=150)])
    xs, zs, cs, off = grouped(xs, zs, cs)
    # shuffle whole groups
    G = len(off) - 1
    perm = rng.permutation(G)
    parts = [np.arange(off[g], off[g + 1]) for g in perm]
    idx = np.concatenate(parts)
    xs, zs, cs = xs[idx], zs[idx], cs[idx]
    off = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    psi0 = qi.random_state(n, 50 + n)
    plan = qf.Plan(n, None, qf.terms_array(xs, zs, cs), off)
    lam = torch.empty_like(dev(psi0))
    e = plan.sigma(dev(psi0), lam)
    want = core.sigma(psi0, n, xs, zs, cs)
    assert np.max(np.abs(host(lam) - want)) < 1e-11
    assert e == pytest.approx(core.energy(psi0, n, xs, zs, cs, off), abs=E_TOL)


def test_plan_matches_one_shot_and_is_deterministic(qf):
    w, n, occ, (x, z, c, off), (ax, az, ac, aoff, th) = system("8q")
    H = qf.terms_array(x, z, c)
    A = qf.terms_array(ax, az, ac)
    plan = qf.Plan(n, A, H, off)
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    e1, g1 = plan.energy_grad(occ, th, ws)
    e2, g2 = plan.energy_grad(occ, th, ws)
    e3, g3 = qf.energy_grad(n, occ, A, th, H, off)
    assert e1 == e2 == e3
    assert np.array_equal(g1, g2) and np.array_equal(g1, g3)


# --------------------------------------------------------- full workloads

def _golden(name):
    path = os.path.join(GOLD, f"oracle_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


def _build_device_system(qf, name):
    w, h, g = qi.workload(name)
    n = 2 * w["n_orb"]
    H, off, _ = qf.build_paulis("hamiltonian", w["n_orb"], w["n_elec"], h, g)
    if w["ansatz"] == "uccd_top":
        _, off_all, _ = qf.build_paulis("uccd", w["n_orb"], w["n_elec"])
        t_all = qi.amplitudes(len(off_all) - 1, w["seed"], w["t_scale"])
        A, aoff, kept = qf.build_paulis("uccd_top", w["n_orb"], w["n_elec"], t_rank=t_all, top_k=w["top_k"])
        t = t_all[kept]
    else:
        A, aoff, kept = qf.build_paulis("uccsd", w["n_orb"], w["n_elec"])
        t = qi.amplitudes(len(aoff) - 1, w["seed"], w["t_scale"])
    return w, n, (1 << w["n_elec"]) - 1, H, off, A, aoff, qf.ansatz_angles(A, aoff, t)


def test_20q_energy_grad_vs_golden(qf):
    gold = _golden("20q")
    w, n, occ, H, off, A, aoff, th = _build_device_system(qf, "20q")
    assert (len(H), len(off) - 1, len(A)) == (gold["n_strings"], gold["n_groups"], gold["K"])
    plan = qf.Plan(n, A, H, off)
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, n, occ)
    plan.apply(psi, th)
    e = plan.energy(psi)
    assert e == pytest.approx(gold["energy"], abs=E_TOL)
    idx = np.array(gold["sample_index"])
    got = host(psi)[idx]
    want = np.array(gold["sample_re"]) + 1j * np.array(gold["sample_im"])
    assert np.max(np.abs(got - want)) < A_TOL
    lam = torch.empty_like(psi)
    e_s = plan.sigma(psi, lam)
    assert e_s == pytest.approx(gold["energy"], abs=E_TOL)
    want_l = np.array(gold["sigma_re"]) + 1j * np.array(gold["sigma_im"])
    assert np.max(np.abs(host(lam)[idx] - want_l)) < 1e-10
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    e_g, g = plan.energy_grad(occ, th, ws)
    assert e_g == pytest.approx(gold["energy"], abs=E_TOL)
    assert np.max(np.abs(g - np.array(gold["grad_theta"]))) < G_TOL
    assert np.max(np.abs(qf.grad_t(A, aoff, g) - np.array(gold["grad_t"]))) < G_TOL


def test_28q_hf_energy_closed_form(qf):
    w, h, g = qi.workload("28q")
    H, off, _ = qf.build_paulis("hamiltonian", 14, 14, h, g)
    psi = torch.empty(1 << 28, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, 28, (1 << 14) - 1)
    e_cf = 2 * sum(h[i, i] for i in range(7)) + sum(2 * g[i, i, j, j] - g[i, j, j, i]
                                                    for i in range(7) for j in range(7))
    assert qf.energy(psi, 28, H, off) == pytest.approx(e_cf, abs=E_TOL)
    del psi
    torch.cuda.empty_cache()


def test_30q_reference_energy_and_identity_ansatz(qf):
    """30 qubits (16 GiB state, the largest the library accepts): the
    closed-form Hartree-Fock energy through the streaming energy kernel, and
    the blocked apply with all angles zero leaving the reference exactly."""
    h, g = qi.integrals(15, 15, 1130)
    H, off, _ = qf.build_paulis("hamiltonian", 15, 15, h, g)
    A, aoff, _ = qf.build_paulis("uccd", 15, 15)
    A = A[: int(aoff[64])]  # the first 64 doubles
    n, occ = 30, (1 << 15) - 1
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    plan = qf.Plan(n, A, H, off)
    qf.prepare_state(psi, n, occ)
    plan.apply(psi, np.zeros(len(A)))
    # open shell: 8 alpha (orbitals 0..7), 7 beta (orbitals 0..6)
    occ_a, occ_b = list(range(8)), list(range(7))
    e_cf = sum(h[i, i] for i in occ_a) + sum(h[i, i] for i in occ_b)
    for P in occ_a:
        for Q in occ_a:
            e_cf += 0.5 * (g[P, P, Q, Q] - g[P, Q, Q, P])
    for P in occ_b:
        for Q in occ_b:
            e_cf += 0.5 * (g[P, P, Q, Q] - g[P, Q, Q, P])
    for P in occ_a:
        for Q in occ_b:
            e_cf += g[P, P, Q, Q]
    assert plan.energy(psi) == pytest.approx(e_cf, abs=E_TOL)
    # the reference amplitude and a sample elsewhere are untouched
    assert complex(psi[occ].item()) == 1.0
    assert float(torch.max(torch.abs(psi[occ + 1: occ + 1 + (1 << 20)]))) == 0.0
    del psi
    torch.cuda.empty_cache()


def test_28q_energy_vs_golden(qf):
    gold = _golden("28q")
    w, n, occ, H, off, A, aoff, th = _build_device_system(qf, "28q")
    plan = qf.Plan(n, A, H, off)
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, n, occ)
    plan.apply(psi, th)
    e = plan.energy(psi)
    assert e == pytest.approx(gold["energy"], abs=E_TOL)
    idx = torch.from_numpy(np.array(gold["sample_index"])).to("cuda")
    got = host(psi[idx])
    want = np.array(gold["sample_re"]) + 1j * np.array(gold["sample_im"])
    assert np.max(np.abs(got - want)) < A_TOL
    norm = float(torch.vdot(psi, psi).real)
    assert norm == pytest.approx(1.0, abs=1e-12)
    del psi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("L,merged", [(0, False), (10, False), (11, False), (12, False),
                                      (10, True), (11, True), (12, True)])
def test_energy_tile_variants_match_oracle(qf, L, merged):
    n = 14
    xs, zs, cs = qi.random_paulis(n, 500, 90)
    xs[:40] = 0                        # diagonal group
    xs[40:120] &= np.uint64(0x3FF)     # flip bits inside a tile
    xs[120:200] &= np.uint64(0x3C00)   # flip bits only above the tile
    xs, zs, cs, off = grouped(xs, zs, cs)
    psi0 = qi.random_state(n, 91)
    plan = qf.Plan(n, None, qf.terms_array(xs, zs, cs), off)
    plan.set_energy_tile(L, merged)
    info = plan.info()
    assert info["tile_bits"] == (-L if merged else L)
    e = plan.energy(dev(psi0))
    assert e == pytest.approx(core.energy(psi0, n, xs, zs, cs, off), abs=E_TOL)


def test_20q_energy_untiled_and_tiled_agree_with_golden(qf):
    gold = _golden("20q")
    w, n, occ, H, off, A, aoff, th = _build_device_system(qf, "20q")
    plan = qf.Plan(n, A, H, off)
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, n, occ)
    plan.apply(psi, th)
    for L, merged in ((0, False), (11, False), (11, True), (12, True)):
        plan.set_energy_tile(L, merged)
        assert plan.energy(psi) == pytest.approx(gold["energy"], abs=E_TOL)


@pytest.mark.parametrize("B", [0, 6, 9, 12])
@pytest.mark.parametrize("inverse", [False, True])
def test_blocked_apply_matches_oracle(qf, B, inverse):
    """Sub-cube application: segments of runs, incl. runs too wide to fit."""
    n = 14
    xs, zs = runs_of_terms(n, 40 + B, 160)
    # a block of low-mask excitation-like runs so that segments hold many runs
    rng = np.random.default_rng(7 + B)
    lowx = [int(v) for v in rng.choice([0b1111, 0b110011, 0b101000101, 0b11], 40)]
    xs = np.concatenate([np.array(lowx, dtype=np.uint64), xs])
    zs = np.concatenate([rng.integers(0, 1 << n, 40).astype(np.uint64), zs])
    th = qi.random_angles(len(xs), 60 + B)
    psi0 = qi.random_state(n, 61)
    A = qf.terms_array(xs, zs, np.ones(len(xs)))
    plan = qf.Plan(n, A)
    plan.set_block_bits(B)
    info = plan.apply_info()
    assert info["block_bits"] == B and info["passes"] <= info["runs"]
    psi = dev(psi0)
    plan.apply(psi, th, inverse=inverse)
    want = sv.apply_product(psi0, n, xs, zs, th, inverse=inverse)
    assert np.max(np.abs(host(psi) - want)) < A_TOL


def test_blocked_apply_20q_ansatz_matches_golden_samples(qf):
    gold = _golden("20q")
    w, n, occ, H, off, A, aoff, th = _build_device_system(qf, "20q")
    plan = qf.Plan(n, A, H, off)
    info = plan.apply_info()
    assert info["block_bits"] == 12 and info["passes"] < info["runs"] // 10
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, n, occ)
    plan.apply(psi, th)
    idx = np.array(gold["sample_index"])
    want = np.array(gold["sample_re"]) + 1j * np.array(gold["sample_im"])
    assert np.max(np.abs(host(psi)[idx] - want)) < A_TOL
    assert plan.energy(psi) == pytest.approx(gold["energy"], abs=E_TOL)


@pytest.mark.parametrize("B", [0, 10, 11, 12])
def test_blocked_adjoint_matches_oracle(qf, B):
    """Blocked reverse sweep (segments of runs undone in LDS sub-cubes of phi
    and lambda), incl. diagonal runs and runs too wide for a sub-cube."""
    n = 13
    xs, zs = runs_of_terms(n, 80 + B, 150)
    rng = np.random.default_rng(9 + B)
    lowx = [int(v) for v in rng.choice([0, 0b1111, 0b110011, 0b101000101, 0b11], 40)]
    xs = np.concatenate([np.array(lowx, dtype=np.uint64), xs])
    zs = np.concatenate([rng.integers(0, 1 << n, 40).astype(np.uint64), zs])
    th = qi.random_angles(len(xs), 90 + B, 1.0)
    hx, hz, hc = qi.random_paulis(n, 150, 91 + B)
    hx, hz, hc, off = grouped(hx, hz, hc)
    occ = (1 << 6) - 1
    plan = qf.Plan(n, qf.terms_array(xs, zs, np.ones(len(xs))), qf.terms_array(hx, hz, hc), off)
    plan.set_block_bits(B)
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    e, g = plan.energy_grad(occ, th, ws)
    e_o, g_o = core.energy_grad(n, occ, xs, zs, th, hx, hz, hc)
    assert e == pytest.approx(e_o, abs=E_TOL)
    assert np.max(np.abs(g - g_o)) < G_TOL


def multi_run_terms(n, seed, runs=120):
    """Runs that form the multi-run LDS passes (flip runs with an odd number
    of Y, rank <= 3, masks inside qubits 0..11) interleaved with runs that
    must take the one-run path: diagonal runs, even-Y runs, runs of rank > 3
    and runs repeating the previous mask."""
    rng = np.random.default_rng([seed, 131])
    xs, zs = [], []
    prev = 0
    for r in range(runs):
        kind = rng.random()
        if kind < 0.08:
            x = 0
        elif kind < 0.12 and prev:
            x = prev
        else:
            bits = rng.choice(12, size=int(rng.integers(2, 5)), replace=False)
            x = int(sum(1 << int(b) for b in bits))
        odd = kind >= 0.2 or x == 0
        wide = 0.16 <= kind < 0.2
        m = int(rng.integers(6, 9)) if wide else int(rng.integers(1, 5))
        for _ in range(m):
            z = int(rng.integers(0, 1 << n))
            if x and ((bin(x & z).count("1") & 1) != (1 if odd else 0)):
                z ^= 1 << int(np.flatnonzero([(x >> q) & 1 for q in range(n)])[0])
            xs.append(x)
            zs.append(z)
        prev = x
    return np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64)


@pytest.mark.parametrize("seed", [1, 2])
def test_multi_run_passes_match_oracle(qf, seed):
    """Three-run apply passes (2^12 sub-cubes, forward and inverse) and
    two-run reverse-sweep passes (2^11 sub-cubes) against the oracle, on runs
    built to form them, mixed with runs that break them."""
    n = 14
    xs, zs = multi_run_terms(n, seed)
    th = qi.random_angles(len(xs), 140 + seed, 1.0)
    psi0 = qi.random_state(n, 150 + seed)
    hx, hz, hc = qi.random_paulis(n, 200, 160 + seed)
    hx, hz, hc, off = grouped(hx, hz, hc)
    A = qf.terms_array(xs, zs, np.ones(len(xs)))
    plan = qf.Plan(n, A, qf.terms_array(hx, hz, hc), off)
    plan.set_block_bits(12)
    for inverse in (False, True):
        psi = dev(psi0)
        qf.apply_pauli_exp(psi, n, A, th, inverse=inverse)
        want = sv.apply_product(psi0, n, xs, zs, th, inverse=inverse)
        assert np.max(np.abs(host(psi) - want)) < A_TOL
    occ = (1 << 7) - 1
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    e_o, g_o = core.energy_grad(n, occ, xs, zs, th, hx, hz, hc)
    for B in (12, 11):
        plan.set_block_bits(B)
        e, g = plan.energy_grad(occ, th, ws)
        assert e == pytest.approx(e_o, abs=E_TOL)
        assert np.max(np.abs(g - g_o)) < G_TOL


@pytest.mark.parametrize("B", [10, 11])
def test_blocked_adjoint_20q_matches_golden(qf, B):
    """20 qubits: more sub-cubes than resident workgroups at B = 10, so
    workgroups loop over several sub-cubes; gradient against the oracle run."""
    gold = _golden("20q")
    w, n, occ, H, off, A, aoff, th = _build_device_system(qf, "20q")
    plan = qf.Plan(n, A, H, off)
    plan.set_block_bits(B)
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    e_g, g = plan.energy_grad(occ, th, ws)
    assert e_g == pytest.approx(gold["energy"], abs=E_TOL)
    assert np.max(np.abs(g - np.array(gold["grad_theta"]))) < G_TOL
    e2, g2 = plan.energy_grad(occ, th, ws)
    assert e2 == e_g and np.array_equal(g2, g)


@pytest.mark.parametrize("n", [12, 14])
def test_sigma_shared_pattern_groups_match_oracle(qf, n):
    """Groups of several strings whose z bits 9 and 10 agree within each
    phase part (the summed form of the class-tiled sigma), with real- and
    imaginary-phase parts of different patterns, beside groups whose parts
    mix patterns (per-string signs)."""
    rng = np.random.default_rng([n, 97])
    xs, zs = [], []
    for g in range(60):
        x = int(rng.integers(1, 1 << n))
        shared = g % 2 == 0
        pat = {0: int(rng.integers(0, 4)), 1: int(rng.integers(0, 4))}  # per phase parity
        for _ in range(int(rng.integers(3, 9))):
            z = int(rng.integers(0, 1 << n))
            if shared:
                ph = bin(x & z).count("1") & 1
                z = (z & ~(3 << 9)) | (pat[ph] << 9)
                if bin(x & z).count("1") & 1 != ph:  # bits 9, 10 of x changed the phase: flip a free z bit
                    free = [q for q in range(n) if q not in (9, 10) and (x >> q) & 1]
                    if not free:
                        continue
                    z ^= 1 << free[0]
            xs.append(x)
            zs.append(z)
    xs, zs = np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64)
    cs = rng.normal(size=len(xs))
    xs, zs, cs, off = grouped(xs, zs, cs)
    psi0 = qi.random_state(n, 98 + n)
    plan = qf.Plan(n, None, qf.terms_array(xs, zs, cs), off)
    lam = torch.empty_like(dev(psi0))
    e = plan.sigma(dev(psi0), lam)
    want = core.sigma(psi0, n, xs, zs, cs)
    assert np.max(np.abs(host(lam) - want)) < 1e-11
    assert e == pytest.approx(core.energy(psi0, n, xs, zs, cs, off), abs=E_TOL)


@pytest.mark.parametrize("n", [13, 16])
def test_sigma_merged_lo_terms_and_split_windows_match_oracle(qf, n):
    """Sigma with strings merged per output tile: many strings of one group
    part sharing their low 11 z bits (runs longer than one lo-term holds),
    a diagonal group with more lo-terms than one window and one wave hold
    (the group is cut), a class of more than 256 groups (the class is cut
    into several windows over the same partner tile), and imaginary-phase
    parts."""
    rng = np.random.default_rng([n, 131])
    xs, zs = [], []
    # 800 diagonal strings over 40 distinct low parts: long equal-z_lo runs
    lows = rng.integers(0, 1 << 11, 40)
    for k in range(800):
        xs.append(0)
        zs.append(int(lows[k % 40]) | (int(rng.integers(0, 1 << (n - 11))) << 11))
    # 330 groups with flips below bit 11 (all in the class of the own tile),
    # each with a few strings sharing z_lo
    for x in rng.choice(np.arange(1, 1 << 11), 330, replace=False):
        zl = int(rng.integers(0, 1 << 11))
        for _ in range(int(rng.integers(1, 6))):
            xs.append(int(x))
            zs.append(zl | (int(rng.integers(0, 1 << (n - 11))) << 11))
    # groups with high flips and mixed parts
    for _ in range(40):
        x = int(rng.integers(1 << 11, 1 << n))
        for _ in range(int(rng.integers(2, 12))):
            xs.append(x)
            zs.append(int(rng.integers(0, 1 << n)))
    xs, zs = np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64)
    cs = rng.normal(size=len(xs))
    xs, zs, cs, off = grouped(xs, zs, cs)
    psi0 = qi.random_state(n, 140 + n)
    plan = qf.Plan(n, None, qf.terms_array(xs, zs, cs), off)
    lam = torch.empty_like(dev(psi0))
    e = plan.sigma(dev(psi0), lam)
    want = core.sigma(psi0, n, xs, zs, cs)
    assert np.max(np.abs(host(lam) - want)) < 1e-11
    assert e == pytest.approx(core.energy(psi0, n, xs, zs, cs, off), abs=E_TOL)


# ------------------------------------ largest batched and served instances

def _mix_instance(qf, gold):
    r = gold["recipe"]
    h, g = qi.integrals(r["n_orb"], r["n_elec"], r["seed"])
    H, off, _ = qf.build_paulis("hamiltonian", r["n_orb"], r["n_elec"], h, g)
    A, aoff, _ = qf.build_paulis("uccsd", r["n_orb"], r["n_elec"])
    th = qf.ansatz_angles(A, aoff, qi.amplitudes(len(aoff) - 1, r["seed"], r["t_scale"]))
    assert (len(H), len(off) - 1, len(A)) == (gold["n_strings"], gold["n_groups"], gold["K"])
    return dict(n=2 * r["n_orb"], occ=(1 << r["n_elec"]) - 1, H=H, off=off, A=A, aoff=aoff, theta=th)


def _check_gold(qf, gold, d, e, g):
    assert e == pytest.approx(gold["energy"], abs=E_TOL)
    assert np.max(np.abs(g - np.array(gold["grad_theta"]))) < G_TOL
    assert np.max(np.abs(qf.grad_t(d["A"], d["aoff"], g) - np.array(gold["grad_t"]))) < G_TOL


def test_batch22q_instance_vs_oracle_golden(qf):
    """The first 22-qubit instance of the 256-instance batched recipe: plan
    path, the batched kernel alone with its tuned team, and the batched kernel
    inside a mix, each against the oracle's energy and full gradient."""
    gold = _golden("batch22q")
    d = _mix_instance(qf, gold)
    n = d["n"]
    plan = qf.Plan(n, d["A"], d["H"], d["off"])
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    e, g = plan.energy_grad(d["occ"], d["theta"], ws)
    _check_gold(qf, gold, d, e, g)
    psi = ws[: 1 << n]
    qf.prepare_state(psi, n, d["occ"])
    plan.apply(psi, d["theta"])
    idx = np.array(gold["sample_index"])
    want = np.array(gold["sample_re"]) + 1j * np.array(gold["sample_im"])
    assert np.max(np.abs(host(psi)[idx] - want)) < A_TOL
    plan.close()
    del ws, psi
    B = qf.Batch([d])
    print("tuned team at 22 qubits:", B.info()["team"], flush=True)
    E, G = B.run([d["theta"]], use_graph=False)
    _check_gold(qf, gold, d, E[0], G[0])
    B.close()
    small = []
    for s in (2101, 2102, 2103):
        h, gg = qi.integrals(6, 6, s)
        H, off, _ = qf.build_paulis("hamiltonian", 6, 6, h, gg)
        A, aoff, _ = qf.build_paulis("uccsd", 6, 6)
        small.append(dict(n=12, occ=63, H=H, off=off, A=A, aoff=aoff,
                          theta=qf.ansatz_angles(A, aoff, qi.amplitudes(len(aoff) - 1, s, 0.2))))
    B = qf.Batch(small[:2] + [d] + small[2:])
    E, G = B.run([x["theta"] for x in small[:2]] + [d["theta"]] + [small[2]["theta"]], use_graph=True)
    _check_gold(qf, gold, d, E[2], G[2])
    B.close()
    torch.cuda.empty_cache()


def test_serve24q_request_vs_oracle_golden(qf):
    """The first 24-qubit request of the serving trace (the solo lane's
    kernels: an arena plan) against the oracle's energy and full gradient."""
    gold = _golden("serve24q")
    d = _mix_instance(qf, gold)
    n = d["n"]
    need = qf.Plan.arena_bytes(n, d["A"], d["H"], d["off"])
    buf = torch.empty(need + (2 << n) * 16 + 512, dtype=torch.uint8, device="cuda")
    base = (buf.data_ptr() + 255) // 256 * 256
    plan = qf.Plan(n, d["A"], d["H"], d["off"], arena=(base, need))

    class _At:
        def data_ptr(self):
            return (base + need + 255) // 256 * 256

    e, g = plan.energy_grad(d["occ"], d["theta"], _At())
    _check_gold(qf, gold, d, e, g)
    plan.close()
    del buf
    torch.cuda.empty_cache()
