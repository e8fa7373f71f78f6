"""Particle-number / S_z restricted state vector on the GPU against the
oracle: the sector ansatz state equals the restriction of the full-space
oracle state (amplitudes 1e-12), energies within 1e-10 of the oracle's,
including the 20- and 28-qubit workloads' stored oracle values."""
import json
import os

import numpy as np
import pytest

import qf_inputs as qi
from oracle import ansatz as an, core, hamiltonian as ham, sector

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def qf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2108_04413_amd as qf
    return qf


def _sector(qf, n_orb, n_elec, h, g, kind="uccsd", t_rank=None, top_k=0):
    na, nb = (n_elec + 1) // 2, n_elec // 2
    H, off, _ = qf.build_paulis("hamiltonian", n_orb, n_elec, h, g)
    ops = qf.excitations(kind, n_orb, n_elec, t_rank=t_rank, top_k=top_k)
    return qf.Sector(n_orb, na, nb, ops, H, off), na, nb


@pytest.mark.parametrize("n_orb,n_elec,seed,scale", [(4, 4, 1008, 0.3), (5, 3, 1101, 0.3), (6, 6, 1102, 0.2),
                                                     (7, 7, 1103, 0.2)])
def test_sector_state_and_energy_match_full_space_oracle(qf, n_orb, n_elec, seed, scale):
    n = 2 * n_orb
    h, g = qi.integrals(n_orb, n_elec, seed)
    S, na, nb = _sector(qf, n_orb, n_elec, h, g)
    excs, ax, az, ac, aoff, _ = an.build(n_orb, n_elec)
    t = qi.amplitudes(len(excs), seed, scale)
    occ = an.reference_mask(n_elec)
    psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
    S.prepare(psi, occ)
    S.apply(psi, t)
    got = psi.cpu().numpy()
    full = core.apply_product(core.prepare(n, occ), n, ax, az, an.angles(ac, aoff, t))
    want = sector.restrict(full, n_orb, na, nb)
    assert float(np.max(np.abs(got - want))) < 1e-12
    hx, hz, hc, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    e = S.energy(psi)
    assert e == pytest.approx(core.energy(full, n, hx, hz, hc, goff), abs=1e-10)
    if n <= 10:
        assert e == pytest.approx(sector.energy(want, n_orb, na, nb, hx, hz, hc, goff), abs=1e-10)
    # the adjoint restores the reference
    S.apply(psi, t, inverse=True)
    back = psi.cpu().numpy()
    ref = sector.prepare(n_orb, na, nb, occ)
    assert float(np.max(np.abs(back - ref))) < 1e-12


def _gold(name):
    path = os.path.join(GOLD, f"oracle_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


def test_sector_20q_matches_golden(qf):
    gold = _gold("20q")
    w, h, g = qi.workload("20q")
    S, na, nb = _sector(qf, 10, 10, h, g)
    t = qi.amplitudes(len(qf.excitations("uccsd", 10, 10)), w["seed"], w["t_scale"])
    psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
    S.prepare(psi, (1 << 10) - 1)
    S.apply(psi, t)
    assert S.energy(psi) == pytest.approx(gold["energy"], abs=1e-10)
    dets = sector.determinants(10, na, nb)
    where = {int(d): i for i, d in enumerate(dets)}
    got = psi.cpu().numpy()
    for idx, re, im in zip(gold["sample_index"], gold["sample_re"], gold["sample_im"]):
        j = where.get(int(idx))
        want = complex(re, im)
        if j is None:
            assert abs(want) < 1e-12  # the full-space state has nothing outside the sector
        else:
            assert abs(got[j] - want) < 1e-12


def test_sector_28q_matches_golden(qf):
    gold = _gold("28q")
    w, h, g = qi.workload("28q")
    n_d = len(qf.excitations("uccd", 14, 14))
    t_all = qi.amplitudes(n_d, w["seed"], w["t_scale"])
    S, na, nb = _sector(qf, 14, 14, h, g, kind="uccd_top", t_rank=t_all, top_k=w["top_k"])
    _, _, kept = qf.build_paulis("uccd_top", 14, 14, t_rank=t_all, top_k=w["top_k"])
    psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
    S.prepare(psi, (1 << 14) - 1)
    S.apply(psi, t_all[kept])
    print(f"28q sector: dim {S.dim} ({S.dim * 16 / 2**20:.0f} MiB), {S.groups} groups", flush=True)
    assert S.energy(psi) == pytest.approx(gold["energy"], abs=1e-10)
    del psi
    torch.cuda.empty_cache()


def test_sector_24q_matches_served_request_golden(qf):
    gold = _gold("serve24q")
    r = gold["recipe"]
    h, g = qi.integrals(r["n_orb"], r["n_elec"], r["seed"])
    S, na, nb = _sector(qf, r["n_orb"], r["n_elec"], h, g)
    t = qi.amplitudes(len(qf.excitations("uccsd", r["n_orb"], r["n_elec"])), r["seed"], r["t_scale"])
    psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
    S.prepare(psi, (1 << r["n_elec"]) - 1)
    S.apply(psi, t)
    assert S.energy(psi) == pytest.approx(gold["energy"], abs=1e-10)


def test_sector_32q_reference_energy_closed_form(qf):
    # 16 orbitals, 16 electrons: 165,636,900 determinants (2.5 GiB) instead of
    # 2^32 amplitudes (64 GiB); theta = 0 leaves the reference, whose energy
    # is the closed-form Hartree-Fock value
    h, g = qi.integrals(16, 16, 1132)
    S, na, nb = _sector(qf, 16, 16, h, g)
    assert S.dim == 12870 * 12870
    psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
    S.prepare(psi, (1 << 16) - 1)
    e_cf = 2 * sum(h[i, i] for i in range(8)) + sum(2 * g[i, i, j, j] - g[i, j, j, i]
                                                    for i in range(8) for j in range(8))
    assert S.energy(psi) == pytest.approx(e_cf, abs=1e-10)
    del psi
    torch.cuda.empty_cache()


def test_sector_rejects_bad_inputs(qf):
    h, g = qi.integrals(3, 2, 5)
    H, off, _ = qf.build_paulis("hamiltonian", 3, 2, h, g)
    with pytest.raises(qf.QFError):  # changes N_alpha
        qf.Sector(3, 1, 1, np.array([[2, -1, 1, -1]], dtype=np.int32), H, off)
    S = qf.Sector(3, 1, 1, None, H, off)
    psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
    with pytest.raises(qf.QFError):  # reference outside the sector
        S.prepare(psi, 0b1111)


@pytest.mark.parametrize("n_orb,n_elec,seed,scale", [(4, 4, 1008, 0.3), (5, 3, 1111, 0.3), (7, 7, 1113, 0.2)])
def test_sector_energy_grad_matches_full_space_oracle(qf, n_orb, n_elec, seed, scale):
    """dE/dt_mu from the sector's reverse sweep equals the chain rule of the
    full-space oracle's adjoint gradient, dE/dt = -sum_k c_k dE/dtheta_k."""
    n = 2 * n_orb
    h, g = qi.integrals(n_orb, n_elec, seed)
    S, na, nb = _sector(qf, n_orb, n_elec, h, g)
    excs, ax, az, ac, aoff, _ = an.build(n_orb, n_elec)
    t = qi.amplitudes(len(excs), seed, scale)
    occ = an.reference_mask(n_elec)
    e, gt = S.energy_grad(occ, t)
    hx, hz, hc, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    e_o, gth = core.energy_grad(n, occ, ax, az, an.angles(ac, aoff, t), hx, hz, hc)
    assert e == pytest.approx(e_o, abs=1e-10)
    assert float(np.max(np.abs(gt - an.grad_t(ac, aoff, gth)))) < 1e-9
    assert float(np.max(np.abs(gt))) > 1e-3
    e2, gt2 = S.energy_grad(occ, t)  # repeatable bit for bit
    assert e2 == e and bool(np.array_equal(gt2, gt))


@pytest.mark.parametrize("name", ["20q", "batch22q", "serve24q"])
def test_sector_energy_grad_matches_stored_oracle_gradients(qf, name):
    gold = _gold(name)
    if name == "20q":
        r = dict(n_orb=10, n_elec=10, seed=1020, t_scale=0.1)
    else:
        r = gold["recipe"]
    h, g = qi.integrals(r["n_orb"], r["n_elec"], r["seed"])
    S, na, nb = _sector(qf, r["n_orb"], r["n_elec"], h, g)
    t = qi.amplitudes(len(qf.excitations("uccsd", r["n_orb"], r["n_elec"])), r["seed"], r["t_scale"])
    e, gt = S.energy_grad((1 << r["n_elec"]) - 1, t)
    print(f"{name}: sector dim {S.dim}, {len(gt)} excitations", flush=True)
    assert e == pytest.approx(gold["energy"], abs=1e-10)
    assert float(np.max(np.abs(gt - np.array(gold["grad_t"])))) < 1e-9
