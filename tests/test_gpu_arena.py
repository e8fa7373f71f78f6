"""Plans whose device tables live in a caller's arena (qf_plan_create_arena):
the same results as a library-allocated plan, bit for bit, and the size and
argument rules of the call."""
import numpy as np
import pytest

import qf_inputs as qi
from oracle import ansatz as an, core, hamiltonian as ham

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def qf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2108_04413_amd as qf
    return qf


def _instance(qf, n_orb, n_elec, seed, scale=0.1):
    h, g = qi.integrals(n_orb, n_elec, seed)
    H, off, _ = qf.build_paulis("hamiltonian", n_orb, n_elec, h, g)
    A, aoff, _ = qf.build_paulis("uccsd", n_orb, n_elec)
    th = qf.ansatz_angles(A, aoff, qi.amplitudes(len(aoff) - 1, seed, scale))
    return 2 * n_orb, (1 << n_elec) - 1, H, off, A, aoff, th, h, g


@pytest.mark.parametrize("n_orb,n_elec,seed", [(5, 4, 811), (7, 7, 812), (9, 9, 813)])
def test_arena_plan_equals_owned_plan(qf, n_orb, n_elec, seed):
    n, occ, H, off, A, aoff, th, _, _ = _instance(qf, n_orb, n_elec, seed)
    need = qf.Plan.arena_bytes(n, A, H, off)
    # tables placed after an unaligned-looking offset of the buffer: the call
    # gets a 256-byte aligned address inside it
    buf = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
    base = (buf.data_ptr() + 255) // 256 * 256 + 512
    stream = torch.cuda.current_stream()
    pa = qf.Plan(n, A, H, off, arena=(base, need), stream=stream)
    po = qf.Plan(n, A, H, off)
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    ea, ga = pa.energy_grad(occ, th, ws)
    eo, go = po.energy_grad(occ, th, ws)
    assert ea == eo and np.array_equal(ga, go)
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, n, occ)
    pa.apply(psi, th)
    ea2 = pa.energy(psi)
    qf.prepare_state(psi, n, occ)
    po.apply(psi, th)
    assert ea2 == po.energy(psi) and ea2 == pytest.approx(eo, abs=1e-12)
    assert pa.info() == po.info() and pa.apply_info() == po.apply_info()
    with pytest.raises(qf.QFError, match="arena plan"):
        pa.set_block_bits(10)
    with pytest.raises(qf.QFError, match="arena plan"):
        pa.set_energy_tile(10)
    pa.close()
    po.close()


def test_arena_plan_matches_oracle_and_rejects_small_arena(qf):
    n, occ, H, off, A, aoff, th, h, g = _instance(qf, 6, 6, 821)
    need = qf.Plan.arena_bytes(n, A, H, off)
    buf = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    base = (buf.data_ptr() + 255) // 256 * 256
    with pytest.raises(qf.QFError) as ei:
        qf.Plan(n, A, H, off, arena=(base, need - 256))
    assert ei.value.status == -5  # QF_E_SIZE
    with pytest.raises(qf.QFError) as ei:
        qf.Plan(n, A, H, off, arena=(base + 8, need))
    assert ei.value.status == -1  # QF_E_ARG: not 256-byte aligned
    p = qf.Plan(n, A, H, off, arena=(base, need))
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    e, gr = p.energy_grad(occ, th, ws)
    x, z, c, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    _, ax, az, ac, oaoff, _ = an.build(6, 6)
    e_o, g_o = core.energy_grad(n, occ, ax, az, an.angles(ac, oaoff, qi.amplitudes(len(oaoff) - 1, 821, 0.1)),
                                x, z, c)
    assert e == pytest.approx(e_o, abs=1e-10)
    assert np.max(np.abs(gr - g_o)) < 1e-9
