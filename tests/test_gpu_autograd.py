"""torch.autograd wrapper: backward equals central finite differences and
the parameter-shift rule (both computed from device energies), and the
oracle's adjoint gradient."""
import math

import numpy as np
import pytest

import qf_inputs as qi
from oracle import core

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available()
    import paper_2108_04413_amd as qf
    h, g = qi.integrals(5, 4, 61)
    H, off, _ = qf.build_paulis("hamiltonian", 5, 4, h, g)
    A, aoff, _ = qf.build_paulis("uccsd", 5, 4)
    t0 = qi.amplitudes(len(aoff) - 1, 61, 0.3)
    return qf, qf.UCCEnergy(10, 0b1111, A, aoff, H, off), A, aoff, H, off, t0


def energy_at(qf, mod, t):
    theta = qf.ansatz_angles(mod.A, mod.aoff, t)
    psi = torch.empty(1 << mod.n, dtype=torch.complex128, device="cuda")
    qf.prepare_state(psi, mod.n, mod.occ)
    mod.plan.apply(psi, theta)
    return mod.plan.energy(psi)


def test_backward_matches_fd_and_oracle(setup):
    qf, mod, A, aoff, H, off, t0 = setup
    t = torch.tensor(t0, dtype=torch.float64, device="cuda", requires_grad=True)
    e = mod(t)
    e.backward()
    g = t.grad.cpu().numpy()
    theta = qf.ansatz_angles(A, aoff, t0)
    e_o, g_o = core.energy_grad(10, 0b1111, A["x"], A["z"], theta, H["x"], H["z"], H["c"])
    assert float(e.detach()) == pytest.approx(e_o, abs=1e-10)
    assert np.max(np.abs(g - qf.grad_t(A, aoff, g_o))) < 1e-9
    hstep = 1e-5
    for mu in (0, 7, mod.n_par - 1):
        tp, tm = t0.copy(), t0.copy()
        tp[mu] += hstep
        tm[mu] -= hstep
        fd = (energy_at(qf, mod, tp) - energy_at(qf, mod, tm)) / (2 * hstep)
        assert fd == pytest.approx(g[mu], abs=1e-7)


def test_dtheta_matches_parameter_shift(setup):
    qf, mod, A, aoff, H, off, t0 = setup
    t = torch.tensor(t0, dtype=torch.float64, device="cuda", requires_grad=True)
    mod(t).backward()
    gth = mod.last_grad_theta
    theta = qf.ansatz_angles(A, aoff, t0)
    for k in (0, 3, len(theta) // 2, len(theta) - 1):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += math.pi / 4
        tm[k] -= math.pi / 4
        e = []
        for th in (tp, tm):
            psi = torch.empty(1 << 10, dtype=torch.complex128, device="cuda")
            qf.prepare_state(psi, 10, 0b1111)
            mod.plan.apply(psi, th)
            e.append(mod.plan.energy(psi))
        assert e[0] - e[1] == pytest.approx(gth[k], abs=1e-9)


def test_optimizer_step_lowers_energy(setup):
    qf, mod, A, aoff, H, off, t0 = setup
    t = torch.zeros(mod.n_par, dtype=torch.float64, device="cuda", requires_grad=True)
    opt = torch.optim.SGD([t], lr=0.05)
    e_prev = None
    for _ in range(5):
        opt.zero_grad()
        e = mod(t)
        e.backward()
        opt.step()
        if e_prev is not None:
            assert float(e) <= e_prev + 1e-12
        e_prev = float(e)
