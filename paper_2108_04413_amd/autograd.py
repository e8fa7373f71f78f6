"""torch.autograd face of the energy + adjoint-gradient call.

UCCEnergy(system)(t) returns E(t) = <Phi_0|U(t)^dagger H U(t)|Phi_0> for the
dUCC ansatz U(t) = prod_mu exp(t_mu kappa_mu) (Sec. 3.1, Eqs. (16)-(18)) as
a 0-dim float64 tensor; backward returns dE/dt from the same device call
(qf_plan_energy_grad: one forward sweep, sigma = H psi, one reverse sweep).
The adjoint gradient is computed with the energy in forward and kept for
backward, so one optimizer step costs one call.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


class _EnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, t, module):
        tt = t.detach().to("cpu", torch.float64).numpy()
        theta = api.ansatz_angles(module.A, module.aoff, tt)
        e, g_theta = module.plan.energy_grad(module.occ, theta, module.workspace)
        g_t = api.grad_t(module.A, module.aoff, g_theta)
        ctx.save_for_backward(torch.from_numpy(g_t).to(t.device, t.dtype))
        module.last_grad_theta = g_theta
        return torch.tensor(e, dtype=t.dtype, device=t.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None


class UCCEnergy(torch.nn.Module):
    """Energy of a dUCC state as a differentiable function of the amplitudes t.

    n_qubits, occ_mask: register size and reference determinant;
    A, aoff: ansatz strings and excitation offsets (qf_build_paulis);
    H, off: grouped Hamiltonian.  The plan and a two-state workspace stay
    on the device for the module's lifetime.
    """

    def __init__(self, n_qubits: int, occ_mask: int, A: np.ndarray, aoff: np.ndarray, H: np.ndarray,
                 off: np.ndarray):
        super().__init__()
        self.n = n_qubits
        self.occ = occ_mask
        self.A = A
        self.aoff = np.ascontiguousarray(aoff, dtype=np.int64)
        self.plan = api.Plan(n_qubits, A, H, off)
        self.workspace = torch.empty(2 << n_qubits, dtype=torch.complex128, device="cuda")
        self.last_grad_theta = None

    @property
    def n_par(self) -> int:
        return len(self.aoff) - 1

    def forward(self, t: torch.Tensor) -> torch.Tensor:
        return _EnergyFn.apply(t, self)
