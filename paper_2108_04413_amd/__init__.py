"""MI355X-native Pauli-exponential state-vector path (QForte hot path).

Importing this package loads libqforte_mi355x.so and fails loudly if it has
not been built; there is no CPU fallback.
"""
from ._lib import TERM_DTYPE, QFError, lib, terms_array  # noqa: F401
from .api import (Batch, Plan, PoolPlan, Sector, ansatz_angles, apply_pauli_exp, build_paulis, energy,  # noqa: F401
                  energy_grad, energy_static, excitations, excited_determinants, grad_t, mp_denominators, pool_grad,
                  pqe_residuals, prepare_state)

__version__ = lib.qf_version().decode()
from .autograd import UCCEnergy  # noqa: E402,F401
