"""Projective quantum eigensolver (PQE) residuals and update (Sec. 3.3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For the dUCC state U(t)|Phi_0> (Sec. 3.1), the residual of excitation mu
(Eq. (ucc2)) is
    r_mu = <Phi_mu| U^dagger H U |Phi_0>,   Phi_mu = tau_mu Phi_0.
Two ways are written out here:

* direct: lambda = H U Phi_0, then U^dagger lambda (the ansatz undone in
  reverse), then the amplitude at the excited determinant: with
  tau_mu Phi_0 = s_mu |d_mu> (s_mu = +-1 the fermionic sign of the
  excitation acting on the reference bit string),
      r_mu = s_mu [U^dagger H U Phi_0](d_mu);
* three energies (the measurement form of Sec. 3.3):
      r_mu = E(Omega_mu) - E(Phi_0)/2 - E(Phi_mu)/2,
      Omega_mu = exp(pi/4 kappa_mu) Phi_0 = (Phi_0 + Phi_mu)/sqrt(2),
  with E(chi) = <chi|U^dagger H U|chi>.

Update (Eq. (fixed_point)): t_mu <- t_mu + r_mu / Delta_mu with the
Moller-Plesset denominators Delta_mu = sum eps_occ - sum eps_vir.  Reading:
the random integrals have no canonical orbitals, so eps_p is the diagonal of
the Fock matrix of the reference, eps_p = h_pp + sum_{j occ} <pj||pj>
(spin orbitals), the usual choice for non-canonical references.
"""
from __future__ import annotations

import math

import numpy as np

from . import statevec as sv
from .hamiltonian import spin_orbital_integrals


def excitation_sign(occ: int, creators, annihilators):
    """(s, d) with tau |occ> = s |d> for tau = a+_{c1} .. a_{a1} .. applied
    right to left, each ladder operator picking up (-1)^(occupied below)."""
    b = occ
    s = 1
    for p, dag in [(p, False) for p in reversed(annihilators)] + [(p, True) for p in reversed(creators)]:
        bit = (b >> p) & 1
        if bit == int(dag):
            return 0, None
        if bin(b & ((1 << p) - 1)).count("1") & 1:
            s = -s
        b ^= 1 << p
    return s, b


def residuals(n, occ, ax, az, th, hx, hz, hc, excs):
    """(E, r) by the direct form; excs as (creators, annihilators) per mu."""
    psi = sv.apply_product(sv.prepare(n, occ), n, ax, az, th)
    lam = sv.sigma(psi, n, hx, hz, hc)
    e = float(np.vdot(psi, lam).real)
    back = sv.apply_product(lam, n, ax, az, th, inverse=True)
    r = np.zeros(len(excs))
    for mu, (cre, ann) in enumerate(excs):
        s, d = excitation_sign(occ, cre, ann)
        r[mu] = s * back[d].real
    return e, r


def residuals_core(n, occ, ax, az, th, hx, hz, hc, excs):
    """(E, r) by the direct form with the C core's loops (20+ qubits)."""
    from . import core
    psi = core.apply_product(core.prepare(n, occ), n, ax, az, th)
    lam = core.sigma(psi, n, hx, hz, hc)
    e = core.vdot(psi, lam, n).real
    back = core.apply_product(lam, n, ax, az, th, inverse=True)
    r = np.zeros(len(excs))
    for mu, (cre, ann) in enumerate(excs):
        s, d = excitation_sign(occ, cre, ann)
        r[mu] = s * back[d].real
    return e, r


def residuals_three_energies(n, occ, ax, az, th, hx, hz, hc, excs):
    """r by the symmetric expectation values of Sec. 3.3 (three energies per mu)."""
    def e_of(chi):
        v = sv.apply_product(chi, n, ax, az, th)
        return sv.energy(v, n, hx, hz, hc)

    phi0 = sv.prepare(n, occ)
    e0 = e_of(phi0)
    r = np.zeros(len(excs))
    for mu, (cre, ann) in enumerate(excs):
        s, d = excitation_sign(occ, cre, ann)
        phimu = np.zeros(1 << n, dtype=np.complex128)
        phimu[d] = s
        omega = (phi0 + phimu) / math.sqrt(2.0)
        r[mu] = e_of(omega) - 0.5 * e0 - 0.5 * e_of(phimu)
    return r


def fock_diagonal(h: np.ndarray, g: np.ndarray, n_elec: int) -> np.ndarray:
    """eps_p = h_pp + sum_{j < n_elec} <pj||pj> over spin orbitals."""
    h_so, v = spin_orbital_integrals(h, g)
    N = h_so.shape[0]
    return np.array([h_so[p, p] + sum(v[p, j, p, j] for j in range(n_elec)) for p in range(N)])


def mp_denominators(eps: np.ndarray, excs) -> np.ndarray:
    """Delta_mu = sum of eps over the annihilated (occupied) minus the created."""
    return np.array([sum(eps[i] for i in ann) - sum(eps[a] for a in cre) for cre, ann in excs])


def update(t: np.ndarray, r: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """t_mu + r_mu / Delta_mu (Eq. (fixed_point))."""
    return t + r / delta
