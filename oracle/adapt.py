"""ADAPT-VQE operator pool and its energy gradients (Sec. 3.2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The pool is built from generalized single and double excitations: no
occupied/virtual split, every spin orbital may be created or annihilated.
Readings (the paper points to the original ADAPT publication for the pool
and gives no index rules):

* spin-orbital operators that conserve S_z, one parameter each (as for the
  dUCC ansatz of Sec. 3.1);
* singles tau = a+_p a_q with p > q of equal spin;
* doubles tau = a+_p a+_q a_s a_r with p < q, r < s, (p, q) > (r, s) in
  lexicographic order and spin(p) + spin(q) = spin(r) + spin(s); index sets
  may overlap (p = r gives a density-weighted single), each unordered pair of
  distinct index pairs appears once;
* order: singles by (q, p), then doubles by ((r, s), (p, q)), ascending;
* kappa_nu = tau_nu - tau_nu^dagger, JW(kappa_nu) = i sum_k c_k P_k.

The gradient of the energy with respect to the parameter of kappa_nu
appended at the end of the ansatz, at zero, is
    g_nu = <Psi|[H, kappa_nu]|Psi> = 2 Re <H Psi|kappa_nu Psi>,
because kappa_nu is anti-Hermitian and H Hermitian.  With the strings,
<H Psi|kappa_nu Psi> = i sum_k c_k <H Psi|P_k Psi>, so
    g_nu = -2 sum_k c_k Im <H Psi|P_k|Psi>.
"""
from __future__ import annotations

import numpy as np

from . import statevec as sv
from .ansatz import ansatz_terms


def gsd_pool(n_qubits: int):
    """Generalized singles and doubles as (creators, annihilators) pairs,
    tau = a+_{c1} [a+_{c2}] [a_{a1}] a_{a2} in the order written."""
    N = n_qubits
    out = []
    for q in range(N):
        for p in range(q + 1, N):
            if (p & 1) == (q & 1):
                out.append(((p,), (q,)))
    pairs = [(a, b) for a in range(N) for b in range(a + 1, N)]
    for (r, s) in pairs:
        for (p, q) in pairs:
            if (p, q) > (r, s) and (p & 1) + (q & 1) == (r & 1) + (s & 1):
                out.append(((p, q), (s, r)))
    return out


def pool_terms(n_qubits: int):
    """(ops, x, z, c, off): the pool and the JW strings of each kappa_nu."""
    ops = gsd_pool(n_qubits)
    x, z, c, off = ansatz_terms(ops)
    return ops, x, z, c, off


def pool_gradients(psi, n, px, pz, pc, poff, hx, hz, hc):
    """g_nu = 2 Re <H psi|kappa_nu psi> for every pool member (numpy, small n)."""
    lam = sv.sigma(psi, n, hx, hz, hc)
    g = np.zeros(len(poff) - 1)
    for nu in range(len(poff) - 1):
        kpsi = np.zeros_like(psi)
        for k in range(poff[nu], poff[nu + 1]):
            kpsi += 1j * float(pc[k]) * sv.apply_pauli(psi, n, int(px[k]), int(pz[k]))
        g[nu] = 2.0 * np.vdot(lam, kpsi).real
    return g
