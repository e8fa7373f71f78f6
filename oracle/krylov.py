"""Quantum Krylov (QK) basis from Trotterized real-time evolution (Sec. 3.7).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. (m_trotter_step2): with H = sum_l h_l P_l,
    exp(-i t H) ~ ( prod_l exp(-i t h_l P_l / r) )^r,
the product taken over the strings in the order given (the first string acts
first), r Trotter steps.  The QK basis (Eq. (wfnqk)) is
    psi_n = exp(-i t_n H) Phi,  t_n = n dt,  n = 0 .. s,
each state evolved from Phi with r steps of t_n / r (the reading of the
paper's formula with t = t_n), and the matrices of the generalized
eigenproblem H c = S c E are S_mn = <psi_m|psi_n>, H_mn = <psi_m|H|psi_n>.
"""
from __future__ import annotations

import numpy as np

from . import statevec as sv


def trotter(psi, n, hx, hz, hc, t, r):
    """(prod_l exp(-i t h_l P_l / r))^r psi (numpy)."""
    th = np.asarray(hc, dtype=np.float64) * (t / r)
    for _ in range(r):
        psi = sv.apply_product(psi, n, hx, hz, th)
    return psi


def trotter_core(psi, n, hx, hz, hc, t, r):
    """The same with the C core's loops (in place on psi, returned)."""
    from . import core
    th = np.asarray(hc, dtype=np.float64) * (t / r)
    for _ in range(r):
        core.apply_product(psi, n, hx, hz, th)
    return psi


def qk_matrices(n, occ, hx, hz, hc, dt, s, r, use_core=False):
    """(S, Hm): (s+1) x (s+1) complex overlap and Hamiltonian matrices."""
    from . import core
    states = []
    for k in range(s + 1):
        phi = sv.prepare(n, occ)
        states.append(trotter_core(phi, n, hx, hz, hc, k * dt, r) if use_core
                      else trotter(phi, n, hx, hz, hc, k * dt, r))
    sig = [core.sigma(p, n, hx, hz, hc) if use_core else sv.sigma(p, n, hx, hz, hc) for p in states]
    S = np.zeros((s + 1, s + 1), dtype=np.complex128)
    Hm = np.zeros_like(S)
    for m in range(s + 1):
        for k in range(s + 1):
            if use_core:
                S[m, k] = core.vdot(states[m], states[k], n)
                Hm[m, k] = core.vdot(states[m], sig[k], n)
            else:
                S[m, k] = np.vdot(states[m], states[k])
                Hm[m, k] = np.vdot(states[m], sig[k])
    return S, Hm


def qk_energy(S, Hm, thresh=1e-10):
    """Lowest root of H c = S c E after dropping the directions of S with
    eigenvalue below thresh (canonical orthogonalization)."""
    w, V = np.linalg.eigh(S)
    keep = w > thresh * w.max()
    X = V[:, keep] / np.sqrt(w[keep])
    Hp = X.conj().T @ Hm @ X
    return float(np.linalg.eigvalsh(0.5 * (Hp + Hp.conj().T))[0])
