"""Molecular Hamiltonian -> Jordan-Wigner qubit Hamiltonian, grouped by flip mask.

The paper's Hamiltonian (Sec. 1, Eq. (1)):
    H = sum_pq h_pq a^dagger_p a_q + 1/4 sum_pqrs v_pqrs a^dagger_p a^dagger_q a_s a_r
over spin orbitals, mapped by JW to H_q = sum_l h_l P_l (Eq. (2)).

Readings (the paper gives spin-orbital integrals from Psi4; here spatial
integrals are given):
* spin orbital 2p = alpha, 2p+1 = beta of spatial orbital p;
* h_PQ = h_pq if the spins of P and Q agree, else 0;
* v_PQRS = <PQ||RS> = <PQ|RS> - <PQ|SR>, <PQ|RS> = (pr|qs) delta(sP,sR)
  delta(sQ,sS), with g[p,q,r,s] = (pq|rs) in chemists' notation;
* e_core multiplies the identity string.
After collecting like strings, imaginary parts must vanish (|Im| <= 1e-12:
real integrals give a real symmetric matrix) and strings with |c| <= 1e-12
are dropped.
"""
from __future__ import annotations

import numpy as np

from .pauli import ladder, op_mul


def spin_orbital_integrals(h: np.ndarray, g: np.ndarray):
    """Return (h_so[N,N], v[N,N,N,N]) for N = 2 * n_orb spin orbitals."""
    n = h.shape[0]
    N = 2 * n
    sp = np.arange(N) % 2
    orb = np.arange(N) // 2
    same = sp[:, None] == sp[None, :]
    h_so = np.where(same, h[orb[:, None], orb[None, :]], 0.0)
    # <PQ|RS> = (pr|qs) d(sP,sR) d(sQ,sS)
    P, Q, R, S = np.ix_(np.arange(N), np.arange(N), np.arange(N), np.arange(N))
    pr = g[orb[P], orb[R], orb[Q], orb[S]]
    phys = np.where((sp[P] == sp[R]) & (sp[Q] == sp[S]), pr, 0.0)
    v = phys - np.transpose(phys, (0, 1, 3, 2))
    return h_so, v


def fermion_hamiltonian_terms(h: np.ndarray, g: np.ndarray):
    """Yield (coeff, creators, annihilators) of Eq. (1), zero terms skipped."""
    h_so, v = spin_orbital_integrals(h, g)
    N = h_so.shape[0]
    for p in range(N):
        for q in range(N):
            if h_so[p, q] != 0.0:
                yield h_so[p, q], (p,), (q,)
    for p in range(N):
        for q in range(N):
            for r in range(N):
                for s in range(N):
                    if v[p, q, r, s] != 0.0:
                        yield 0.25 * v[p, q, r, s], (p, q), (s, r)


def qubit_hamiltonian(h: np.ndarray, g: np.ndarray, e_core: float = 0.0,
                      drop: float = 1e-12) -> dict:
    """JW qubit Hamiltonian {(x, z): real c} of Eq. (2)."""
    N = 2 * h.shape[0]
    cre = [ladder(p, True) for p in range(N)]
    ann = [ladder(p, False) for p in range(N)]
    pair_cc = {}
    pair_aa = {}
    acc: dict = {}
    if e_core != 0.0:
        acc[(0, 0)] = complex(e_core)
    for coeff, cs, an in fermion_hamiltonian_terms(h, g):
        if len(cs) == 1:
            op = op_mul(cre[cs[0]], ann[an[0]])
        else:
            left = pair_cc.get(cs)
            if left is None:
                left = pair_cc[cs] = op_mul(cre[cs[0]], cre[cs[1]])
            right = pair_aa.get(an)
            if right is None:
                right = pair_aa[an] = op_mul(ann[an[0]], ann[an[1]])
            op = op_mul(left, right)
        for key, c in op.items():
            acc[key] = acc.get(key, 0.0) + coeff * c
    out = {}
    for key, c in acc.items():
        if abs(c.imag) > 1e-12:
            raise ValueError(f"non-real coefficient {c} for string {key}")
        if abs(c.real) > drop:
            out[key] = float(c.real)
    return out


def group_by_flip_mask(op: dict):
    """Sort strings by (x, z) and return (x, z, c, group_off).

    x, z are uint64 arrays, c float64; strings of group g are
    group_off[g]:group_off[g+1], all sharing the flip mask x.
    """
    keys = sorted(op.keys())
    x = np.array([k[0] for k in keys], dtype=np.uint64)
    z = np.array([k[1] for k in keys], dtype=np.uint64)
    c = np.array([op[k] for k in keys], dtype=np.float64)
    off = [0]
    for i in range(1, len(keys)):
        if keys[i][0] != keys[i - 1][0]:
            off.append(i)
    off.append(len(keys))
    return x, z, c, np.array(off, dtype=np.int64)
