"""Particle-number and S_z restricted state vector (Sec. 6 names it as the
way to run past ~24 qubits).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A Hamiltonian and a UCC ansatz that conserve N_alpha and N_beta keep a
state built from the reference inside the sector of determinants with
those occupation numbers, so only those amplitudes need to be stored.
Layout (readings; the paper gives none): spin orbital 2j is alpha and
2j + 1 is beta of spatial orbital j, as everywhere in this package; an
alpha (beta) string is the n_orb-bit mask of the occupied alpha (beta)
orbitals; the strings of one spin are ranked by increasing integer value;
determinant (a, b) sits at index rank(a) * D_beta + rank(b).

* restrict / embed: the plain definition, the full vector's entries at the
  sector's determinants and back;
* apply_excitations: exp(t kappa) for kappa = tau - tau^dagger acts on each
  pair of determinants D, D' with tau D = s D' (s = +-1 the fermionic sign)
  as D -> cos t D + s sin t D', D' -> cos t D' - s sin t D, and leaves every
  other determinant alone (Sec. 3.1, one factor of Eq. (ducc));
* energy: sum over flip-mask groups g of sum over sector determinants y with
  y ^ x_g also in the sector of conj(psi[y ^ x_g]) D_g(y) psi[y], which is
  the full-space group sum of Eq. (17) restricted to the amplitudes that can
  be nonzero.
"""
from __future__ import annotations

import math
from itertools import combinations

import numpy as np


def strings(n_orb: int, k: int) -> np.ndarray:
    """The n_orb-bit masks with k bits set, ascending."""
    out = [sum(1 << p for p in c) for c in combinations(range(n_orb), k)]
    return np.array(sorted(out), dtype=np.int64)


def interleave(a: int, b: int, n_orb: int) -> int:
    """Spin-orbital bit string: bit 2j = a_j, bit 2j + 1 = b_j."""
    y = 0
    for j in range(n_orb):
        y |= ((a >> j) & 1) << (2 * j)
        y |= ((b >> j) & 1) << (2 * j + 1)
    return y


def determinants(n_orb: int, na: int, nb: int) -> np.ndarray:
    """Full-space index of every sector determinant, in sector order."""
    A, B = strings(n_orb, na), strings(n_orb, nb)
    return np.array([interleave(int(a), int(b), n_orb) for a in A for b in B], dtype=np.int64)


def restrict(psi_full: np.ndarray, n_orb: int, na: int, nb: int) -> np.ndarray:
    return psi_full[determinants(n_orb, na, nb)].copy()


def embed(psi: np.ndarray, n_orb: int, na: int, nb: int) -> np.ndarray:
    full = np.zeros(1 << (2 * n_orb), dtype=np.complex128)
    full[determinants(n_orb, na, nb)] = psi
    return full


def prepare(n_orb: int, na: int, nb: int, occ: int) -> np.ndarray:
    dets = determinants(n_orb, na, nb)
    psi = np.zeros(len(dets), dtype=np.complex128)
    psi[int(np.nonzero(dets == occ)[0][0])] = 1.0
    return psi


def _excite(y: int, creators, annihilators):
    """(s, y') with tau |y> = s |y'>, operators applied right to left with
    (-1)^(occupied spin orbitals below p) each; (0, None) if tau |y> = 0."""
    s = 1
    for p, dag in [(p, False) for p in reversed(annihilators)] + [(p, True) for p in reversed(creators)]:
        if ((y >> p) & 1) == int(dag):
            return 0, None
        if bin(y & ((1 << p) - 1)).count("1") & 1:
            s = -s
        y ^= 1 << p
    return s, y


def apply_excitations(psi: np.ndarray, n_orb: int, na: int, nb: int, excs, t) -> np.ndarray:
    """prod_mu exp(t_mu kappa_mu) psi, the first excitation acting first."""
    dets = determinants(n_orb, na, nb)
    where = {int(d): i for i, d in enumerate(dets)}
    psi = psi.copy()
    for (cre, ann), tm in zip(excs, t):
        c, sn = math.cos(tm), math.sin(tm)
        for i, d in enumerate(dets):
            s, d2 = _excite(int(d), cre, ann)
            if not s:
                continue
            j = where[d2]
            u, v = psi[i], psi[j]
            psi[i] = c * u - s * sn * v
            psi[j] = c * v + s * sn * u
    return psi


def energy(psi: np.ndarray, n_orb: int, na: int, nb: int, hx, hz, hc, goff) -> float:
    """<psi|H|psi> from the grouped Pauli strings, over sector pairs only."""
    dets = determinants(n_orb, na, nb)
    where = {int(d): i for i, d in enumerate(dets)}
    total = []
    for g in range(len(goff) - 1):
        x = int(hx[goff[g]])
        acc = 0.0
        for i, y in enumerate(dets):
            j = where.get(int(y) ^ x)
            if j is None:
                continue
            dg = 0.0 + 0.0j
            for k in range(goff[g], goff[g + 1]):
                z = int(hz[k])
                ph = (bin(x & z).count("1") + 2 * bin(int(y) & z).count("1")) % 4
                dg += float(hc[k]) * (1, 1j, -1, -1j)[ph]
            acc += (np.conj(psi[j]) * dg * psi[i]).real
        total.append(acc)
    return math.fsum(total)
