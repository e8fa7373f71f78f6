"""Disentangled UCC ansatz: excitations, canonical order and JW exponents.

Sec. 3.1, Eq. (18): U(t) = prod_mu exp(t_mu kappa_mu), kappa_mu = tau_mu -
tau_mu^dagger, tau_mu = a^dagger_a a^dagger_b ... a_j a_i a particle-hole
excitation out of the reference determinant.

Readings:
* reference: the n_elec lowest spin orbitals (bits 0..n_elec-1) are occupied;
  with interleaved spin orbitals an odd electron count puts the extra
  electron in alpha;
* singles a <- i and doubles (a < b) <- (i < j) that conserve S_z, one
  amplitude each, with tau = a^dagger_a a^dagger_b a_j a_i literally;
* order: ascending integer value of the excited determinant's bit string
  (Sec. 3.1 orders the factors by the binary representation of the
  determinants); the first factor in the list acts first on the reference;
* JW(kappa_mu) = i sum_k c_k P_k with real c_k (kappa is anti-Hermitian), so
  exp(t kappa) = prod_k exp(-i theta_k P_k) with theta_k = -c_k t.  The
  strings of one kappa_mu commute, so this factorization is exact;
* truncated doubles: rank by |t| descending, ties by canonical position,
  keep top_k, apply them in canonical order.
"""
from __future__ import annotations

import numpy as np

from .pauli import clean, op_add, sq_term


def reference_mask(n_elec: int) -> int:
    return (1 << n_elec) - 1


def excitations(n_qubits: int, n_elec: int, singles: bool = True, doubles: bool = True):
    """S_z-conserving particle-hole excitations in canonical order.

    Each item is (creators, annihilators) = ((a,), (i,)) or ((a, b), (j, i)),
    so that tau = a^dagger_a [a^dagger_b] [a_j] a_i.
    """
    occ = list(range(n_elec))
    vir = list(range(n_elec, n_qubits))
    ref = reference_mask(n_elec)
    items = []
    if singles:
        for i in occ:
            for a in vir:
                if (i & 1) == (a & 1):
                    det = ref ^ (1 << i) ^ (1 << a)
                    items.append((det, (a,), (i,)))
    if doubles:
        for ii in range(len(occ)):
            for jj in range(ii + 1, len(occ)):
                i, j = occ[ii], occ[jj]
                for aa in range(len(vir)):
                    for bb in range(aa + 1, len(vir)):
                        a, b = vir[aa], vir[bb]
                        if (i & 1) + (j & 1) == (a & 1) + (b & 1):
                            det = ref ^ (1 << i) ^ (1 << j) ^ (1 << a) ^ (1 << b)
                            items.append((det, (a, b), (j, i)))
    items.sort(key=lambda it: it[0])
    return [(cre, ann) for _, cre, ann in items]


def paired_doubles(n_qubits: int, n_elec: int):
    """Seniority-zero doubles i_alpha i_beta -> a_alpha a_beta (Sec. 5 example).

    tau = a^dagger_{a_beta} a^dagger_{a_alpha} a_{i_alpha} a_{i_beta} as the
    p-dUCCD operator of Sec. 5 is written; occupied spatial i outer loop,
    virtual a inner loop.
    """
    nocc = n_elec // 2
    nvir = (n_qubits - n_elec) // 2
    out = []
    for i in range(nocc):
        for a in range(nvir):
            ia, ib = 2 * i, 2 * i + 1
            aa, ab = 2 * nocc + 2 * a, 2 * nocc + 2 * a + 1
            out.append(((ab, aa), (ia, ib)))
    return out


def kappa_strings(creators, annihilators):
    """JW(kappa) for tau = a^dagger... a...: returns {(x, z): c} with JW(kappa) = i sum c P."""
    tau = sq_term(1.0, creators, annihilators)
    tau_dag = sq_term(1.0, tuple(reversed(annihilators)), tuple(reversed(creators)))
    kappa = op_add(dict(tau), tau_dag, -1.0)
    out = {}
    for key, c in clean(kappa).items():
        if abs(c.real) > 1e-12:
            raise ValueError("kappa has a non-imaginary coefficient")
        out[key] = float(c.imag)
    return out


def ansatz_terms(excs):
    """Concatenate the JW strings of each kappa_mu (sorted by (x, z) within mu).

    Returns (x, z, c, exc_off) with exc_off[mu]:exc_off[mu+1] the strings of
    excitation mu.
    """
    xs, zs, cs, off = [], [], [], [0]
    for cre, ann in excs:
        st = kappa_strings(cre, ann)
        for key in sorted(st):
            xs.append(key[0])
            zs.append(key[1])
            cs.append(st[key])
        off.append(len(xs))
    return (np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
            np.array(cs, dtype=np.float64), np.array(off, dtype=np.int64))


def top_k(t: np.ndarray, k: int) -> np.ndarray:
    """Indices (ascending) of the k largest |t|; ties go to the earlier index."""
    order = sorted(range(len(t)), key=lambda m: (-abs(float(t[m])), m))
    return np.array(sorted(order[:k]), dtype=np.int64)


def angles(c: np.ndarray, exc_off: np.ndarray, t: np.ndarray) -> np.ndarray:
    """theta_k = -c_k t_mu for every string k of excitation mu."""
    theta = np.empty(len(c))
    for mu in range(len(exc_off) - 1):
        for k in range(exc_off[mu], exc_off[mu + 1]):
            theta[k] = -c[k] * t[mu]
    return theta


def grad_t(c: np.ndarray, exc_off: np.ndarray, dtheta: np.ndarray) -> np.ndarray:
    """dE/dt_mu = sum_k (d theta_k / d t_mu) dE/dtheta_k = -sum_k c_k dE/dtheta_k."""
    g = np.zeros(len(exc_off) - 1)
    for mu in range(len(exc_off) - 1):
        for k in range(exc_off[mu], exc_off[mu + 1]):
            g[mu] += -c[k] * dtheta[k]
    return g


def build(n_orb: int, n_elec: int, ansatz: str = "uccsd", t_all=None, k: int = 0):
    """Excitation list and JW strings for a workload recipe.

    ansatz "uccsd": singles + doubles; "uccd_top": doubles, truncated to the
    k largest |t_all| (t_all drawn for every double in canonical order).
    Returns (excs, x, z, c, exc_off, kept) where kept indexes t_all.
    """
    nq = 2 * n_orb
    if ansatz == "uccsd":
        excs = excitations(nq, n_elec)
        kept = np.arange(len(excs), dtype=np.int64)
    elif ansatz == "uccd_top":
        allx = excitations(nq, n_elec, singles=False)
        kept = top_k(t_all, k)
        excs = [allx[m] for m in kept]
    elif ansatz == "pduccd":
        excs = paired_doubles(nq, n_elec)
        kept = np.arange(len(excs), dtype=np.int64)
    else:
        raise ValueError(ansatz)
    x, z, c, off = ansatz_terms(excs)
    return excs, x, z, c, off, kept
