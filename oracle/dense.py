"""Dense-matrix toolkit for tiny systems (n <= ~10 qubits).

Three constructions that share no code with the Pauli-dict builder:

* ``pauli_matrix``: Kronecker products of 2x2 matrices, qubit q = bit q of
  the row index (Sec. 2.1.1, Eq. (3)).
* ``ladder_matrix`` / ``fermion_matrix``: second quantization acting on
  occupation bit strings with the sign (-1)^(number of occupied orbitals
  below p), i.e. creation/annihilation in a fixed orbital order; no Pauli
  strings are involved.
* ``gate`` / ``circuit``: the gates of Sec. 2.1.3-2.1.4 (H, X, Z, CNOT,
  R_z) used to build the circuit of Fig. "exp_pt".
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X2 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z2 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H2 = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)


def embed(ops: dict, n: int) -> np.ndarray:
    """Kronecker product with ops[q] on qubit q; qubit n-1 is leftmost."""
    m = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(range(n)):
        m = np.kron(m, ops.get(q, I2))
    return m


def pauli_matrix(x: int, z: int, n: int) -> np.ndarray:
    """Dense P(x, z): X, Y or Z on each qubit according to (x_q, z_q)."""
    ops = {}
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        if xb and zb:
            ops[q] = Y2
        elif xb:
            ops[q] = X2
        elif zb:
            ops[q] = Z2
    return embed(ops, n)


def pauli_sum_matrix(xs, zs, cs, n: int) -> np.ndarray:
    m = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for x, z, c in zip(xs, zs, cs):
        m += complex(c) * pauli_matrix(int(x), int(z), n)
    return m


def ladder_matrix(p: int, dagger: bool, n: int) -> np.ndarray:
    """a_p or a_p^dagger on occupation bit strings (1 = occupied)."""
    dim = 1 << n
    m = np.zeros((dim, dim), dtype=np.complex128)
    below = (1 << p) - 1
    for b in range(dim):
        occ = (b >> p) & 1
        if dagger and not occ:
            m[b | (1 << p), b] = (-1) ** bin(b & below).count("1")
        if not dagger and occ:
            m[b & ~(1 << p), b] = (-1) ** bin(b & below).count("1")
    return m


def apply_string(b: int, creators, annihilators):
    """Apply a^dagger_{c1} ... a_{a1} ... (rightmost first) to determinant b.

    Returns (sign, b') or (0, None) if the result vanishes.
    """
    sign = 1
    for p, dag in [(p, False) for p in reversed(annihilators)] + \
                  [(p, True) for p in reversed(creators)]:
        occ = (b >> p) & 1
        if occ == dag:  # create on occupied / annihilate empty
            return 0, None
        if bin(b & ((1 << p) - 1)).count("1") & 1:
            sign = -sign
        b ^= 1 << p
    return sign, b


def fermion_matrix(terms, n: int) -> np.ndarray:
    """Dense matrix of sum coeff * a^dagger... a... over all 2^n determinants."""
    dim = 1 << n
    m = np.zeros((dim, dim), dtype=np.complex128)
    for coeff, cre, ann in terms:
        for b in range(dim):
            s, b2 = apply_string(b, cre, ann)
            if s:
                m[b2, b] += s * coeff
    return m


def ground_energy_in_sector(hmat: np.ndarray, n: int, n_elec: int, sz2: int | None = None) -> float:
    """Lowest eigenvalue of H restricted to N = n_elec (and 2 S_z = sz2)."""
    idx = []
    for b in range(1 << n):
        if bin(b).count("1") != n_elec:
            continue
        if sz2 is not None:
            na = bin(b & int("01" * (n // 2 + 1), 2)).count("1")
            nb = n_elec - na
            if na - nb != sz2:
                continue
        idx.append(b)
    sub = hmat[np.ix_(idx, idx)]
    return float(np.linalg.eigvalsh(sub)[0])


# ---- gates of Sec. 2.1.3 -------------------------------------------------

def gate(kind: str, target: int, control: int | None = None, angle: float = 0.0, n: int = 1):
    """Dense gate; gate('CNOT', target, control) as in the paper's listings."""
    if kind == "CNOT":
        dim = 1 << n
        m = np.zeros((dim, dim), dtype=np.complex128)
        for b in range(dim):
            b2 = b ^ (1 << target) if (b >> control) & 1 else b
            m[b2, b] = 1.0
        return m
    if kind == "Rz":
        # R_z(phi) = exp(-i phi Z / 2)
        one = np.diag([np.exp(-0.5j * angle), np.exp(0.5j * angle)])
    else:
        one = {"H": H2, "X": X2, "Y": Y2, "Z": Z2, "I": I2}[kind]
    return embed({target: one}, n)


def circuit(gates, n: int) -> np.ndarray:
    """Product of gates; the first gate in the list acts first."""
    u = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        u = g @ u
    return u
