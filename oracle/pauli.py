"""Pauli-string algebra with exact phases and the Jordan-Wigner map.

A Pauli string on qubits 0..63 is a pair of bit masks (x, z):
P(x, z) = i^popcount(x & z) * X^x Z^z, where X^x = prod_{q in x} X_q and
Z^z = prod_{q in z} Z_q.  A qubit with both bits set carries Y = i X Z, so
P(x, z) is the usual Hermitian tensor product of I/X/Y/Z (Sec. 2.1.4, Eq. (9)).

Operators are dicts {(x, z): complex coefficient}.  Phases are tracked as
integer exponents of i modulo 4, never as floats, so masks and phases are
exact.
"""
from __future__ import annotations

PHASE = (1.0 + 0.0j, 1.0j, -1.0 + 0.0j, -1.0j)  # i^k, k = 0..3


def popcount(v: int) -> int:
    return bin(v).count("1")


def pauli_mul(x1: int, z1: int, x2: int, z2: int):
    """P(x1,z1) P(x2,z2) = i^k P(x1^x2, z1^z2); returns (x, z, k mod 4).

    X^a Z^b X^c Z^d = (-1)^popcount(b & c) X^(a^c) Z^(b^d) because Z_q X_q =
    -X_q Z_q; converting both sides between X^x Z^z and P(x, z) adds and
    removes one factor i per Y.
    """
    x3 = x1 ^ x2
    z3 = z1 ^ z2
    k = popcount(x1 & z1) + popcount(x2 & z2) + 2 * popcount(z1 & x2) - popcount(x3 & z3)
    return x3, z3, k % 4


def op_mul(a: dict, b: dict) -> dict:
    """Product of two Pauli-sum operators (a on the left)."""
    out: dict = {}
    for (x1, z1), c1 in a.items():
        for (x2, z2), c2 in b.items():
            x3, z3, k = pauli_mul(x1, z1, x2, z2)
            out[(x3, z3)] = out.get((x3, z3), 0.0) + c1 * c2 * PHASE[k]
    return out


def op_add(acc: dict, b: dict, scale: complex = 1.0) -> dict:
    for key, c in b.items():
        acc[key] = acc.get(key, 0.0) + scale * c
    return acc


def ladder(p: int, dagger: bool) -> dict:
    """Jordan-Wigner image of a_p (dagger=False) or a_p^dagger (Sec. 2.2).

    a_p = (X_p + i Y_p)/2 Z_{p-1}...Z_0 and a_p^dagger = (X_p - i Y_p)/2 Z_{p-1}...Z_0
    (Eqs. (13)-(14)).  With the Z chain on qubits below p written as the mask
    (1 << p) - 1:  X_p Z_chain = P(1<<p, chain) and Y_p Z_chain =
    P(1<<p, chain | 1<<p).
    """
    bit = 1 << p
    chain = bit - 1
    s = -1.0 if dagger else 1.0
    return {(bit, chain): 0.5 + 0.0j, (bit, chain | bit): s * 0.5j}


def sq_term(coeff: complex, creators, annihilators) -> dict:
    """JW image of coeff * a^dagger_{c1} a^dagger_{c2} ... a_{a1} a_{a2} ...

    Operators are multiplied in the order written, matching the paper's
    SQOperator.add_term(coeff, creators, annihilators) (Sec. 2.2).
    """
    op = {(0, 0): complex(coeff)}
    for p in creators:
        op = op_mul(op, ladder(p, True))
    for p in annihilators:
        op = op_mul(op, ladder(p, False))
    return op


def clean(op: dict, tol: float = 1e-12) -> dict:
    return {k: c for k, c in op.items() if abs(c) > tol}


def to_string(x: int, z: int, n: int) -> str:
    """Human-readable label, e.g. 'X2 Z1 Z0' for x=0b100, z=0b011."""
    parts = []
    for q in reversed(range(n)):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        if xb or zb:
            parts.append(("Y" if (xb and zb) else "X" if xb else "Z") + str(q))
    return " ".join(parts) if parts else "I"
