"""Plain numpy state vector (complex128, 2^n amplitudes, qubit q = bit q).

Every operation is one whole-vector numpy expression per Pauli string, in
the order the paper writes the math; nothing is fused or blocked.

* P(x, z)|b> = i^popcount(x & z) (-1)^popcount(b & z) |b ^ x>  (Sec. 2.1.1:
  a basis state is an integer, a Pauli string flips the bits in x).
* exp(-i theta P) = cos(theta) I - i sin(theta) P since P^2 = I; the paper's
  circuit for it (Sec. 2.1.4, Eqs. (8)-(11)) rotates by 2 theta with the
  exp(-i theta P) sign convention of its worked example.
* E = sum_l h_l <psi|P_l|psi> (Sec. 3.1, Eq. (17)).
* gradient of E(theta) for psi = U_{K-1} ... U_0 |Phi>, U_k = exp(-i theta_k P_k):
  dE/dtheta_k = 2 Im <lambda_k| P_k |phi_k> with phi_k = U_k ... U_0 Phi and
  lambda_k = U_{k+1}^dagger ... U_{K-1}^dagger H psi (the adjoint sweep), and
  independently E(theta_k + pi/4) - E(theta_k - pi/4) (parameter shift, exact
  for P^2 = I).
"""
from __future__ import annotations

import math

import numpy as np


def _indices(n: int) -> np.ndarray:
    return np.arange(1 << n, dtype=np.uint64)


def _parity(v: np.ndarray) -> np.ndarray:
    return (np.bitwise_count(v) & 1).astype(np.int64)


PHASE = np.array([1.0 + 0j, 1j, -1.0 + 0j, -1j])


def omega(n: int, x: int, z: int) -> np.ndarray:
    """omega(b) with P|b> = omega(b) |b ^ x>, for every basis state b."""
    b = _indices(n)
    k = bin(x & z).count("1") + 2 * _parity(b & np.uint64(z))
    return PHASE[k % 4]


def prepare(n: int, occ_mask: int) -> np.ndarray:
    """The determinant |occ_mask> (Sec. 3.1 reference state Phi_0)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[occ_mask] = 1.0
    return psi


def apply_pauli(psi: np.ndarray, n: int, x: int, z: int) -> np.ndarray:
    out = np.empty_like(psi)
    b = _indices(n)
    out[b ^ np.uint64(x)] = omega(n, x, z) * psi
    return out


def apply_exp(psi: np.ndarray, n: int, x: int, z: int, theta: float) -> np.ndarray:
    """exp(-i theta P(x, z)) psi."""
    return math.cos(theta) * psi - 1j * math.sin(theta) * apply_pauli(psi, n, x, z)


def apply_product(psi, n, xs, zs, thetas, inverse=False):
    """prod_k exp(-i theta_k P_k) psi with k = 0 acting first.

    inverse=True applies the adjoint: exp(+i theta_k P_k) for k = K-1 ... 0.
    """
    order = range(len(xs) - 1, -1, -1) if inverse else range(len(xs))
    sign = -1.0 if inverse else 1.0
    for k in order:
        psi = apply_exp(psi, n, int(xs[k]), int(zs[k]), sign * float(thetas[k]))
    return psi


def expval_pauli(psi: np.ndarray, n: int, x: int, z: int) -> complex:
    return complex(np.vdot(psi, apply_pauli(psi, n, x, z)))


def energy(psi, n, xs, zs, cs) -> float:
    """sum_l c_l <psi|P_l|psi>, the outer sum taken exactly (math.fsum)."""
    vals = [float(cs[k]) * expval_pauli(psi, n, int(xs[k]), int(zs[k])).real
            for k in range(len(xs))]
    return math.fsum(vals)


def sigma(psi, n, xs, zs, cs) -> np.ndarray:
    """H|psi> = sum_l c_l P_l |psi>."""
    out = np.zeros_like(psi)
    for k in range(len(xs)):
        out += float(cs[k]) * apply_pauli(psi, n, int(xs[k]), int(zs[k]))
    return out


def energy_of(n, occ_mask, ax, az, thetas, hx, hz, hc) -> float:
    psi = apply_product(prepare(n, occ_mask), n, ax, az, thetas)
    return energy(psi, n, hx, hz, hc)


def adjoint_gradient(n, occ_mask, ax, az, thetas, hx, hz, hc):
    """(E, dE/dtheta) by the reverse sweep described in the module docstring."""
    K = len(ax)
    psi = apply_product(prepare(n, occ_mask), n, ax, az, thetas)
    lam = sigma(psi, n, hx, hz, hc)
    e = float(np.vdot(psi, lam).real)
    phi = psi
    grad = np.zeros(K)
    for k in range(K - 1, -1, -1):
        x, z, th = int(ax[k]), int(az[k]), float(thetas[k])
        grad[k] = 2.0 * np.vdot(lam, apply_pauli(phi, n, x, z)).imag
        phi = apply_exp(phi, n, x, z, -th)
        lam = apply_exp(lam, n, x, z, -th)
    return e, grad


def parameter_shift_gradient(n, occ_mask, ax, az, thetas, hx, hz, hc):
    """dE/dtheta_k = E(theta_k + pi/4) - E(theta_k - pi/4), one pair per k."""
    K = len(ax)
    grad = np.zeros(K)
    for k in range(K):
        tp = np.array(thetas, dtype=np.float64)
        tm = tp.copy()
        tp[k] += math.pi / 4
        tm[k] -= math.pi / 4
        grad[k] = (energy_of(n, occ_mask, ax, az, tp, hx, hz, hc)
                   - energy_of(n, occ_mask, ax, az, tm, hx, hz, hc))
    return grad


def number_expectation(psi: np.ndarray, n: int, mask: int = -1) -> float:
    """<N> restricted to the qubits in mask (all qubits by default)."""
    if mask < 0:
        mask = (1 << n) - 1
    counts = np.bitwise_count(_indices(n) & np.uint64(mask)).astype(np.float64)
    return float(np.sum(np.abs(psi) ** 2 * counts))
