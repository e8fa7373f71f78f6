"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and nothing else: it holds no Pauli
algebra, no Jordan-Wigner mapping and no state-vector arithmetic, so that the
CPU oracle and the HIP path can both consume the same arrays without sharing
any of the method's code.

The paper's workloads are hydrogen chains in a minimal basis whose integrals
come from Psi4 (Sec. 4, Fig. "hn_timings"; Sec. 2.3).  No electronic-structure
package is available here, so random real integrals with the symmetry of real
molecular integrals stand in for them:

* h_pq: upper triangle (diagonal included, row-major order) drawn i.i.d.
  N(0, 1), then mirrored; h_ii is lowered by 2 for the spatial orbitals that
  the Hartree-Fock determinant occupies (i < ceil(n_elec / 2)).
* (pq|rs) (chemists' notation): one N(0, 0.1^2) draw per 8-fold symmetry
  class, classes visited with compound indices pq = p(p+1)/2 + q (p >= q),
  rs likewise, pq ascending, rs <= pq ascending; the draw is copied to all
  eight index permutations.
* cluster amplitudes t_mu ~ U[-a, a] from a second stream (seed, 1), one per
  excitation in the order the caller enumerates them.
"""
from __future__ import annotations

import math

import numpy as np

# name -> recipe.  "uccsd": all S_z-conserving singles and doubles;
# "uccd_top": doubles only, the top_k by |t| survive.
WORKLOADS = {
    "8q": dict(n_orb=4, n_elec=4, seed=1008, t_scale=0.1, ansatz="uccsd", top_k=0),
    "20q": dict(n_orb=10, n_elec=10, seed=1020, t_scale=0.1, ansatz="uccsd", top_k=0),
    "28q": dict(n_orb=14, n_elec=14, seed=1028, t_scale=0.1, ansatz="uccd_top", top_k=512),
}

BATCH_QUBITS = (12, 14, 16, 18, 20, 22)
BATCH_SEED = 2000
SERVE_QUBITS = (12, 14, 16, 18, 20, 22, 24)
SERVE_WEIGHTS = (0.10, 0.15, 0.40, 0.15, 0.10, 0.06, 0.04)
SERVE_REQ_SEED = 3000
SERVE_TRACE_SEED = 4000


def integrals(n_orb: int, n_elec: int, seed: int):
    """Return (h[n,n], g[n,n,n,n]) float64 arrays for the recipe above."""
    n = int(n_orb)
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    iu = np.triu_indices(n)
    h[iu] = rng.standard_normal(len(iu[0]))
    h = h + h.T - np.diag(np.diag(h))
    for i in range((int(n_elec) + 1) // 2):
        h[i, i] -= 2.0
    # compound pairs (p, q), q <= p, in row-major order; classes (pq, rs)
    # with rs <= pq, again row-major; one draw per class, in that order
    P, Q = np.tril_indices(n)
    ca, cb = np.tril_indices(len(P))
    p, q, r, s = P[ca], Q[ca], P[cb], Q[cb]
    vals = 0.1 * rng.standard_normal(len(ca))
    g = np.zeros((n, n, n, n))
    for (a, b, c, d) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                         (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
        g[a, b, c, d] = vals  # every index tuple lies in exactly one class
    return h, g


def amplitudes(n_par: int, seed: int, scale: float):
    """n_par cluster amplitudes ~ U[-scale, scale] from stream (seed, 1)."""
    rng = np.random.default_rng([int(seed), 1])
    return rng.uniform(-scale, scale, int(n_par))


def workload(name: str):
    """(recipe dict, h, g) for one of the named workloads."""
    w = dict(WORKLOADS[name])
    h, g = integrals(w["n_orb"], w["n_elec"], w["seed"])
    return w, h, g


def batched_instances(count: int = 256, seed: int = BATCH_SEED, t_scale: float = 0.2):
    """Instance recipes for the batched configuration.

    Qubit counts are drawn uniformly from BATCH_QUBITS with stream (seed, 0);
    instance i uses integral seed seed + i and electrons = qubits / 2.
    """
    rng = np.random.default_rng([int(seed), 0])
    qs = rng.choice(np.array(BATCH_QUBITS), size=int(count))
    out = []
    for i, nq in enumerate(qs):
        nq = int(nq)
        out.append(dict(n_orb=nq // 2, n_elec=nq // 2, seed=int(seed) + i,
                        t_scale=t_scale, ansatz="uccsd", top_k=0))
    return out


def serving_trace(count: int = 10000, rate: float = 2000.0, seed: int = SERVE_TRACE_SEED,
                  req_seed: int = SERVE_REQ_SEED, t_scale: float = 0.1):
    """Poisson arrival trace: list of (arrival_s, recipe) sorted by arrival."""
    rng = np.random.default_rng(int(seed))
    gaps = rng.exponential(1.0 / rate, int(count))
    arrivals = np.cumsum(gaps)
    qs = rng.choice(np.array(SERVE_QUBITS), size=int(count), p=np.array(SERVE_WEIGHTS))
    out = []
    for j in range(int(count)):
        nq = int(qs[j])
        out.append((float(arrivals[j]),
                    dict(n_orb=nq // 2, n_elec=nq // 2, seed=int(req_seed) + j,
                         t_scale=t_scale, ansatz="uccsd", top_k=0)))
    return out


def random_state(n_qubits: int, seed: int):
    """A normalized random complex128 vector of length 2**n_qubits."""
    rng = np.random.default_rng([int(seed), 2])
    v = rng.standard_normal(1 << n_qubits) + 1j * rng.standard_normal(1 << n_qubits)
    return v / math.sqrt(float(np.vdot(v, v).real))


def random_paulis(n_qubits: int, count: int, seed: int, max_weight: int = 0):
    """Random (x, z, c) Pauli terms as uint64/uint64/float64 arrays.

    With max_weight > 0 every string acts non-trivially on at most that many
    qubits; coefficients ~ N(0, 1).
    """
    rng = np.random.default_rng([int(seed), 3])
    xs = np.zeros(count, dtype=np.uint64)
    zs = np.zeros(count, dtype=np.uint64)
    for k in range(count):
        if max_weight:
            w = int(rng.integers(1, max_weight + 1))
            qubits = rng.choice(n_qubits, size=min(w, n_qubits), replace=False)
            x = z = 0
            for q in qubits:
                kind = int(rng.integers(1, 4))  # 1 X, 2 Z, 3 Y
                if kind & 1:
                    x |= 1 << int(q)
                if kind & 2:
                    z |= 1 << int(q)
        else:
            x = int(rng.integers(0, 1 << n_qubits))
            z = int(rng.integers(0, 1 << n_qubits))
        xs[k] = x
        zs[k] = z
    cs = rng.standard_normal(count)
    return xs, zs, cs


def random_angles(count: int, seed: int, scale: float = math.pi):
    rng = np.random.default_rng([int(seed), 4])
    return rng.uniform(-scale, scale, int(count))
