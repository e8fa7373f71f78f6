"""Time one operation of the library on a seeded instance (meant to run under
a profiler, e.g. `rocprofv3 --kernel-trace --stats -- python3 -m
paper_2108_04413_amd.measure --op pool --qubits 20`).

    --op eg      energy + adjoint gradient (Sec. 3.1), plan path
    --op pool    ADAPT pool gradients over the generalized pool (Sec. 3.2)
    --op pqe     PQE residuals of the UCCSD excitations (Sec. 3.3)
    --op qk      QK basis by Trotterized evolution, S and H (Sec. 3.7),
                 dt 0.5, s 3, r 1
    --op sector  restricted state vector: reference, UCCSD factors, energy
    --op sector_eg  restricted state vector: energy and dE/dt per excitation
    --op sigma   lambda = H psi (Eq. (17) as a sigma) on the UCCSD state

The instance is the autotuner's: n/2 spatial orbitals and n/2 electrons,
seeded random integrals, all UCCSD excitations, amplitudes ~ U[-0.2, 0.2].
Prints the pass counts and the best of `reps` timed calls (after one
untimed).
"""
from __future__ import annotations

import argparse
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--op", default="eg", choices=("eg", "pool", "pqe", "qk", "sector", "sector_eg", "sigma"))
    ap.add_argument("--qubits", type=int, default=24)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=None)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2108_04413_amd as qf
    from paper_2108_04413_amd.autotune import _instances
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import qf_inputs as qi

    n = args.qubits
    seed = args.seed if args.seed is not None else 7000 + n
    d = _instances(qf, qi, n, 1, seed)[0]
    no = n // 2
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    plan = qf.Plan(n, d["A"], d["H"], d["off"])
    print(f"{n} qubits: {len(d['A'])} ansatz strings, {len(d['H'])} Hamiltonian strings in "
          f"{len(d['off']) - 1} groups; apply {plan.apply_info()}; sweep {plan.grad_info()}", flush=True)
    if args.op == "eg":
        def call():
            return plan.energy_grad(d["occ"], d["theta"], ws)[0]
    elif args.op == "pool":
        pool, poff, _ = qf.build_paulis("gsd_pool", no, 0)
        Q = qf.PoolPlan(n, pool, poff)
        print(f"pool: {len(poff) - 1} members, {len(pool)} strings, sweep {Q.grad_info()}", flush=True)

        def call():
            return plan.pool_grad(Q, d["occ"], d["theta"], ws)[0]
    elif args.op == "pqe":
        det, sign = qf.excited_determinants("uccsd", no, no)

        def call():
            return plan.pqe_residuals(d["occ"], d["theta"], det, sign, ws)[0]
    elif args.op == "qk":
        del ws
        hp = qf.Plan(n, d["H"], d["H"], d["off"])
        states = torch.empty(5 << n, dtype=torch.complex128, device="cuda")
        print(f"Trotter step: {hp.apply_info()}", flush=True)

        def call():
            S, Hm, _ = hp.qk_matrices(d["occ"], 0.5, 3, 1, states)
            return float(Hm[0, 0].real)
    elif args.op == "sigma":
        del ws
        psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
        lam = torch.empty_like(psi)
        qf.prepare_state(psi, n, d["occ"])
        plan.apply(psi, d["theta"])

        def call():
            return plan.sigma(psi, lam)
    else:
        ops = qf.excitations("uccsd", no, no)
        t = qi.amplitudes(len(ops), seed, 0.2)
        S = qf.Sector(no, (no + 1) // 2, no // 2, ops, d["H"], d["off"])
        psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
        print(f"sector: dim {S.dim}, {S.groups} groups, {len(ops)} excitations", flush=True)

        if args.op == "sector_eg":
            del psi
            wsec = torch.empty(2 * S.dim, dtype=torch.complex128, device="cuda")

            def call():
                return S.energy_grad(d["occ"], t, wsec)[0]
        else:
            def call():
                S.prepare(psi, d["occ"])
                S.apply(psi, t)
                return S.energy(psi)
    E = call()
    best = float("inf")
    for _ in range(args.reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E = call()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    print(f"{args.op}: {best * 1e3:.2f} ms (best of {args.reps}), E = {E:.12f}", flush=True)
    _ = np


if __name__ == "__main__":
    main()
