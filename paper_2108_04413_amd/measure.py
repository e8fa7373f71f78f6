"""Time energy + adjoint gradient of one seeded UCCSD instance on the plan path.

    python -m paper_2108_04413_amd.measure --qubits 24 --reps 3

The instance is the autotuner's: n/2 spatial orbitals and n/2 electrons,
seeded random integrals, all UCCSD excitations, amplitudes ~ U[-0.2, 0.2].
Prints the plan's segment and class counts and the best of `reps` timed
evaluations (after one untimed).  Meant to run under a profiler, e.g.
`rocprofv3 --kernel-trace --stats -- python3 -m paper_2108_04413_amd.measure`.
"""
from __future__ import annotations

import argparse
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--qubits", type=int, default=24)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=None)
    args = ap.parse_args()

    import torch

    import paper_2108_04413_amd as qf
    from paper_2108_04413_amd.autotune import _instances
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import qf_inputs as qi

    n = args.qubits
    d = _instances(qf, qi, n, 1, args.seed if args.seed is not None else 7000 + n)[0]
    plan = qf.Plan(n, d["A"], d["H"], d["off"])
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    print(f"{n} qubits: {len(d['A'])} ansatz strings, {len(d['H'])} Hamiltonian strings in "
          f"{len(d['off']) - 1} groups; apply {plan.apply_info()}; energy {plan.info()}", flush=True)
    E, _ = plan.energy_grad(d["occ"], d["theta"], ws)
    best = float("inf")
    for _ in range(args.reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, _ = plan.energy_grad(d["occ"], d["theta"], ws)
        best = min(best, time.perf_counter() - t0)
    print(f"energy + gradient: {best * 1e3:.2f} ms (best of {args.reps}), E = {E:.12f}", flush=True)
    plan.close()


if __name__ == "__main__":
    main()
