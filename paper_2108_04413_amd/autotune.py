"""Autotuner for the persistent batched kernel.

Two kinds of knobs are tuned per qubit count.

Plan tiles (`plan` in the table): the sub-cube size B of the blocked apply
(and of the reverse sweep, min(B, 11)) and the tile of the energy passes
(2^L amplitudes, merged lo-terms).  For each n the tuner builds one seeded
instance and times energy + gradient for B in {10, 11, 12} and the energy
for L in {10, 11, 12}; api.Plan applies the winners when the table matches
the device.

The schedule knob of qf_batch is the team size W(n): how many workgroups
cooperate on one instance of n qubits.  Small W runs many instances side by
side (each pass is short and stays in one CU's cache); large W spreads one
instance over the chip (needed when few large instances remain).  For each
qubit count the tuner builds `count` seeded instances of that size, runs one
batch launch per candidate W (powers of two up to the limit the library
clamps to) and keeps the fastest.  The table is written as JSON
{"arch": ..., "team": {n: W}, "ms": {n: {W: ms}}} and picked up by
api.Batch when it matches the running device.

The per-size search sees one size at a time, while a mixed batch shares the
grid between sizes: a team that is fastest for 43 instances of one size can
slow the mixed launch.  `--what mixed` therefore refines the table on the
mixed batched configuration (`qf_inputs.batched_instances`): for each size
in turn it tries half and twice the team and keeps a change only when the
whole launch gets faster (coordinate descent from the per-size table).

    python -m paper_2108_04413_amd.autotune --out tuned_gfx950.json
    python -m paper_2108_04413_amd.autotune --what mixed --merge
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned_gfx950.json")


def device_arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def load_table(arch: str | None = None) -> dict | None:
    """The committed team table for this architecture, or None."""
    if not os.path.exists(TABLE):
        return None
    with open(TABLE) as f:
        tab = json.load(f)
    if arch is not None and tab.get("arch") != arch:
        return None
    return {int(k): int(v) for k, v in tab["team"].items()}


def _instances(qf, qi, n_qubits: int, count: int, seed0: int):
    out = []
    for i in range(count):
        n_orb = n_qubits // 2
        seed = seed0 + i
        h, g = qi.integrals(n_orb, n_orb, seed)
        H, off, _ = qf.build_paulis("hamiltonian", n_orb, n_orb, h, g)
        A, aoff, _ = qf.build_paulis("uccsd", n_orb, n_orb)
        t = qi.amplitudes(len(aoff) - 1, seed, 0.2)
        out.append(dict(n=n_qubits, occ=(1 << n_orb) - 1, H=H, off=off, A=A,
                        theta=qf.ansatz_angles(A, aoff, t)))
    return out


def tune(ns=(12, 14, 16, 18, 20, 22, 24), count: int = 43, reps: int = 2, max_team: int = 256,
         log=print) -> dict:
    import paper_2108_04413_amd as qf
    sys.path.insert(0, os.path.dirname(HERE))
    import qf_inputs as qi

    result = {"arch": device_arch(), "count": count, "team": {}, "ms": {}}
    for n in ns:
        insts = _instances(qf, qi, n, count, 9000 + 100 * n)
        thetas = [d["theta"] for d in insts]
        tiles = max(1, (1 << (n - 1)) // 1024)  # the library's clamp: one 2^11 sub-cube per member
        # a single workgroup per instance is hopeless beyond 20 qubits
        w_min = 1 << max(0, n - 20)
        cands = [w for w in (1, 2, 4, 8, 16, 32, 64, 128, 256) if w_min <= w <= min(tiles, max_team)]
        times = {}
        for w in cands:
            B = qf.Batch(insts, team=[w] * count)
            if B.info()["team"][0] != w:  # clamped by the grid
                B.close()
                continue
            B.run(thetas, use_graph=True)  # capture + warm
            best = float("inf")
            for _ in range(reps):
                t0 = time.perf_counter()
                B.run(thetas, use_graph=True)
                best = min(best, time.perf_counter() - t0)
            B.close()
            times[w] = best * 1e3
            log(f"autotune n={n} W={w}: {times[w]:.2f} ms for {count} instances")
        wbest = min(times, key=times.get)
        result["team"][str(n)] = int(wbest)
        result["ms"][str(n)] = {str(k): v for k, v in times.items()}
        log(f"autotune n={n}: W={wbest}")
    return result


def tune_mixed(team: dict, count: int = 256, reps: int = 2, max_team: int = 256, log=print) -> dict:
    """Refine per-size teams on the mixed batch: for each size, try W / 2
    and 2 W and keep a change that makes the whole launch faster."""
    import paper_2108_04413_amd as qf
    sys.path.insert(0, os.path.dirname(HERE))
    import qf_inputs as qi

    insts = []
    for r in qi.batched_instances(count):
        h, g = qi.integrals(r["n_orb"], r["n_elec"], r["seed"])
        H, off, _ = qf.build_paulis("hamiltonian", r["n_orb"], r["n_elec"], h, g)
        A, aoff, _ = qf.build_paulis("uccsd", r["n_orb"], r["n_elec"])
        t = qi.amplitudes(len(aoff) - 1, r["seed"], r["t_scale"])
        insts.append(dict(n=2 * r["n_orb"], occ=(1 << r["n_elec"]) - 1, H=H, off=off, A=A,
                          theta=qf.ansatz_angles(A, aoff, t)))
    thetas = [d["theta"] for d in insts]
    sizes = sorted({d["n"] for d in insts})

    def launch_ms(tab):
        B = qf.Batch(insts, team=[tab.get(d["n"], 0) for d in insts])
        B.run(thetas, use_graph=True)  # capture + warm
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            B.run(thetas, use_graph=True)
            best = min(best, time.perf_counter() - t0)
        B.close()
        return best * 1e3

    cur = {n: int(team.get(n, 0)) for n in sizes}
    t_cur = launch_ms(cur)
    log(f"autotune mixed: start {cur}: {t_cur:.1f} ms for {count} instances")
    trials = {}
    for n in sorted(sizes, reverse=True):
        if cur[n] <= 0:
            continue
        for w in (cur[n] // 2, cur[n] * 2):
            # the library's clamp: one 2^11 sub-cube per member
            if w < 1 or w > max_team or w > max(1, (1 << (n - 1)) // 1024):
                continue
            tab = dict(cur)
            tab[n] = w
            t = launch_ms(tab)
            trials[f"{n}:{w}"] = t
            log(f"autotune mixed: n={n} W={w}: {t:.1f} ms")
            # keep a change only if it clears the launch-to-launch spread
            if t < 0.98 * t_cur:
                cur, t_cur = tab, t
                log(f"autotune mixed: keep n={n} W={w}")
    return {"team": {str(n): w for n, w in cur.items()}, "mixed_ms": {"final": t_cur, "trials": trials}}


def load_plan_table(arch: str | None = None) -> dict:
    """Tuned plan tiles {n: {"block_bits": B, "energy_tile": L}} for this
    architecture ({} if none)."""
    if not os.path.exists(TABLE):
        return {}
    with open(TABLE) as f:
        tab = json.load(f)
    if arch is not None and tab.get("arch") != arch:
        return {}
    return {int(k): v for k, v in tab.get("plan", {}).items()}


def tune_plan(ns=(12, 14, 16, 18, 20, 22, 24), reps: int = 3, log=print) -> dict:
    """Per n: the blocked-apply sub-cube bits (timed on energy + gradient,
    which also runs the reverse sweep) and the energy tile bits (timed on
    the energy of the prepared state)."""
    import torch

    import paper_2108_04413_amd as qf
    sys.path.insert(0, os.path.dirname(HERE))
    import qf_inputs as qi

    def best_of(fn):
        fn()
        t = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t = min(t, time.perf_counter() - t0)
        return t * 1e3

    out, ms = {}, {}
    for n in ns:
        d = _instances(qf, qi, n, 1, 8000 + n)[0]
        plan = qf.Plan(n, d["A"], d["H"], d["off"], tuned=False)
        ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
        psi = ws[:1 << n]
        tb = {}
        for B in (10, 11, 12):
            if B > n:
                continue
            plan.set_block_bits(B)
            tb[B] = best_of(lambda: plan.energy_grad(d["occ"], d["theta"], ws))
            log(f"autotune plan n={n} block bits {B}: energy + gradient {tb[B]:.3f} ms")
        bbest = min(tb, key=tb.get)
        plan.set_block_bits(bbest)
        qf.prepare_state(psi, n, d["occ"])
        plan.apply(psi, d["theta"])
        te = {}
        for L in (10, 11, 12):
            if L >= n:
                continue
            plan.set_energy_tile(L, True)
            te[L] = best_of(lambda: plan.energy(psi))
            log(f"autotune plan n={n} energy tile {L}: energy {te[L]:.3f} ms")
        lbest = min(te, key=te.get) if te else 0
        out[str(n)] = {"block_bits": int(bbest), "energy_tile": int(lbest)}
        ms[str(n)] = {"energy_grad": {str(k): v for k, v in tb.items()},
                      "energy": {str(k): v for k, v in te.items()}}
        log(f"autotune plan n={n}: block bits {bbest}, energy tile {lbest}")
        del ws, psi
        plan.close()
        torch.cuda.empty_cache()
    return {"plan": out, "plan_ms": ms}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--count", type=int, default=43)
    ap.add_argument("--ns", default="12,14,16,18,20,22,24")
    ap.add_argument("--merge", action="store_true", help="update the existing table instead of replacing it")
    ap.add_argument("--what", default="all", choices=["all", "team", "plan", "mixed"])
    args = ap.parse_args()
    ns = tuple(int(v) for v in args.ns.split(","))
    say = lambda m: print(m, flush=True)  # noqa: E731
    res = {"arch": device_arch(), "count": args.count, "team": {}, "ms": {}}
    if args.what in ("all", "team"):
        res.update(tune(ns, count=args.count, log=say))
    if args.what in ("all", "plan"):
        res.update(tune_plan(ns, log=say))
    if args.what in ("all", "mixed"):
        start = res["team"] if res["team"] else {}
        if not start and os.path.exists(args.out):
            with open(args.out) as f:
                start = json.load(f).get("team", {})
        res.update(tune_mixed({int(k): int(v) for k, v in start.items()}, log=say))
    if args.merge and os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
        for key in ("team", "ms", "plan", "plan_ms", "mixed_ms"):
            if key in res:
                old.setdefault(key, {}).update(res[key])
        res = old
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({"team": res.get("team"), "plan": res.get("plan")}))


if __name__ == "__main__":
    main()
