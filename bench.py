"""Benchmark: state GB/s of the Pauli-exponential state-vector path on MI355X.

One step = one pass of the hot path on the 28-qubit workload (4 GiB
complex128 state): prepare the Hartree-Fock determinant, apply the 512
truncated-UCCD exponentials (4096 Pauli strings in 512 fused runs, applied
as 122 blocked passes over 2^12-amplitude sub-cubes), and evaluate
<psi|H|psi> over 55371 strings in 10466 flip-mask groups, fused into one
pass per class of groups that agree above bit 11 (2038 passes).  `value` =
algorithmic state bytes of the step / step time, inputs resident in HBM.

Algorithmic bytes (S = 2^n * 16 B), counted from the passes executed:
prepare S (write), each apply pass 2S (read + write), each energy pass S
(read).

Extra legs (each with the state bytes of the passes it executes):
- energy + adjoint gradient at 20 and 24 qubits (evals/s; the 24-qubit step
  is the second roofline entry);
- the 28-qubit workload in the particle-number / S_z restricted state
  vector (and a 32-qubit restricted reference energy);
- ADAPT pool gradients (Sec. 3.2), PQE residuals (Sec. 3.3) and the QK
  Trotter basis with its S and H matrices (Sec. 3.7) at 20 qubits;
- 256 batched instances in one persistent launch vs plain calls;
- the 10 000-request serving trace (2000 req/s) through continuous batching
  and through the plain serial path, plus an arrival-rate sweep;
- the CPU oracle timed on a bounded sample of the 28-qubit step (rank 0,
  N = 1), with a one-thread sample and the host's triad bandwidth.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "state GB/s vs HBM peak; energy+grad evals/s and p99 latency, batched vs plain"
HBM_PEAK_GBS = 8000.0


def profiled_traffic(kernel, version):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if that summary was taken on another library version."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if line.startswith("traffic_bytes_per_launch "):
                parts = line.split()
                if parts[1] == kernel and " ".join(parts[2:-1]) == version:
                    return float(parts[-1])
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def device_system(qf, qi, name):
    w, h, g = qi.workload(name)
    n = 2 * w["n_orb"]
    H, off, _ = qf.build_paulis("hamiltonian", w["n_orb"], w["n_elec"], h, g)
    if w["ansatz"] == "uccd_top":
        _, off_all, _ = qf.build_paulis("uccd", w["n_orb"], w["n_elec"])
        t_all = qi.amplitudes(len(off_all) - 1, w["seed"], w["t_scale"])
        A, aoff, kept = qf.build_paulis("uccd_top", w["n_orb"], w["n_elec"], t_rank=t_all, top_k=w["top_k"])
        t = t_all[kept]
    else:
        A, aoff, _ = qf.build_paulis("uccsd", w["n_orb"], w["n_elec"])
        t = qi.amplitudes(len(aoff) - 1, w["seed"], w["t_scale"])
    th = qf.ansatz_angles(A, aoff, t)
    return dict(w=w, n=n, n_elec=w["n_elec"], occ=(1 << w["n_elec"]) - 1, H=H, off=off, A=A, aoff=aoff,
                theta=th)


def cpu_baseline(qi, sysd, budget_s=20.0):
    """Oracle (plain C, OpenMP) on a bounded sample of the 28-qubit step."""
    from oracle import ansatz as an, core, hamiltonian as ham
    w, h, g = qi.workload("28q")
    n = sysd["n"]
    x, z, c, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    n_all = len(an.excitations(n, w["n_elec"], singles=False))
    t_all = qi.amplitudes(n_all, w["seed"], w["t_scale"])
    _, ax, az, ac, aoff, kept = an.build(w["n_orb"], w["n_elec"], "uccd_top", t_all, w["top_k"])
    th = an.angles(ac, aoff, t_all[kept])
    S = (1 << n) * 16
    psi = core.prepare(n, sysd["occ"])
    bytes_done, t_used = 0.0, 0.0
    # apply the first excitations term by term, then energy groups 1.. (skip
    # the 407-string diagonal group), until the time budget is spent
    n_terms = 0
    t0 = time.perf_counter()
    for mu in range(4):
        sl = slice(int(aoff[mu]), int(aoff[mu + 1]))
        core.apply_product(psi, n, ax[sl], az[sl], th[sl])
        n_terms += sl.stop - sl.start
    t_apply = time.perf_counter() - t0
    bytes_done += n_terms * 2 * S
    t_used += t_apply
    n_groups = 0
    g = 1
    while t_used < budget_s and g < len(goff) - 1:
        t0 = time.perf_counter()
        core.energy(psi, n, x, z, c, goff[g:g + 2])
        dt = time.perf_counter() - t0
        t_used += dt
        bytes_done += S
        n_groups += 1
        g += 1
    return {"value": bytes_done / t_used / 1e9, "unit": "GB/s", "cores": core.threads(), "kind": "oracle",
            "sample": f"28q: {n_terms} ansatz strings applied one pass each (4 excitations) + "
                      f"{n_groups} flip-mask groups of the energy (groups 1..{n_groups}), "
                      f"{t_used:.1f} s on the host; same algorithmic byte count as the GPU step"}


def core_threads():
    from oracle import core
    return core.threads()


def host_info():
    """CPU model and thread count of the host the oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def triad_gbps(n=1 << 25, reps=3):
    """Host STREAM-style triad a = b + s c over float64 arrays (numpy, one
    thread), in GB/s of 3 arrays moved; the best of reps."""
    b = np.ones(n)
    c = np.full(n, 2.0)
    a = np.empty(n)
    best = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        np.multiply(c, 3.0, out=a)
        np.add(a, b, out=a)
        dt = time.perf_counter() - t0
        best = max(best, 3 * 8 * n / dt / 1e9)
    return best


def oracle_group_sample(qf, qi, n_threads, budget_s):
    """Energy groups 1.. of the first 24-qubit served request's Hamiltonian on
    its reference state by the oracle's C core with n_threads threads, until
    budget_s is spent: GB/s of state read (one 256 MiB read per group)."""
    from oracle import core, hamiltonian as ham
    r = mix_recipe(qi, 24)
    h, g = qi.integrals(r["n_orb"], r["n_elec"], r["seed"])
    x, z, c, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    before = core.threads()
    core.set_threads(n_threads)
    try:
        psi = core.prepare(24, (1 << 12) - 1)
        t_used, k = 0.0, 1
        while t_used < budget_s and k < len(goff) - 1:
            t0 = time.perf_counter()
            core.energy(psi, 24, x, z, c, goff[k:k + 2])
            t_used += time.perf_counter() - t0
            k += 1
    finally:
        core.set_threads(before)
    return {"threads": n_threads, "workload": "24q served request, energy groups 1..", "groups": k - 1,
            "seconds": t_used, "GBps": (k - 1) * (1 << 24) * 16 / t_used / 1e9}


def oracle_energy_grad_20q(qi, reps=3):
    """The oracle's energy + adjoint gradient of the 20-qubit workload (C
    core, all host threads): median wall time of reps evaluations."""
    from oracle import ansatz as an, core, hamiltonian as ham
    w, h, g = qi.workload("20q")
    n = 2 * w["n_orb"]
    x, z, c, _ = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    _, ax, az, ac, aoff, _ = an.build(w["n_orb"], w["n_elec"], "uccsd")
    th = an.angles(ac, aoff, qi.amplitudes(len(aoff) - 1, w["seed"], w["t_scale"]))
    occ = an.reference_mask(w["n_elec"])
    ts = []
    e = None
    for _ in range(reps):
        t0 = time.perf_counter()
        e, _g = core.energy_grad(n, occ, ax, az, th, x, z, c)
        ts.append(time.perf_counter() - t0)
    med = float(np.median(ts))
    return {"threads": core.threads(), "workload": "20q energy + adjoint gradient (6700 ansatz, 14251 H strings)",
            "seconds": ts, "seconds_median": med, "evals_per_s": 1.0 / med, "energy": e}


def instance_from_recipe(qf, qi, r):
    h, g = qi.integrals(r["n_orb"], r["n_elec"], r["seed"])
    H, off, _ = qf.build_paulis("hamiltonian", r["n_orb"], r["n_elec"], h, g)
    A, aoff, _ = qf.build_paulis("uccsd", r["n_orb"], r["n_elec"])
    t = qi.amplitudes(len(aoff) - 1, r["seed"], r["t_scale"])
    return dict(n=2 * r["n_orb"], n_elec=r["n_elec"], occ=(1 << r["n_elec"]) - 1, H=H, off=off, A=A, aoff=aoff,
                theta=qf.ansatz_angles(A, aoff, t))


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def batched_leg(qf, qi, count=256, reps=2):
    """256 (molecule, theta) instances of 12-22 qubits: one persistent graph
    launch vs the plain path (one plan call per instance, in order)."""
    import torch
    t0 = time.perf_counter()
    insts = [instance_from_recipe(qf, qi, r) for r in qi.batched_instances(count)]
    log(f"batched: built {count} instances in {time.perf_counter() - t0:.1f} s")
    thetas = [d["theta"] for d in insts]
    B = qf.Batch(insts)
    info = B.info()
    B.run(thetas, use_graph=True)
    tb = []
    for _ in range(reps):
        t0 = time.perf_counter()
        Eb, gb = B.run(thetas, use_graph=True)
        tb.append(time.perf_counter() - t0)
    t_batch = min(tb)
    log(f"batched: {count} energy+grad in {t_batch * 1e3:.1f} ms (grid {info['grid']})")
    # per-instance latency: the same launch with each instance published to a
    # host mailbox as soon as its team finishes (largest instances run first)
    Ec, gc, t_done = B.run_completion(thetas)
    same = bool(np.array_equal(Ec, Eb) and all(np.array_equal(a, b) for a, b in zip(gc, gb)))
    log(f"batched (mailbox launch): p50 {pct(t_done, 50) * 1e3:.1f} ms, p99 {pct(t_done, 99) * 1e3:.1f} ms, "
        f"identical to the graph launch: {same}")
    B.close()
    plans = [qf.Plan(d["n"], d["A"], d["H"], d["off"]) for d in insts]
    ws = torch.empty(2 << max(d["n"] for d in insts), dtype=torch.complex128, device="cuda")
    for d, p in list(zip(insts, plans))[:8]:
        p.energy_grad(d["occ"], d["theta"], ws)
    lat, done = [], []
    dE = dG = 0.0
    t_start = time.perf_counter()
    for i, (d, p) in enumerate(zip(insts, plans)):
        t0 = time.perf_counter()
        e, g = p.energy_grad(d["occ"], d["theta"], ws)
        t1 = time.perf_counter()
        lat.append(t1 - t0)
        done.append(t1 - t_start)
        dE = max(dE, abs(e - Eb[i]))
        dG = max(dG, float(np.max(np.abs(g - gb[i]))) if len(g) else 0.0)
    t_plain = time.perf_counter() - t_start
    log(f"plain: {count} energy+grad in {t_plain * 1e3:.1f} ms; max |dE| {dE:.2e}, max |dgrad| {dG:.2e}")
    for p in plans:
        p.close()
    del ws
    torch.cuda.empty_cache()
    return {"batched_evals_per_s": count / t_batch, "plain_evals_per_s": count / t_plain,
            "batched_ms": t_batch * 1e3, "plain_ms": t_plain * 1e3, "speedup": t_plain / t_batch,
            "batched_latency_ms_p50": pct(t_done, 50) * 1e3, "batched_latency_ms_p99": pct(t_done, 99) * 1e3,
            "batched_mailbox_launch_identical": same,
            "plain_latency_from_submit_ms_p50": pct(done, 50) * 1e3,
            "plain_latency_from_submit_ms_p99": pct(done, 99) * 1e3,
            "plain_per_call_ms_p50": pct(lat, 50) * 1e3, "plain_per_call_ms_p99": pct(lat, 99) * 1e3,
            "max_abs_dE_batched_vs_plain": dE, "max_abs_dgrad_batched_vs_plain": dG,
            "teams": sorted(set(zip((d["n"] for d in insts), info["team"]))), "grid": info["grid"]}


def _reset(reqs):
    for r in reqs:
        r.E = r.grad = r.t_admit = r.t_done = r.error = None
        r.team, r.solo = 0, False


def serving_leg(qf, qi, n_req=10000, plain_req=10000, sweep=(25.0, 50.0, 100.0), sweep_req=200):
    """The Poisson trace of n_req requests (2000 req/s, 12-24 qubits):
    continuous batching vs the plain one-at-a-time path on the first
    plain_req of the same requests; then continuous batching on the first
    sweep_req requests re-timed to lower arrival rates (context)."""
    from paper_2108_04413_amd import serve
    trace = qi.serving_trace(10000)[:n_req]
    t0 = time.perf_counter()
    reqs = serve.make_requests(qf, qi, trace)
    log(f"serving: built {n_req} requests in {time.perf_counter() - t0:.1f} s")
    srv = serve.Server(arena_bytes=48 << 30, slots=2, max_wave=64, solo_qubits=serve.SOLO_QUBITS)
    st_b = srv.serve(reqs)
    srv.close()
    log(f"serving (continuous batching): {st_b}")
    E_b = [r.E for r in reqs[:plain_req]]
    plain = reqs[:plain_req]
    _reset(plain)
    st_p = serve.serve_plain(plain, max(r.n for r in plain))
    log(f"serving (plain serial, first {plain_req}): {st_p}")
    dE = max(abs(a - b.E) for a, b in zip(E_b, plain) if a is not None and b.E is not None)
    mix = {}
    for r in reqs:
        mix[r.n] = mix.get(r.n, 0) + 1
    rates = []
    for rate in sweep:
        sub = reqs[:sweep_req]
        _reset(sub)
        arr0 = [r.arrival for r in sub]
        gaps = qi.serving_trace(sweep_req, rate=rate)  # same draws, arrivals scaled to the rate
        for r, (t, _) in zip(sub, gaps):
            r.arrival = float(t)
        srv = serve.Server(arena_bytes=48 << 30, slots=2, max_wave=64, solo_qubits=serve.SOLO_QUBITS)
        st = srv.serve(sub)
        srv.close()
        for r, a in zip(sub, arr0):
            r.arrival = a
        rates.append({"offered_req_per_s": rate, "requests": sweep_req,
                      **{k: st[k] for k in ("throughput_req_per_s", "latency_ms_p50", "latency_ms_p99", "failed")}})
        log(f"serving sweep at {rate} req/s: {rates[-1]}")
    return {"requests": n_req, "offered_rate_req_per_s": 2000.0, "qubit_mix": dict(sorted(mix.items())),
            "solo_qubits": serve.SOLO_QUBITS,
            "continuous_batching": st_b, "plain_serial": dict(st_p, requests_replayed=plain_req),
            "throughput_ratio": st_b["throughput_req_per_s"] / st_p["throughput_req_per_s"],
            "max_abs_dE_batched_vs_plain": dE, "rate_sweep_continuous_batching": rates}


def mix_recipe(qi, nq):
    """The first request of nq qubits in the serving trace."""
    for _, r in qi.serving_trace(10000):
        if 2 * r["n_orb"] == nq:
            return r
    raise ValueError(nq)


def eg_leg(qf, qi, name, reps=5):
    """Energy + adjoint gradient of one workload on the plan kernels, with
    the state bytes of the passes executed: prepare S, each forward segment
    2S, sigma (classes + 1) S read + S write, each sweep segment 4S."""
    import torch
    if name == "24q":
        r = mix_recipe(qi, 24)
        d = instance_from_recipe(qf, qi, r)
    else:
        d = device_system(qf, qi, name)
    n = d["n"]
    S = (1 << n) * 16
    p = qf.Plan(n, d["A"], d["H"], d["off"])
    ws = torch.empty(2 << n, dtype=torch.complex128, device="cuda")
    p.energy_grad(d["occ"], d["theta"], ws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        e, g = p.energy_grad(d["occ"], d["theta"], ws)
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    ai, gi = p.apply_info(), p.grad_info()
    nbytes = S + 2 * S * ai["passes"] + (gi["sigma_passes"] + 2) * S + 4 * S * gi["sweep_passes"]
    out = {"ms": dt * 1e3, "evals_per_s": 1.0 / dt, "energy": e, "apply_passes": ai["passes"],
           "sigma_passes": gi["sigma_passes"], "sweep_passes": gi["sweep_passes"], "state_bytes": nbytes,
           "GBps": nbytes / dt / 1e9, "frac_of_hbm_peak": nbytes / dt / 1e9 / HBM_PEAK_GBS}
    log(f"energy+grad {name}: {out}")
    return out, (d, p, ws)


def pool_leg(qf, qi, d, p, ws, reps=3):
    """ADAPT pool gradients (Sec. 3.2) on the state of d: forward, sigma,
    then one read-only pass (2S) per pool-sweep segment."""
    import torch
    n = d["n"]
    S = (1 << n) * 16
    pool, poff, _ = qf.build_paulis("gsd_pool", n // 2, 0)
    Q = qf.PoolPlan(n, pool, poff)
    p.pool_grad(Q, d["occ"], d["theta"], ws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        e, g = p.pool_grad(Q, d["occ"], d["theta"], ws)
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    ai, gi, qi_ = p.apply_info(), p.grad_info(), Q.grad_info()
    nbytes = S + 2 * S * ai["passes"] + (gi["sigma_passes"] + 2) * S + 2 * S * qi_["sweep_passes"]
    out = {"ms": dt * 1e3, "pool_members": len(poff) - 1, "pool_strings": len(pool),
           "pool_sweep_passes": qi_["sweep_passes"], "state_bytes": nbytes, "GBps": nbytes / dt / 1e9,
           "max_abs_g": float(np.max(np.abs(g)))}
    log(f"pool gradients {n}q: {out}")
    Q.close()
    return out


def pqe_leg(qf, qi, d, p, ws, reps=3):
    """PQE residuals (Sec. 3.3): forward, sigma, the inverse pass on lambda,
    a gather: S + 4S per segment pass + sigma."""
    import torch
    n = d["n"]
    S = (1 << n) * 16
    det, sign = qf.excited_determinants("uccsd", n // 2, d["n_elec"])
    p.pqe_residuals(d["occ"], d["theta"], det, sign, ws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        e, r = p.pqe_residuals(d["occ"], d["theta"], det, sign, ws)
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    ai, gi = p.apply_info(), p.grad_info()
    nbytes = S + 4 * S * ai["passes"] + (gi["sigma_passes"] + 2) * S
    out = {"ms": dt * 1e3, "residuals": len(det), "state_bytes": nbytes, "GBps": nbytes / dt / 1e9,
           "max_abs_r": float(np.max(np.abs(r)))}
    log(f"PQE residuals {n}q: {out}")
    return out


def sector_pairs(n_orb, na, nb, H, off):
    """Sum over the groups kept by the sector of the sector determinants whose
    partner under the group's flips is in the sector (exact counts)."""
    from math import comb
    tot = 0
    for g in range(len(off) - 1):
        x = int(H["x"][off[g]])
        ka = bin(sum(((x >> (2 * j)) & 1) << j for j in range(n_orb))).count("1")
        kb = bin(sum(((x >> (2 * j + 1)) & 1) << j for j in range(n_orb))).count("1")
        if ka % 2 or kb % 2:
            continue
        fa = comb(ka, ka // 2) * comb(n_orb - ka, na - ka // 2)
        fb = comb(kb, kb // 2) * comb(n_orb - kb, nb - kb // 2)
        tot += fa * fb
    return tot


def sector_leg(qf, qi, s28, e28):
    """The 28-qubit workload in the (7, 7) sector: reference, the 512
    truncated-UCCD factors as determinant-pair rotations, the energy; the
    energy + dE/dt of the 24-qubit served request in its (6, 6) sector; and
    the reference energy of a 32-qubit (8, 8) sector."""
    import torch
    w, h, g = qi.workload("28q")
    n_d = len(qf.excitations("uccd", 14, 14))
    t_all = qi.amplitudes(n_d, w["seed"], w["t_scale"])
    _, _, kept = qf.build_paulis("uccd_top", 14, 14, t_rank=t_all, top_k=w["top_k"])
    ops = qf.excitations("uccd_top", 14, 14, t_rank=t_all, top_k=w["top_k"])
    S = qf.Sector(14, 7, 7, ops, s28["H"], s28["off"])
    psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
    S.prepare(psi, s28["occ"])
    S.apply(psi, t_all[kept])
    S.energy(psi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.prepare(psi, s28["occ"])
    S.apply(psi, t_all[kept])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    e = S.energy(psi)
    t2 = time.perf_counter()
    pairs = sector_pairs(14, 7, 7, s28["H"], s28["off"])
    ebytes = 16 * (S.dim + pairs)
    out = {"dim": S.dim, "state_MiB": S.dim * 16 / 2 ** 20, "groups": S.groups, "excitations": len(ops),
           "prepare_apply_ms": (t1 - t0) * 1e3, "energy_ms": (t2 - t1) * 1e3, "energy": e,
           "abs_dE_vs_full_space": abs(e - e28), "energy_bytes": ebytes, "energy_GBps": ebytes / (t2 - t1) / 1e9}
    del psi
    S.close()
    torch.cuda.empty_cache()
    # energy + gradient (dE/dt per excitation) of the 24-qubit served request
    r = mix_recipe(qi, 24)
    d = instance_from_recipe(qf, qi, r)
    ops = qf.excitations("uccsd", r["n_orb"], r["n_elec"])
    t24 = qi.amplitudes(len(ops), r["seed"], r["t_scale"])
    S = qf.Sector(r["n_orb"], (r["n_elec"] + 1) // 2, r["n_elec"] // 2, ops, d["H"], d["off"])
    ws = torch.empty(2 * S.dim, dtype=torch.complex128, device="cuda")
    S.energy_grad(d["occ"], t24, ws)
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        e24, g24 = S.energy_grad(d["occ"], t24, ws)
        ts.append(time.perf_counter() - t0)
    out["energy_grad_24q"] = {"dim": S.dim, "excitations": len(ops), "ms": float(np.median(ts)) * 1e3,
                              "evals_per_s": 1.0 / float(np.median(ts)), "energy": e24}
    del ws
    S.close()
    h, g = qi.integrals(16, 16, 1132)
    H, off, _ = qf.build_paulis("hamiltonian", 16, 16, h, g)
    S = qf.Sector(16, 8, 8, None, H, off)
    psi = torch.empty(S.dim, dtype=torch.complex128, device="cuda")
    S.prepare(psi, (1 << 16) - 1)
    t0 = time.perf_counter()
    e32 = S.energy(psi)
    t1 = time.perf_counter()
    pairs = sector_pairs(16, 8, 8, H, off)
    out["sector_32q"] = {"dim": S.dim, "state_GiB": S.dim * 16 / 2 ** 30, "groups": S.groups,
                         "energy_ms": (t1 - t0) * 1e3, "energy_reference": e32,
                         "energy_GBps": 16 * (S.dim + pairs) / (t1 - t0) / 1e9}
    del psi
    S.close()
    torch.cuda.empty_cache()
    log(f"sector: {out}")
    return out


def qk_leg(qf, qi, name="20q", dt_=0.5, s_=3, r_=1):
    """QK basis (Sec. 3.7): s Trotter evolutions of r steps over H's strings,
    s + 1 sigma passes and the S, H inner products."""
    import torch
    w, h, g = qi.workload(name)
    n = 2 * w["n_orb"]
    S = (1 << n) * 16
    H, off, _ = qf.build_paulis("hamiltonian", w["n_orb"], w["n_elec"], h, g)
    p = qf.Plan(n, H, H, off)
    states = torch.empty((s_ + 2) << n, dtype=torch.complex128, device="cuda")
    p.qk_matrices((1 << w["n_elec"]) - 1, dt_, s_, r_, states)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Sm, Hm, _ = p.qk_matrices((1 << w["n_elec"]) - 1, dt_, s_, r_, states)
    dt = time.perf_counter() - t0
    ai, gi = p.apply_info(), p.grad_info()
    J = s_ + 1
    nbytes = J * S + s_ * r_ * 2 * S * ai["passes"] + J * (gi["sigma_passes"] + 2) * S + J * (J + 2) * S
    from oracle import krylov  # the generalized eigenproblem is the caller's (host)
    out = {"ms": dt * 1e3, "s": s_, "r": r_, "dt": dt_, "trotter_step_passes": ai["passes"],
           "hamiltonian_strings": len(H), "state_bytes": nbytes, "GBps": nbytes / dt / 1e9,
           "qk_lowest_root": krylov.qk_energy(Sm, Hm), "H00": float(Hm[0, 0].real)}
    log(f"QK {name}: {out}")
    del states
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-20q", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sector", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the serving trace replayed (default: all 10 000)")
    ap.add_argument("--plain-requests", type=int, default=10000,
                    help="of those, requests replayed through the plain serial path")
    ap.add_argument("--calib", action="store_true",
                    help="run one torch copy of one state (4 GiB) first: a plain copy kernel of known "
                         "size for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the state-vector path "
              "runs on a single MI355X here).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2108_04413_amd as qf
    import qf_inputs as qi

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.calib:
        src = torch.zeros(1 << 28, dtype=torch.complex128, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        log("calibration copy of 4 GiB done")
    log("building 28q tables")
    s28 = device_system(qf, qi, "28q")
    n = s28["n"]
    S = (1 << n) * 16
    G = len(s28["off"]) - 1
    plan = qf.Plan(n, s28["A"], s28["H"], s28["off"])
    ainfo = plan.apply_info()
    passes = ainfo["passes"]  # state passes of the blocked apply
    pinfo = plan.info()
    e_passes = pinfo["energy_passes"]  # one state read per class of groups
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    step_bytes = S + passes * 2 * S + e_passes * S
    energy_bytes = e_passes * S

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t_step, t_energy, t_apply = [], [], []
    E = None
    for it in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        ev[0].record(stream)
        qf.prepare_state(psi, n, s28["occ"])
        plan.apply(psi, s28["theta"])
        ev[1].record(stream)
        ev[2].record(stream)
        E = plan.energy(psi)
        ev[3].record(stream)
        torch.cuda.synchronize()
        ta = ev[0].elapsed_time(ev[1])
        te = ev[2].elapsed_time(ev[3])
        log(f"step {it} ({'warmup' if it < args.warmup else 'timed'}): prep+apply {ta:.1f} ms, "
            f"energy {te:.1f} ms, E = {E:.12f}")
        if it >= args.warmup:
            t_apply.append(ta)
            t_energy.append(te)
            t_step.append(ta + te)
    ms = float(np.mean(t_step))
    value = step_bytes / (ms * 1e-3) / 1e9
    traffic = profiled_traffic("k_energy_stream", qf.__version__)
    e_ms = float(np.mean(t_energy))
    achieved = energy_bytes / (e_ms * 1e-3) / 1e9
    # the one-pass-per-group energy kernel on the same state, for comparison
    plan.set_energy_tile(0, False)
    ev[2].record(stream)
    E0 = plan.energy(psi)
    ev[3].record(stream)
    torch.cuda.synchronize()
    e0_ms = ev[2].elapsed_time(ev[3])
    log(f"untiled energy (one pass per group): {e0_ms:.1f} ms, E = {E0:.12f}")
    del psi
    torch.cuda.empty_cache()
    sector = None if args.no_sector else sector_leg(qf, qi, s28, E)

    extra = {"energy_28q": E, "apply_ms": float(np.mean(t_apply)), "energy_ms": e_ms,
             "apply_passes": passes, "apply_runs": ainfo["runs"], "apply_block_bits": ainfo["block_bits"],
             "energy_groups": G, "energy_passes": e_passes,
             "energy_tile_bits": pinfo["tile_bits"],
             "apply_GBps": (S + passes * 2 * S) / (np.mean(t_apply) * 1e-3) / 1e9,
             "energy_untiled_ms": e0_ms, "energy_untiled_E": E0,
             "energy_untiled_GBps": G * S / (e0_ms * 1e-3) / 1e9,
             "energy_speedup_vs_untiled": e0_ms / e_ms}
    if sector is not None:
        extra["sector_28q"] = sector

    if not args.no_20q:
        eg = {}
        for name in ("20q", "24q"):
            res, (d, p, ws) = eg_leg(qf, qi, name)
            eg[name] = res
            if name == "20q":
                extra["pool_gradients_20q"] = pool_leg(qf, qi, d, p, ws)
                extra["pqe_residuals_20q"] = pqe_leg(qf, qi, d, p, ws)
            p.close()
            del ws
            torch.cuda.empty_cache()
        extra["energy_grad"] = eg
        extra["qk_20q"] = qk_leg(qf, qi, "20q")

    if not args.no_batch:
        log("batched leg (256 instances, 12-22 qubits)")
        extra["batched_256"] = batched_leg(qf, qi)

    if not args.no_serve:
        log(f"serving leg ({args.serve_requests} requests of the 10k trace)")
        extra["serving"] = serving_leg(qf, qi, n_req=args.serve_requests,
                                       plain_req=min(args.serve_requests, args.plain_requests))

    line = {"metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "28q: 14 orbitals / 14 electrons, seeded random integrals, "
                                   "UCCD top-512 ansatz (4096 strings), H of 55371 strings / 10466 groups, "
                                   "complex128 2^28 state; step = prepare + apply (blocked passes) + "
                                   "energy (tiled passes)",
                       "n_qubits": n, "state_bytes": S, "step_algorithmic_bytes": step_bytes},
            "roofline": {"bound": "hbm", "kernel": "k_energy_stream", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                         "achieved_from_counters": None if traffic is None else traffic / (e_ms * 1e-3) / 1e9,
                         "bytes_per_launch": energy_bytes, "launch_ms": e_ms},
            "extra": extra}
    if "energy_grad" in extra:
        r24 = extra["energy_grad"]["24q"]
        line["roofline_energy_grad"] = {
            "bound": "hbm", "kernel": "energy + gradient step at 24 qubits (k_apply_block, k_sigma_stream, "
                                      "k_adjoint_block, k_grad_reduce)",
            "achieved": r24["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": r24["GBps"] / HBM_PEAK_GBS,
            "traffic": None, "bytes_per_step": r24["state_bytes"], "step_ms": r24["ms"]}
    if not args.no_cpu:
        log("cpu baseline (oracle on a bounded sample)")
        cb = cpu_baseline(qi, s28)
        model, nthreads = host_info()
        one = oracle_group_sample(qf, qi, 1, 5.0)
        allt = oracle_group_sample(qf, qi, core_threads(), 5.0)
        cb.update({"host_cpu": model, "host_threads": nthreads, "one_thread_24q": one, "all_threads_24q": allt,
                   "host_triad_GBps_one_thread": triad_gbps(), "oracle_energy_grad_20q": oracle_energy_grad_20q(qi)})
        log(f"cpu baseline: {cb}")
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
