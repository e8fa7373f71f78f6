"""Write oracle reference values for the 20- and 28-qubit workloads and for
the largest instances of the batched and served mixes.

Calls only the CPU oracle (oracle/) and the seeded input module.  Usage:

    python tests/golden/make_golden.py 20q       # ~1 min on 8 cores
    python tests/golden/make_golden.py 28q       # hours on 8 cores
    python tests/golden/make_golden.py batch22q  # ~5 min: first 22-qubit instance of the batched mix
    python tests/golden/make_golden.py serve24q  # ~1 h: first 24-qubit request of the serving trace
    python tests/golden/make_golden.py 20q_pool  # ADAPT pool gradients on the 20-qubit final state
    python tests/golden/make_golden.py 20q_pqe   # PQE residuals of the 20-qubit workload
    python tests/golden/make_golden.py 20q_qk    # QK matrices (dt 0.5, s 2, r 1) of the 20-qubit Hamiltonian

Each output JSON holds the recipe, the energy, sampled final-state
amplitudes, and (all but 28q) the full gradient dE/dtheta and dE/dt.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import qf_inputs as qi  # noqa: E402
from oracle import ansatz as an, core, hamiltonian as ham  # noqa: E402


def sample_indices(n, psi, seed, count=256):
    rng = np.random.default_rng([seed, 9])
    rand = rng.integers(0, 1 << n, count)
    top = np.argsort(-np.abs(psi), kind="stable")[:count]
    return np.unique(np.concatenate([rand, top]))


def mix_recipe(name):
    """Recipe of the first instance of the named size in the batched mix
    (256 instances) or the serving trace (10 000 requests)."""
    if name.startswith("batch"):
        nq = int(name[5:-1])
        idx, rcp = next((i, r) for i, r in enumerate(qi.batched_instances(256)) if 2 * r["n_orb"] == nq)
    else:
        nq = int(name[5:-1])
        idx, (_, rcp) = next((j, tr) for j, tr in enumerate(qi.serving_trace(10000)) if 2 * tr[1]["n_orb"] == nq)
    w = dict(rcp)
    w["mix_index"] = idx
    return w, *qi.integrals(w["n_orb"], w["n_elec"], w["seed"])


def system(name):
    w, h, g = mix_recipe(name) if name.startswith(("batch", "serve")) else qi.workload(name)
    n = 2 * w["n_orb"]
    hx, hz, hc, goff = ham.group_by_flip_mask(ham.qubit_hamiltonian(h, g))
    if w["ansatz"] == "uccd_top":
        n_all = len(an.excitations(n, w["n_elec"], singles=False))
        t_all = qi.amplitudes(n_all, w["seed"], w["t_scale"])
        excs, ax, az, ac, off, kept = an.build(w["n_orb"], w["n_elec"], "uccd_top", t_all, w["top_k"])
        t = t_all[kept]
    else:
        excs, ax, az, ac, off, kept = an.build(w["n_orb"], w["n_elec"])
        t = qi.amplitudes(len(excs), w["seed"], w["t_scale"])
    th = an.angles(ac, off, t)
    return w, n, an.reference_mask(w["n_elec"]), (hx, hz, hc, goff), (ax, az, ac, off, th, t)


def main_pool(name):
    """ADAPT pool gradients (Sec. 3.2) on the final state of a workload."""
    from oracle import adapt
    base = name[:-len("_pool")]
    t0 = time.time()
    w, n, occ, (hx, hz, hc, goff), (ax, az, ac, off, th, t) = system(base)
    ops, px, pz, pc, poff = adapt.pool_terms(n)
    print(f"{name}: pool of {len(ops)} operators, {len(px)} strings", flush=True)
    psi = core.apply_product(core.prepare(n, occ), n, ax, az, th)
    lam = core.sigma(psi, n, hx, hz, hc)
    g = core.pool_grad(psi, lam, n, px, pz, pc, poff)
    out = dict(workload=base, recipe=w, n_qubits=n, occ_mask=occ, n_pool=len(ops), n_pool_strings=len(px),
               energy=core.vdot(psi, lam, n).real, pool_grad=g.tolist(), oracle_threads=core.threads(),
               seconds=time.time() - t0)
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, f"{time.time() - t0:.0f}s", flush=True)


def main_pqe(name):
    """PQE residuals (Sec. 3.3) of a workload's ansatz at its amplitudes."""
    from oracle import pqe
    base = name[:-len("_pqe")]
    t0 = time.time()
    w, n, occ, (hx, hz, hc, goff), (ax, az, ac, off, th, t) = system(base)
    excs = an.excitations(n, w["n_elec"])
    e, r = pqe.residuals_core(n, occ, ax, az, th, hx, hz, hc, excs)
    out = dict(workload=base, recipe=w, n_qubits=n, occ_mask=occ, n_par=len(excs), energy=e,
               residuals=r.tolist(), oracle_threads=core.threads(), seconds=time.time() - t0)
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, f"{time.time() - t0:.0f}s", flush=True)


def main_qk(name, dt=0.5, s=2, r=1):
    """QK overlap and Hamiltonian matrices (Sec. 3.7) of a workload's
    Hamiltonian from its reference."""
    from oracle import krylov
    base = name[:-len("_qk")]
    t0 = time.time()
    w, n, occ, (hx, hz, hc, goff), _ = system(base)
    S, Hm = krylov.qk_matrices(n, occ, hx, hz, hc, dt, s, r, use_core=True)
    out = dict(workload=base, recipe=w, n_qubits=n, occ_mask=occ, dt=dt, s=s, r=r,
               S_re=S.real.tolist(), S_im=S.imag.tolist(), H_re=Hm.real.tolist(), H_im=Hm.imag.tolist(),
               oracle_threads=core.threads(), seconds=time.time() - t0)
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, f"{time.time() - t0:.0f}s", flush=True)


def main(name):
    if name.endswith("_qk"):
        return main_qk(name)
    if name.endswith("_pool"):
        return main_pool(name)
    if name.endswith("_pqe"):
        return main_pqe(name)
    t0 = time.time()
    w, n, occ, (hx, hz, hc, goff), (ax, az, ac, off, th, t) = system(name)
    print(f"{name}: {len(hx)} strings, {len(goff) - 1} groups, K={len(ax)}", flush=True)
    psi = core.apply_product(core.prepare(n, occ), n, ax, az, th)
    print(f"forward done {time.time() - t0:.0f}s", flush=True)
    e_group = core.energy(psi, n, hx, hz, hc, goff)
    print(f"energy {e_group!r} {time.time() - t0:.0f}s", flush=True)
    idx = sample_indices(n, psi, w["seed"])
    out = dict(workload=name, recipe=w, n_qubits=n, occ_mask=occ, n_strings=len(hx),
               n_groups=len(goff) - 1, K=len(ax), n_par=len(off) - 1,
               energy=e_group, norm=core.vdot(psi, psi, n).real,
               sample_index=idx.tolist(), sample_re=psi[idx].real.tolist(),
               sample_im=psi[idx].imag.tolist(), oracle_threads=core.threads())
    if name != "28q":
        lam = core.sigma(psi, n, hx, hz, hc)
        out["sigma_re"] = lam[idx].real.tolist()
        out["sigma_im"] = lam[idx].imag.tolist()
        e_adj, g = core.energy_grad(n, occ, ax, az, th, hx, hz, hc)
        out["energy_adjoint"] = e_adj
        out["grad_theta"] = g.tolist()
        out["grad_t"] = an.grad_t(ac, off, g).tolist()
        print(f"gradient done {time.time() - t0:.0f}s", flush=True)
    out["seconds"] = time.time() - t0
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
