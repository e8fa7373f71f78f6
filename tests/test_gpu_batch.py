"""GPU tests of the persistent batched energy + gradient (one launch).

Parity is against the CPU oracle (C core) per instance; batch-vs-alone and
graph-vs-eager results must be bit-identical (fixed team sizes give fixed
reduction orders).
"""
import numpy as np
import pytest

import qf_inputs as qi
from oracle import core

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
E_TOL, G_TOL = 1e-10, 1e-9


@pytest.fixture(scope="module")
def qf():
    assert torch.cuda.is_available()
    import paper_2108_04413_amd as qf
    return qf


def instance(qf, n_orb, n_e, seed, t_scale=0.2):
    h, g = qi.integrals(n_orb, n_e, seed)
    H, off, _ = qf.build_paulis("hamiltonian", n_orb, n_e, h, g)
    A, aoff, _ = qf.build_paulis("uccsd", n_orb, n_e)
    t = qi.amplitudes(len(aoff) - 1, seed, t_scale)
    return dict(n=2 * n_orb, occ=(1 << n_e) - 1, H=H, off=off, A=A, aoff=aoff,
                theta=qf.ansatz_angles(A, aoff, t))


def oracle(d):
    return core.energy_grad(d["n"], d["occ"], d["A"]["x"], d["A"]["z"], d["theta"],
                            d["H"]["x"], d["H"]["z"], d["H"]["c"])


def check_vs_oracle(d, e, g):
    e_o, g_o = oracle(d)
    assert e == pytest.approx(e_o, abs=E_TOL)
    assert np.max(np.abs(g - g_o)) < G_TOL


def test_batch_uneven_sizes_match_oracle(qf):
    specs = [(2, 2, 11), (3, 3, 12), (4, 4, 13), (5, 5, 14), (6, 6, 15), (4, 3, 16), (7, 7, 17)]
    insts = [instance(qf, *s) for s in specs]
    B = qf.Batch(insts)
    E, grads = B.run([d["theta"] for d in insts], use_graph=False)
    for d, e, g in zip(insts, E, grads):
        check_vs_oracle(d, e, g)


@pytest.mark.parametrize("team", [[1, 1], [2, 4], [4, 16], [16, 64]])
def test_batch_teams_match_oracle(qf, team):
    """Teams split each segment's sub-cubes (forward 2^12, reverse 2^11), so a
    team is clamped to 2^(n - 11) members (14 qubits: 8, 16 qubits: 32);
    members beyond 2^(n - 12) sit out the forward segments."""
    insts = [instance(qf, 7, 7, 21), instance(qf, 8, 8, 22)]  # 14 and 16 qubits
    B = qf.Batch(insts, team=team)
    info = B.info()
    assert info["team"] == [min(team[0], 8), min(team[1], 32)]
    E, grads = B.run([d["theta"] for d in insts], use_graph=False)
    for d, e, g in zip(insts, E, grads):
        check_vs_oracle(d, e, g)


def test_batch_shared_teams(qf):
    """team < 0 splits the grid by work: a lone instance takes every sub-cube
    it can use; in a mix the large instance gets the larger share."""
    big, small = instance(qf, 8, 8, 61), instance(qf, 6, 6, 62)  # 16 and 12 qubits
    alone = qf.Batch([big], team=[-1])
    assert alone.info()["team"] == [16]  # at most 2^(16-12): one forward sub-cube each
    mixed = qf.Batch([big, small], team=[-1, -1])
    wb, ws = mixed.info()["team"]
    assert wb == 16 and ws == 1
    E, grads = mixed.run([big["theta"], small["theta"]], use_graph=False)
    for d, e, g in zip((big, small), E, grads):
        check_vs_oracle(d, e, g)
    Ea, ga = alone.run([big["theta"]], use_graph=False)
    assert Ea[0] == E[0] and np.array_equal(ga[0], grads[0])


def test_batch_18q_instance_matches_oracle(qf):
    d = instance(qf, 9, 9, 2042)
    B = qf.Batch([d])
    E, grads = B.run([d["theta"]])
    check_vs_oracle(d, E[0], grads[0])


def test_batch_alone_equals_mixed_bitwise(qf):
    a = instance(qf, 6, 6, 31)
    b = instance(qf, 8, 8, 32)
    c = instance(qf, 5, 4, 33)
    alone = qf.Batch([b], team=[4])
    Ea, ga = alone.run([b["theta"]])
    mixed = qf.Batch([a, b, c], team=[1, 4, 1])
    Em, gm = mixed.run([a["theta"], b["theta"], c["theta"]])
    assert Ea[0] == Em[1]
    assert np.array_equal(ga[0], gm[1])


def test_batch_graph_replays_match_eager(qf):
    insts = [instance(qf, 6, 6, 41), instance(qf, 7, 7, 42), instance(qf, 8, 8, 43)]
    B = qf.Batch(insts, team=[1, 2, 4])
    for rep in range(3):
        thetas = [d["theta"] * (1.0 + 0.1 * rep) for d in insts]
        Eg, gg = B.run(thetas, use_graph=True)
        x = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        assert float(x.sum()) == float(1 << 20)  # eager work between replays
        Ee, ge = B.run(thetas, use_graph=False)
        assert np.array_equal(Eg, Ee)
        for a, b in zip(gg, ge):
            assert np.array_equal(a, b)
    e_o, g_o = oracle(dict(insts[1], theta=insts[1]["theta"] * 1.2))
    assert Eg[1] == pytest.approx(e_o, abs=E_TOL)


def test_batch_barrier_timeout_reports_error_and_recovers(qf):
    d = instance(qf, 8, 8, 51)
    B = qf.Batch([d], team=[4])
    B.set_spin_limit(1)
    with pytest.raises(qf.QFError) as ei:
        B.run([d["theta"]], use_graph=False)
    assert ei.value.status == -4
    B.set_spin_limit(1 << 28)
    E, grads = B.run([d["theta"]], use_graph=False)
    check_vs_oracle(d, E[0], grads[0])


def test_batch_timeout_fails_only_its_instance(qf):
    """Instances are independent: a team that times out marks only its own
    instance failed; single-workgroup instances of the same launch (no team
    barrier) still return their oracle values."""
    ds = [instance(qf, 6, 6, 52), instance(qf, 8, 8, 53), instance(qf, 6, 6, 54)]
    B = qf.Batch(ds, team=[1, 4, 1])
    B.set_spin_limit(1)
    E, grads, st = B.run([d["theta"] for d in ds], use_graph=False, partial=True)
    print("status with a one-poll barrier limit:", st, flush=True)
    assert st[0] == 0 and st[2] == 0 and st[1] in (0, -4)
    for i in (0, 2):
        check_vs_oracle(ds[i], E[i], grads[i])
    B.set_spin_limit(1 << 28)
    E, grads = B.run([d["theta"] for d in ds], use_graph=False)
    assert B.status() == [0, 0, 0]
    for i in range(3):
        check_vs_oracle(ds[i], E[i], grads[i])


def test_batch_recipe_instances(qf):
    """A slice of the batched workload recipe (qubits 12-16 here), one launch."""
    recs = [r for r in qi.batched_instances(256) if r["n_orb"] <= 8][:6]
    insts = [instance(qf, r["n_orb"], r["n_elec"], r["seed"], r["t_scale"]) for r in recs]
    B = qf.Batch(insts)
    E, grads = B.run([d["theta"] for d in insts])
    for d, e, g in zip(insts, E, grads):
        check_vs_oracle(d, e, g)


def test_batch_full_recipe_sampled(qf):
    """The whole batched workload (256 instances of 12-22 qubits, tuned
    teams, one graph launch, as the benchmark runs it): sampled instances
    the oracle finishes quickly against the oracle, every instance against
    the single-instance plan path."""
    recs = qi.batched_instances(256)
    insts = [instance(qf, r["n_orb"], r["n_elec"], r["seed"], r["t_scale"]) for r in recs]
    B = qf.Batch(insts)
    E, grads = B.run([d["theta"] for d in insts], use_graph=True)
    B.close()
    small = [i for i, d in enumerate(insts) if d["n"] <= 14]
    for i in small[:4] + small[-2:]:
        check_vs_oracle(insts[i], E[i], grads[i])
    ws = torch.empty(2 << max(d["n"] for d in insts), dtype=torch.complex128, device="cuda")
    for i, d in enumerate(insts):
        p = qf.Plan(d["n"], d["A"], d["H"], d["off"])
        e, g = p.energy_grad(d["occ"], d["theta"], ws)
        p.close()
        assert E[i] == pytest.approx(e, abs=E_TOL)
        assert np.max(np.abs(grads[i] - g)) < G_TOL


def test_batch_run_completion_matches_run(qf):
    """Mailbox launch: every instance is published with its completion time,
    and the results are bitwise those of an ordinary launch."""
    insts = [instance(qf, 8, 8, 71), instance(qf, 5, 5, 72), instance(qf, 6, 6, 73), instance(qf, 4, 4, 74)]
    B = qf.Batch(insts, team=[4, 1, 2, 1])
    thetas = [d["theta"] for d in insts]
    E, g = B.run(thetas, use_graph=False)
    Ec, gc, t_done = B.run_completion(thetas)
    B.close()
    assert np.array_equal(E, Ec)
    assert all(np.array_equal(a, b) for a, b in zip(g, gc))
    assert np.all(np.isfinite(t_done)) and np.all(t_done > 0)
    check_vs_oracle(insts[1], Ec[1], gc[1])


def random_instance(qf, n, seed, n_h=300, n_a=60):
    """Random same-mask runs for the ansatz and a random Pauli sum with
    odd-Y (imaginary-phase) strings and a 150-string diagonal group for H,
    its groups handed over in shuffled order."""
    rng = np.random.default_rng([n, seed, 5])
    xs, zs = [], []
    while len(xs) < n_a:
        x = 0 if rng.random() < 0.2 else int(rng.integers(1, 1 << n))
        for _ in range(int(rng.integers(1, 9))):
            xs.append(x)
            zs.append(int(rng.integers(0, 1 << n)))
    ax, az = np.array(xs[:n_a], dtype=np.uint64), np.array(zs[:n_a], dtype=np.uint64)
    hx, hz, hc = qi.random_paulis(n, n_h, seed + 1)
    hx = np.concatenate([hx, np.zeros(150, np.uint64)])
    hz = np.concatenate([hz, rng.integers(0, 1 << n, 150).astype(np.uint64)])
    hc = np.concatenate([hc, rng.normal(size=150)])
    order = np.lexsort((hz, hx))
    hx, hz, hc = hx[order], hz[order], hc[order]
    cut = [0] + [i for i in range(1, len(hx)) if hx[i] != hx[i - 1]] + [len(hx)]
    parts = [np.arange(cut[g], cut[g + 1]) for g in rng.permutation(len(cut) - 1)]
    idx = np.concatenate(parts)
    hx, hz, hc = hx[idx], hz[idx], hc[idx]
    off = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    th = qi.random_angles(n_a, seed + 2, 1.0)
    return dict(n=n, occ=(1 << (n // 2)) - 1, A=qf.terms_array(ax, az, np.ones(n_a)), theta=th,
                H=qf.terms_array(hx, hz, hc), off=off, raw=(ax, az, hx, hz, hc))


def test_batch_random_paulis_match_oracle(qf):
    """General terms through the batched kernel: the class-tiled sigma (12
    and 13 qubits: 2 and 4 tiles, imaginary phases, groups out of order)
    beside the gather form (10 qubits), teams of 1, 2 and 4."""
    insts = [random_instance(qf, 12, 81), random_instance(qf, 10, 82), random_instance(qf, 13, 83)]
    B = qf.Batch(insts, team=[2, 1, 4])
    E, grads = B.run([d["theta"] for d in insts], use_graph=False)
    B.close()
    for d, e, g in zip(insts, E, grads):
        ax, az, hx, hz, hc = d["raw"]
        e_o, g_o = core.energy_grad(d["n"], d["occ"], ax, az, d["theta"], hx, hz, hc)
        assert e == pytest.approx(e_o, abs=E_TOL)
        assert np.max(np.abs(g - g_o)) < G_TOL
